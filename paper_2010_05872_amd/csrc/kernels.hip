// HIP kernels for gfx950 (MI355X): multilevel decomposition / recomposition
// (arXiv 2010.05872, Sec. 2 and Sec. 5) and level-wise quantization (Sec. 4.1).
//
// One decomposition level l (box m0 x m1 x m2 -> coarse c0 x c1 x c2) runs as
//   k_load_vector<DEC>  coefficient computation u - Pi_{l-1}u on N*_l, stores
//                       of the coefficients in level-centric positions
//                       (Sec. 5.1) and of the nodal values into a compact
//                       coarse box, and the load vector F = (R M)^{x3} z of
//                       the multilevel component z, all in one pass over the
//                       level box (z-march over tiles staged in LDS);
//   k_solve_contig      coarse mass-matrix solve along the contiguous axis
//                       (one wavefront scan of the Thomas recurrences);
//   k_solve_strided     solves along the strided axes, lanes across the
//                       contiguous index, the last one fused with the
//                       correction application.
// Mass apply, restriction and the solve act on different tensor axes, so the
// three load-vector stencils run first, on the fine grid, and the three
// solves afterwards on the 8x smaller coarse grid.  Recomposition uses
// k_load_vector<REC> on the stored coefficients, the same solves with the
// correction subtracted, and k_interp_add.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace mgx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give every XCD a contiguous range of logical tiles so that tiles that
// share halo rows run under the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  const int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
  return base + idx;
}

__device__ __forceinline__ int64_t lc_pos(int j, int c) {
  // level-centric position of level index j on an axis with c coarse nodes
  return (j & 1) ? (int64_t)c + (j >> 1) : (int64_t)(j >> 1);
}

template <typename T>
__device__ __forceinline__ T ld(const T *p) {
  return *p;
}

// ---------------------------------------------------------------------------
// k_load_vector: coefficients + load vector of one level
// ---------------------------------------------------------------------------
//
// Tile: coarse columns [X0,X1) x rows [Y0,Y1) x planes [Z0,Z1); the last tile
// along an axis also takes the final coarse node (c = 2^k+1).  The fine
// region needed is [2Y0-2, 2Y1] x [2X0-2, 2X1] (stencil reach 2); fine nodes
// owned (written) by the tile are [2Y0, min(2Y1,m1)) etc.  The kernel
// marches over fine planes j = 2Z0-2 .. 2Z1; plane j adds its yx-restricted
// values into the load vector of the up to three coarse planes it touches.
template <typename T, int TX, int TY, bool DEC>
__global__ void __launch_bounds__(256) k_load_vector(StencilArgs<T> a) {
  constexpr int HR = 2 * TY + 5;  // region rows incl. halo and the extension
  constexpr int W = 2 * TX + 5;   // region row pitch
  constexpr int GW = TX + 1;      // coarse columns per tile (max)
  constexpr int GH = TY + 1;      // coarse rows per tile (max)
  constexpr int NOUT = (GH * GW + 255) / 256;
  constexpr int NV = DEC ? 3 : 1;

  __shared__ T sV[NV][HR * W];
  __shared__ T sZ[HR * W];
  __shared__ T sG[HR * GW];
  __shared__ T sWxl[W], sWxr[W], sWyl[HR], sWyr[HR];
  __shared__ T sW5x[GW * 5], sW5y[GH * 5];

  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int tz = t2 / a.nty;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int Z0 = tz * a.tz, Z1 = (tz == a.nzc - 1) ? c0 : Z0 + a.tz;
  const int nX = X1 - X0, nY = Y1 - Y0;
  const int r0 = 2 * Y0 - 2, q0 = 2 * X0 - 2;  // fine row / column at local 0
  const int nr = 2 * nY + 3, nq = 2 * nX + 3;
  const int own_r0 = 2 * Y0, own_r1 = min(2 * Y1, m1);
  const int own_q0 = 2 * X0, own_q1 = min(2 * X1, m2);
  const int own_p0 = 2 * Z0, own_p1 = min(2 * Z1, m0);

  // stage per-tile weights
  for (int q = tid; q < nq; q += 256) {
    int j2 = q0 + q;
    bool in = j2 >= 0 && j2 < m2;
    sWxl[q] = in ? a.ax[2].wl[j2] : T(0);
    sWxr[q] = in ? a.ax[2].wr[j2] : T(0);
  }
  for (int r = tid; r < nr; r += 256) {
    int j1 = r0 + r;
    bool in = j1 >= 0 && j1 < m1;
    sWyl[r] = in ? a.ax[1].wl[j1] : T(0);
    sWyr[r] = in ? a.ax[1].wr[j1] : T(0);
  }
  for (int i = tid; i < nX * 5; i += 256) sW5x[i] = a.ax[2].w5[X0 * 5 + i];
  for (int i = tid; i < nY * 5; i += 256) sW5y[i] = a.ax[1].w5[Y0 * 5 + i];

  // load a fine plane of the level box into an LDS slot
  auto load_plane = [&](int j, T *dst) {
    const T *src = a.V + (int64_t)j * a.vp0;
    for (int idx = tid; idx < nr * W; idx += 256) {
      int r = idx / W, q = idx - r * W;
      int j1 = r0 + r, j2 = q0 + q;
      T v = T(0);
      if (q < nq && j1 >= 0 && j1 < m1 && j2 >= 0 && j2 < m2) v = src[(int64_t)j1 * a.vp1 + j2];
      dst[idx] = v;
    }
  };

  T acc[3][NOUT];
#pragma unroll
  for (int s = 0; s < 3; s++)
#pragma unroll
    for (int k = 0; k < NOUT; k++) acc[s][k] = T(0);

  const int jstart = 2 * Z0 - 2, jend = 2 * Z1;
  if (DEC && jstart >= 0 && jstart < m0) load_plane(jstart, sV[(jstart + 3) % 3]);

  for (int j = jstart; j <= jend; j++) {
    const bool plane_in = (j >= 0 && j < m0);
    if (DEC && j + 1 >= 0 && j + 1 < m0) load_plane(j + 1, sV[(j + 4) % 3]);
    if (plane_in) {
      __syncthreads();
      // ---- multilevel component z of plane j into sZ (+ DEC stores) ----
      const int pz = j & 1;
      const bool own_plane = (j >= own_p0 && j < own_p1);
      if (DEC) {
        const T *Vm = sV[(j + 2) % 3];  // plane j-1
        const T *V0 = sV[(j + 3) % 3];  // plane j
        const T *Vp = sV[(j + 4) % 3];  // plane j+1
        const T wzl = pz ? a.ax[0].wl[j] : T(1);
        const T wzr = pz ? a.ax[0].wr[j] : T(0);
        const T *Za = pz ? Vm : V0;
        const T *Zb = pz ? Vp : V0;
        for (int idx = tid; idx < nr * W; idx += 256) {
          int r = idx / W, q = idx - r * W;
          int j1 = r0 + r, j2 = q0 + q;
          bool in = q < nq && j1 >= 0 && j1 < m1 && j2 >= 0 && j2 < m2;
          int py = j1 & 1, px = j2 & 1;
          T z = T(0);
          if (in) {
            const T v = V0[idx];
            if (pz | py | px) {
              // 2x2x2 corner stencil with zero weights on even axes
              const T wyl = py ? sWyl[r] : T(1), wyr = py ? sWyr[r] : T(0);
              const T wxl = px ? sWxl[q] : T(1), wxr = px ? sWxr[q] : T(0);
              const int ra = (r - py) * W, rb = (r + py) * W;
              const int qa = q - px, qb = q + px;
              T sa = wyl * (wxl * Za[ra + qa] + wxr * Za[ra + qb]) +
                     wyr * (wxl * Za[rb + qa] + wxr * Za[rb + qb]);
              T sb = wyl * (wxl * Zb[ra + qa] + wxr * Zb[ra + qb]) +
                     wyr * (wxl * Zb[rb + qa] + wxr * Zb[rb + qb]);
              z = v - (wzl * sa + wzr * sb);
              if (own_plane && j1 >= own_r0 && j1 < own_r1 && j2 >= own_q0 && j2 < own_q1)
                a.umc_w[lc_pos(j, c0) * a.up0 + lc_pos(j1, c1) * a.up1 + lc_pos(j2, c2)] = z;
            } else if (own_plane && j1 >= own_r0 && j1 < own_r1 && j2 >= own_q0 && j2 < own_q1) {
              a.Vc[(int64_t)(j >> 1) * a.cp0 + (int64_t)(j1 >> 1) * a.cp1 + (j2 >> 1)] = v;
            }
          }
          sZ[idx] = z;
        }
      } else {
        for (int idx = tid; idx < nr * W; idx += 256) {
          int r = idx / W, q = idx - r * W;
          int j1 = r0 + r, j2 = q0 + q;
          bool in = q < nq && j1 >= 0 && j1 < m1 && j2 >= 0 && j2 < m2;
          T z = T(0);
          if (in && (pz | (j1 & 1) | (j2 & 1)))
            z = a.umc_r[lc_pos(j, c0) * a.up0 + lc_pos(j1, c1) * a.up1 + lc_pos(j2, c2)];
          sZ[idx] = z;
        }
      }
      __syncthreads();
      // ---- restriction along x: sG[r][X] ----
      for (int idx = tid; idx < nr * GW; idx += 256) {
        int r = idx / GW, X = idx - r * GW;
        if (X < nX) {
          const T *zr = sZ + r * W + 2 * X;
          const T *w = sW5x + X * 5;
          sG[idx] = w[0] * zr[0] + w[1] * zr[1] + w[2] * zr[2] + w[3] * zr[3] + w[4] * zr[4];
        }
      }
      __syncthreads();
      // ---- restriction along y, accumulation along z ----
      const int Jc = j >> 1;  // j even: Z = Jc-1, Jc, Jc+1; j odd: Z = Jc, Jc+1
#pragma unroll
      for (int k = 0; k < NOUT; k++) {
        int idx = tid + k * 256;
        int Y = idx / GW, X = idx - Y * GW;
        if (idx < GH * GW && Y < nY && X < nX) {
          const T *w = sW5y + Y * 5;
          const T *g = sG + (2 * Y) * GW + X;
          T gyx = w[0] * g[0] + w[1] * g[GW] + w[2] * g[2 * GW] + w[3] * g[3 * GW] + w[4] * g[4 * GW];
          if (!pz) {
            // contributes to Z = Jc-1 (offset +2), Jc (0), Jc+1 (-2)
            if (Jc - 1 >= 0) acc[0][k] += a.ax[0].w5[(Jc - 1) * 5 + 4] * gyx;
            acc[1][k] += a.ax[0].w5[Jc * 5 + 2] * gyx;
            if (Jc + 1 < c0) acc[2][k] += a.ax[0].w5[(Jc + 1) * 5 + 0] * gyx;
          } else {
            // contributes to Z = Jc (offset +1), Jc+1 (-1)
            acc[0][k] += a.ax[0].w5[Jc * 5 + 3] * gyx;
            if (Jc + 1 < c0) acc[1][k] += a.ax[0].w5[(Jc + 1) * 5 + 1] * gyx;
          }
        }
      }
    }
    // after an even plane j, coarse plane j/2 - 1 is complete
    if (!(j & 1)) {
      const int Zdone = (j >> 1) - 1;
      if (Zdone >= Z0 && Zdone < Z1) {
#pragma unroll
        for (int k = 0; k < NOUT; k++) {
          int idx = tid + k * 256;
          int Y = idx / GW, X = idx - Y * GW;
          if (idx < GH * GW && Y < nY && X < nX)
            a.F[(int64_t)Zdone * a.fp0 + (int64_t)(Y0 + Y) * a.fp1 + X0 + X] = acc[0][k];
        }
      }
#pragma unroll
      for (int k = 0; k < NOUT; k++) {
        acc[0][k] = acc[1][k];
        acc[1][k] = acc[2][k];
        acc[2][k] = T(0);
      }
    }
    if (plane_in) __syncthreads();  // sZ / sG / ring slots are rewritten next
  }
}

// ---------------------------------------------------------------------------
// k_solve_contig: Thomas solve along the contiguous axis, one line per group
// of G lanes, E nodes per lane, line length c = G*E + 1.
// The forward elimination f'_J = f_J - mult_J f'_{J-1} and the back
// substitution y_J = invd_J f'_J - qsup_J y_{J+1} are first-order affine
// recurrences; each lane composes its E maps, the group scans the composed
// maps with shuffles, and each lane then replays its E steps.
// ---------------------------------------------------------------------------
template <typename T, int E, int G>
__global__ void __launch_bounds__(256) k_solve_contig(SolveArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const int li = lane % G;
  const int64_t line = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / G) + lane / G;
  const bool active = line < a.nlines;
  const int c = G * E + 1;
  T *row = a.F + (active ? line : 0) * a.pitch;
  const int J0 = li * E;

  T f[E], mu[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    f[e] = row[J0 + e];
    mu[e] = a.mult[J0 + e];  // mult[0] = 0: the first map is constant
  }
  // forward: compose x -> -mu x + f over the lane's nodes
  T A = T(1), B = T(0);
#pragma unroll
  for (int e = 0; e < E; e++) {
    A = -mu[e] * A;
    B = -mu[e] * B + f[e];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T Ap = __shfl_up(A, off, G);
    T Bp = __shfl_up(B, off, G);
    if (li >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  T xin = __shfl_up(B, 1, G);  // state before the lane's first node
  if (li == 0) xin = T(0);
  T x = xin;
#pragma unroll
  for (int e = 0; e < E; e++) {
    x = -mu[e] * x + f[e];
    f[e] = x;  // f'
  }
  // last node c-1 on the group's last lane
  const T fl = row[c - 1];
  T ylast = a.invd[c - 1] * (fl - a.mult[c - 1] * x);
  ylast = __shfl(ylast, G - 1, G);
  // backward: x -> -qsup x + invd f' over nodes in descending order
  T iv[E], qs[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    iv[e] = a.invd[J0 + e];
    qs[e] = a.qsup[J0 + e];
  }
  A = T(1);
  B = T(0);
#pragma unroll
  for (int e = E - 1; e >= 0; e--) {
    A = -qs[e] * A;
    B = -qs[e] * B + iv[e] * f[e];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T An = __shfl_down(A, off, G);
    T Bn = __shfl_down(B, off, G);
    if (li + off < G) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  T An = __shfl_down(A, 1, G);
  T Bn = __shfl_down(B, 1, G);
  if (li == G - 1) {
    An = T(1);
    Bn = T(0);
  }
  x = An * ylast + Bn;
#pragma unroll
  for (int e = E - 1; e >= 0; e--) {
    x = -qs[e] * x + iv[e] * f[e];
    f[e] = x;
  }
  if (active) {
#pragma unroll
    for (int e = 0; e < E; e++) row[J0 + e] = f[e];
    if (li == G - 1) row[c - 1] = ylast;
  }
}

// ---------------------------------------------------------------------------
// k_solve_strided: Thomas solve along a strided axis of the coarse box.
// One thread per line, consecutive lanes on consecutive contiguous indices
// (coalesced rows).  The forward sweep writes f' in place; the backward
// sweep reads it back.  With APPLY the solution is not stored but added
// (sign +1, decomposition) or subtracted (sign -1, recomposition) to the
// nodal values: out = in + sign * y.
// ---------------------------------------------------------------------------
template <typename T, bool APPLY>
__global__ void __launch_bounds__(256) k_solve_strided(StridedArgs<T> a) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int o = blockIdx.y;
  if (x >= a.nx) return;
  T *p = a.F + (int64_t)o * a.so + x;
  const int c = a.c;
  const int64_t s = a.sj;
  T fp = p[0];
  for (int J = 1; J < c; J++) {
    fp = p[J * s] - a.mult[J] * fp;
    p[J * s] = fp;
  }
  T y = a.invd[c - 1] * fp;
  if (APPLY) {
    const int64_t ii = (int64_t)(c - 1) * a.ij + (int64_t)o * a.io + x;
    const int64_t oo = (int64_t)(c - 1) * a.oj + (int64_t)o * a.oo + x;
    a.out[oo] = a.in[ii] + a.sign * y;
  } else {
    p[(c - 1) * s] = y;
  }
  for (int J = c - 2; J >= 0; J--) {
    y = a.invd[J] * p[J * s] - a.qsup[J] * y;
    if (APPLY) {
      const int64_t ii = (int64_t)J * a.ij + (int64_t)o * a.io + x;
      const int64_t oo = (int64_t)J * a.oj + (int64_t)o * a.oo + x;
      a.out[oo] = a.in[ii] + a.sign * y;
    } else {
      p[J * s] = y;
    }
  }
}

// Correction application for one-dimensional fields (no strided solve):
// out = in + sign * F over a row of the coarse box.
template <typename T>
__global__ void __launch_bounds__(256) k_apply(StridedArgs<T> a) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.nx) return;
  a.out[x] = a.in[x] + a.sign * a.F[x];
}

// ---------------------------------------------------------------------------
// k_interp_add: recomposition step 4 — Q_l u = coefficient + Pi_{l-1} of the
// corrected nodal values (and the nodal values themselves on N_{l-1}).
// Tile as in k_load_vector; the kernel marches over coarse planes J with a
// two-slot ring of nodal planes (J, J+1) and emits fine planes 2J, 2J+1.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(256) k_interp_add(InterpArgs<T> a) {
  constexpr int NW = TX + 2;  // nodal tile pitch
  constexpr int NH = TY + 2;
  constexpr int OW = 2 * TX + 2;  // owned fine columns (max)
  __shared__ T sN[2][NH * NW];
  __shared__ T sWxl[OW], sWxr[OW], sWyl[2 * TY + 2], sWyr[2 * TY + 2];

  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int tz = t2 / a.nty;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int Z0 = tz * a.tz, Z1 = (tz == a.nzc - 1) ? c0 : Z0 + a.tz;
  const int nX = X1 - X0, nY = Y1 - Y0;
  const int ncx = min(nX + 1, c2 - X0), ncy = min(nY + 1, c1 - Y0);  // nodal tile extent
  const int fq = min(2 * X1, m2) - 2 * X0;  // owned fine columns
  const int fr = min(2 * Y1, m1) - 2 * Y0;  // owned fine rows

  for (int q = tid; q < fq; q += 256) {
    sWxl[q] = a.ax[2].wl[2 * X0 + q];
    sWxr[q] = a.ax[2].wr[2 * X0 + q];
  }
  for (int r = tid; r < fr; r += 256) {
    sWyl[r] = a.ax[1].wl[2 * Y0 + r];
    sWyr[r] = a.ax[1].wr[2 * Y0 + r];
  }
  auto load_nodal = [&](int J, T *dst) {
    const T *src = a.nodal + (int64_t)J * a.np0;
    for (int idx = tid; idx < NH * NW; idx += 256) {
      int r = idx / NW, q = idx - r * NW;
      T v = T(0);
      if (r < ncy && q < ncx) v = src[(int64_t)(Y0 + r) * a.np1 + X0 + q];
      dst[idx] = v;
    }
  };
  load_nodal(Z0, sN[Z0 & 1]);
  for (int J = Z0; J < Z1; J++) {
    if (J + 1 < c0) load_nodal(J + 1, sN[(J + 1) & 1]);
    __syncthreads();
    const T *N0 = sN[J & 1];
    const T *N1 = sN[(J + 1) & 1];
    for (int pz = 0; pz < 2; pz++) {
      const int j = 2 * J + pz;
      if (j >= m0) break;
      const T wzl = pz ? a.ax[0].wl[j] : T(1);
      const T wzr = pz ? a.ax[0].wr[j] : T(0);
      const T *Na = N0;
      const T *Nb = pz ? N1 : N0;
      for (int idx = tid; idx < fr * OW; idx += 256) {
        int rr = idx / OW, qq = idx - rr * OW;
        if (qq >= fq) continue;
        int j1 = 2 * Y0 + rr, j2 = 2 * X0 + qq;
        int py = j1 & 1, px = j2 & 1;
        int ra = (rr >> 1) * NW, rb = ((rr >> 1) + py) * NW;
        int qa = qq >> 1, qb = (qq >> 1) + px;
        T outv;
        if (pz | py | px) {
          const T wyl = py ? sWyl[rr] : T(1), wyr = py ? sWyr[rr] : T(0);
          const T wxl = px ? sWxl[qq] : T(1), wxr = px ? sWxr[qq] : T(0);
          T sa = wyl * (wxl * Na[ra + qa] + wxr * Na[ra + qb]) + wyr * (wxl * Na[rb + qa] + wxr * Na[rb + qb]);
          T sb = wyl * (wxl * Nb[ra + qa] + wxr * Nb[ra + qb]) + wyr * (wxl * Nb[rb + qa] + wxr * Nb[rb + qb]);
          T cf = a.umc[lc_pos(j, c0) * a.up0 + lc_pos(j1, c1) * a.up1 + lc_pos(j2, c2)];
          outv = cf + (wzl * sa + wzr * sb);
        } else {
          outv = Na[ra + qa];
        }
        a.out[(int64_t)j * a.op0 + (int64_t)j1 * a.op1 + j2] = outv;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Quantization (Sec. 4.1): label = rint(c / q_l) in FP64; level of a
// position in the level-centric layout = the smallest l whose box holds it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int axis_level(int p, const QuantArgs &a, int k) {
  // sizes[k][i] = box size of level first+i along axis k (increasing)
  int lev = a.first;
  for (int i = 0; i < a.nlev - 1; i++)
    if (p >= a.sizes[k][i]) lev = a.first + i + 1;
  return lev;
}

template <typename T, bool STATS>
__global__ void __launch_bounds__(256) k_quantize(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                                  QuantArgs a) {
  __shared__ int s_max[kMaxLevelsK];
  __shared__ unsigned long long s_ovf, s_nan;
  if (STATS) {
    if (threadIdx.x < kMaxLevelsK) s_max[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      s_ovf = 0;
      s_nan = 0;
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  unsigned long long my_ovf = 0, my_nan = 0;
  for (int64_t row = blockIdx.x; row < a.nrows; row += gridDim.x) {
    const int z = (int)(row / a.n1), y = (int)(row - (int64_t)z * a.n1);
    const int rl = max(axis_level(z, a, 0), axis_level(y, a, 1));
    const T *src = umc + row * a.n2;
    int32_t *dst = labels + row * a.n2;
    for (int x0 = 0; x0 < a.n2; x0 += 256) {
      const int x = x0 + threadIdx.x;
      const bool in = x < a.n2;
      int lev = a.first;
      int absl = 0;
      if (in) {
        lev = max(rl, axis_level(x, a, 2));
        const double qv = a.q[lev - a.first];
        const double v = (double)src[x] / qv;
        int32_t lab;
        if (!(fabs(v) < 2147483647.0)) {
          lab = INT32_MIN;
          if (isnan(v) || isinf(v)) my_nan++;
          else my_ovf++;
        } else {
          lab = (int32_t)rint(v);
          absl = lab < 0 ? -lab : lab;
        }
        dst[x] = lab;
      }
      if (STATS) {
        // per-level wave reduction; usually one level per wave
        unsigned long long todo = __ballot(in);
        while (todo) {
          const int leader = __ffsll((long long)todo) - 1;
          const int L0 = __shfl(lev, leader);
          const bool mine = in && lev == L0;
          int v = mine ? absl : 0;
          for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
          if (lane == leader) atomicMax(&s_max[L0 - a.first], v);
          todo &= ~__ballot(mine);
        }
      }
    }
  }
  if (STATS) {
    for (int off = 32; off > 0; off >>= 1) {
      my_ovf += __shfl_xor(my_ovf, off);
      my_nan += __shfl_xor(my_nan, off);
    }
    if (lane == 0) {
      atomicAdd(&s_ovf, my_ovf);
      atomicAdd(&s_nan, my_nan);
    }
    __syncthreads();
    if (threadIdx.x < a.nlev) atomicMax(&a.stats_max[threadIdx.x], s_max[threadIdx.x]);
    if (threadIdx.x == 0) {
      atomicAdd(a.stats_ovf, s_ovf);
      atomicAdd(a.stats_nan, s_nan);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_dequantize(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                    QuantArgs a) {
  for (int64_t row = blockIdx.x; row < a.nrows; row += gridDim.x) {
    const int z = (int)(row / a.n1), y = (int)(row - (int64_t)z * a.n1);
    const int rl = max(axis_level(z, a, 0), axis_level(y, a, 1));
    const int32_t *src = labels + row * a.n2;
    T *dst = umc + row * a.n2;
    for (int x = threadIdx.x; x < a.n2; x += 256) {
      const int lev = max(rl, axis_level(x, a, 2));
      dst[x] = (T)((double)src[x] * a.q[lev - a.first]);
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T>
struct Tiles;
template <>
struct Tiles<float> {
  static constexpr int TX = 32, TY = 16;
};
template <>
struct Tiles<double> {
  static constexpr int TX = 16, TY = 16;
};

// Tiles of TX x TY coarse columns/rows (the last tile takes the extra node of
// c = 2^k + 1) and z-chunks of tz coarse planes.  Returns false when an axis
// length does not satisfy the tiling assumption (c - 1 a multiple of the
// tile, or smaller than it), so that no kernel is launched on a bad shape.
static bool tile_grid(int c0, int c1, int c2, int TX, int TY, int *ntx, int *nty, int *nzc, int *tz) {
  if (c0 < 1 || c1 < 1 || c2 < 1) return false;
  if ((c2 - 1) >= TX && (c2 - 1) % TX != 0) return false;
  if ((c1 - 1) >= TY && (c1 - 1) % TY != 0) return false;
  *ntx = (c2 - 1) / TX > 0 ? (c2 - 1) / TX : 1;
  *nty = (c1 - 1) / TY > 0 ? (c1 - 1) / TY : 1;
  const int per = *ntx * *nty;
  int want = (2048 + per - 1) / per;
  int maxz = c0 / 4 > 0 ? c0 / 4 : 1;
  if (want > maxz) want = maxz;
  if (want < 1) want = 1;
  *nzc = want;
  *tz = c0 / want;
  return true;
}

template <typename T>
hipError_t launch_load_vector(StencilArgs<T> a, bool dec, hipStream_t st) {
  constexpr int TX = Tiles<T>::TX, TY = Tiles<T>::TY;
  if (!tile_grid(a.ax[0].c, a.ax[1].c, a.ax[2].c, TX, TY, &a.ntx, &a.nty, &a.nzc, &a.tz))
    return hipErrorInvalidValue;
  dim3 grid(a.ntx * a.nty * a.nzc);
  if (dec)
    hipLaunchKernelGGL((k_load_vector<T, TX, TY, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_load_vector<T, TX, TY, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_add(InterpArgs<T> a, hipStream_t st) {
  constexpr int TX = Tiles<T>::TX, TY = Tiles<T>::TY;
  if (!tile_grid(a.ax[0].c, a.ax[1].c, a.ax[2].c, TX, TY, &a.ntx, &a.nty, &a.nzc, &a.tz))
    return hipErrorInvalidValue;
  dim3 grid(a.ntx * a.nty * a.nzc);
  hipLaunchKernelGGL((k_interp_add<T, TX, TY>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T, int E, int G>
static void launch_contig_eg(SolveArgs<T> a, hipStream_t st) {
  const int64_t lines_per_block = 4 * (64 / G);
  dim3 grid((unsigned)((a.nlines + lines_per_block - 1) / lines_per_block));
  hipLaunchKernelGGL((k_solve_contig<T, E, G>), grid, dim3(256), 0, st, a);
}

template <typename T>
hipError_t launch_solve_contig(SolveArgs<T> a, hipStream_t st) {
  switch (a.c) {
    case 3: launch_contig_eg<T, 1, 2>(a, st); break;
    case 5: launch_contig_eg<T, 1, 4>(a, st); break;
    case 9: launch_contig_eg<T, 1, 8>(a, st); break;
    case 17: launch_contig_eg<T, 1, 16>(a, st); break;
    case 33: launch_contig_eg<T, 1, 32>(a, st); break;
    case 65: launch_contig_eg<T, 1, 64>(a, st); break;
    case 129: launch_contig_eg<T, 2, 64>(a, st); break;
    case 257: launch_contig_eg<T, 4, 64>(a, st); break;
    case 513: launch_contig_eg<T, 8, 64>(a, st); break;
    case 1025: launch_contig_eg<T, 16, 64>(a, st); break;
    case 2049: launch_contig_eg<T, 32, 64>(a, st); break;
    case 4097: launch_contig_eg<T, 64, 64>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve_strided(StridedArgs<T> a, bool apply, hipStream_t st) {
  dim3 grid((unsigned)((a.nx + 255) / 256), (unsigned)a.nouter);
  if (apply)
    hipLaunchKernelGGL((k_solve_strided<T, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve_strided<T, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(StridedArgs<T> a, hipStream_t st) {
  dim3 grid((unsigned)((a.nx + 255) / 256));
  hipLaunchKernelGGL((k_apply<T>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

static unsigned quant_grid(int64_t nrows) {
  int64_t g = nrows < 8192 ? nrows : 8192;
  return (unsigned)(g > 0 ? g : 1);
}

template <typename T>
hipError_t launch_quantize(const T *umc, int32_t *labels, QuantArgs a, bool stats, hipStream_t st) {
  dim3 grid(quant_grid(a.nrows));
  if (stats)
    hipLaunchKernelGGL((k_quantize<T, true>), grid, dim3(256), 0, st, umc, labels, a);
  else
    hipLaunchKernelGGL((k_quantize<T, false>), grid, dim3(256), 0, st, umc, labels, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dequantize(const int32_t *labels, T *umc, QuantArgs a, hipStream_t st) {
  dim3 grid(quant_grid(a.nrows));
  hipLaunchKernelGGL((k_dequantize<T>), grid, dim3(256), 0, st, labels, umc, a);
  return hipGetLastError();
}

#define MGX_INSTANTIATE(T)                                                                    \
  template hipError_t launch_load_vector<T>(StencilArgs<T>, bool, hipStream_t);               \
  template hipError_t launch_interp_add<T>(InterpArgs<T>, hipStream_t);                       \
  template hipError_t launch_solve_contig<T>(SolveArgs<T>, hipStream_t);                      \
  template hipError_t launch_solve_strided<T>(StridedArgs<T>, bool, hipStream_t);             \
  template hipError_t launch_apply<T>(StridedArgs<T>, hipStream_t);                           \
  template hipError_t launch_quantize<T>(const T *, int32_t *, QuantArgs, bool, hipStream_t); \
  template hipError_t launch_dequantize<T>(const int32_t *, T *, QuantArgs, hipStream_t);

MGX_INSTANTIATE(float)
MGX_INSTANTIATE(double)

}  // namespace mgx
