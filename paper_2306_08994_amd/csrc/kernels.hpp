// kernels.hpp -- gfx950 device kernels of the multifrontal factor and solve.
//
// Storage: every front f owns an m x m row-major FP64 block at store + desc[f].store.  After the
// front is factored it holds, in place,
//   L (pivots on the diagonal)  at rows p..m-1 of columns p < k,
//   U (unit diagonal, implicit) at columns p+1..m-1 of rows p < k,
//   the Schur complement (contribution block, CB) in rows and columns k..m-1,
// i.e. the result of the division / multiplication / subtraction tasks of Table 2 applied to
// the assembled front.  A parent reads its children's CBs straight from their storage.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "plan.hpp"

namespace mf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kStatusWords = 4;   // [0] error flag, [1] front, [2] pivot

__device__ inline void record_bad_pivot(int *st, int f, int p) {
  if (atomicCAS(st, 0, 1) == 0) {
    st[1] = f;
    st[2] = p;
  }
}

__device__ inline bool good_pivot(double v) { return v != 0.0 && __builtin_isfinite(v); }

__global__ void k_clear_status(int *st) {
  if (threadIdx.x < kStatusWords) st[threadIdx.x] = 0;
}

// Value of entry (i, j) of the assembled front: the element matrix for a leaf, otherwise the sum
// of the children's CB entries that map there (left child first, then right: extend-add).
__device__ inline double gather_entry(const FrontDesc &d, const FrontDesc &a, const FrontDesc &b,
                                      const double *__restrict__ ca, const double *__restrict__ cb,
                                      const double *__restrict__ Ke, int npe, int li, int lj,
                                      int ri, int rj) {
  if (d.elem >= 0) return Ke[li * npe + lj];
  double v = 0.0;
  if ((li | lj) >= 0) v += ca[(int64_t)li * a.m + lj];
  if ((ri | rj) >= 0) v += cb[(int64_t)ri * b.m + rj];
  return v;
}

struct GatherCtx {
  FrontDesc a, b;
  const double *ca, *cb, *Ke;
};

__device__ inline GatherCtx gather_ctx(const FrontDesc *__restrict__ fd, const FrontDesc &d,
                                       const double *__restrict__ store,
                                       const double *__restrict__ K, int npe) {
  GatherCtx g;
  if (d.elem >= 0) {
    g.a = d;
    g.b = d;
    g.ca = g.cb = nullptr;
    g.Ke = K + (int64_t)d.elem * npe * npe;
  } else {
    g.a = fd[d.left];
    g.b = fd[d.right];
    g.ca = store + g.a.store + (int64_t)g.a.k * g.a.m + g.a.k;
    g.cb = store + g.b.store + (int64_t)g.b.k * g.b.m + g.b.k;
    g.Ke = nullptr;
  }
  return g;
}

// ---------------------------------------------------------------------------------------------
// Fused small-front kernel: assemble, partially eliminate and store one front per workgroup with
// the whole front resident in LDS.  Grid-stride over the class's front list (persistent launch).
// For each pivot p: the division tasks scale row p by the pivot, then every (i, j) > p receives
// its multiplication + subtraction F[i][j] -= F[i][p] * U[p][j].
// ---------------------------------------------------------------------------------------------
template <int NT>
__global__ void __launch_bounds__(NT)
k_factor_small(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list, int nlist,
               double *__restrict__ store, const int32_t *__restrict__ inv_l,
               const int32_t *__restrict__ inv_r, const double *__restrict__ K, int npe,
               int *__restrict__ status) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int f = list[li];
    const FrontDesc d = fd[f];
    const int m = d.m, k = d.k, ld = m | 1;
    const int32_t *il = inv_l + d.idx;
    const int32_t *ir = inv_r + d.idx;
    const GatherCtx g = gather_ctx(fd, d, store, K, npe);
    for (int t = tid; t < m * m; t += NT) {
      const int i = t / m, j = t - (t / m) * m;
      sh[i * ld + j] = gather_entry(d, g.a, g.b, g.ca, g.cb, g.Ke, npe, il[i], il[j], ir[i], ir[j]);
    }
    __syncthreads();
    for (int p = 0; p < k; ++p) {
      const double piv = sh[p * ld + p];
      if (!good_pivot(piv)) {
        if (tid == 0) record_bad_pivot(status, f, p);
        break;
      }
      for (int j = p + 1 + tid; j < m; j += NT) sh[p * ld + j] = sh[p * ld + j] / piv;
      __syncthreads();
      const int r = m - p - 1;
      for (int t = tid; t < r * r; t += NT) {
        const int i = p + 1 + t / r, j = p + 1 + (t - (t / r) * r);
        sh[i * ld + j] -= sh[i * ld + p] * sh[p * ld + j];
      }
      __syncthreads();
    }
    double *out = store + d.store;
    for (int t = tid; t < m * m; t += NT) {
      const int i = t / m, j = t - (t / m) * m;
      out[t] = sh[i * ld + j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Tiled (HBM-resident) path for fronts wider than the LDS limit.
// ---------------------------------------------------------------------------------------------

// Extend-add: builds the assembled front in its storage.  grid = (row strips of 4, fronts).
__global__ void __launch_bounds__(256)
k_assemble(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list,
           double *__restrict__ store, const int32_t *__restrict__ inv_l,
           const int32_t *__restrict__ inv_r, const double *__restrict__ K, int npe) {
  const int f = list[blockIdx.y];
  const FrontDesc d = fd[f];
  const int m = d.m;
  const int i0 = blockIdx.x * 4;
  if (i0 >= m) return;
  const int32_t *il = inv_l + d.idx;
  const int32_t *ir = inv_r + d.idx;
  const GatherCtx g = gather_ctx(fd, d, store, K, npe);
  double *F = store + d.store;
  const int i1 = min(i0 + 4, m);
  for (int i = i0; i < i1; ++i) {
    const int li = il[i], ri = ir[i];
    for (int j = threadIdx.x; j < m; j += 256)
      F[(int64_t)i * m + j] = gather_entry(d, g.a, g.b, g.ca, g.cb, g.Ke, npe, li, il[j], ri, ir[j]);
  }
}

// Panel step, part 1: LU of the pb x pb diagonal block at (p0, p0), one workgroup per front.
template <int NB>
__global__ void __launch_bounds__(256)
k_panel_diag(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ fronts,
             const int32_t *__restrict__ p0s, double *__restrict__ store, int *__restrict__ status) {
  __shared__ double D[NB][NB + 1];
  __shared__ int bad;
  const int f = fronts[blockIdx.x];
  const int p0 = p0s[blockIdx.x];
  const FrontDesc d = fd[f];
  const int m = d.m, pb = min(NB, d.k - p0);
  double *F = store + d.store + (int64_t)p0 * m + p0;
  const int tid = threadIdx.x;
  for (int t = tid; t < pb * pb; t += 256) D[t / pb][t % pb] = F[(int64_t)(t / pb) * m + t % pb];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int p = 0; p < pb; ++p) {
    const double piv = D[p][p];
    if (!good_pivot(piv)) {
      if (tid == 0) record_bad_pivot(status, f, p0 + p);
      break;
    }
    for (int j = p + 1 + tid; j < pb; j += 256) D[p][j] = D[p][j] / piv;
    __syncthreads();
    const int r = pb - p - 1;
    for (int t = tid; t < r * r; t += 256) {
      const int i = p + 1 + t / r, j = p + 1 + t % r;
      D[i][j] -= D[i][p] * D[p][j];
    }
    __syncthreads();
  }
  for (int t = tid; t < pb * pb; t += 256) F[(int64_t)(t / pb) * m + t % pb] = D[t / pb][t % pb];
}

// Panel step, part 2: the two triangular solves against the factored diagonal block.
//   U12 = L11^{-1} A12 column by column (rows p0..pe-1, columns pe..m-1),
//   L21 = A21 U11^{-1} row by row       (rows pe..m-1, columns p0..pe-1).
// grid = (item chunks of 256, fronts); item t < m-pe is a column, otherwise a row.
template <int NB>
__global__ void __launch_bounds__(256)
k_panel_trsm(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ fronts,
             const int32_t *__restrict__ p0s, double *__restrict__ store) {
  __shared__ double D[NB][NB + 1];
  const int f = fronts[blockIdx.y];
  const int p0 = p0s[blockIdx.y];
  const FrontDesc d = fd[f];
  const int m = d.m, pb = min(NB, d.k - p0), pe = p0 + pb;
  const int rest = m - pe;
  const int item = blockIdx.x * 256 + threadIdx.x;
  if ((int)(blockIdx.x * 256) >= 2 * rest) return;   // whole block idle (uniform)
  double *F = store + d.store;
  for (int t = threadIdx.x; t < pb * pb; t += 256)
    D[t / pb][t % pb] = F[(int64_t)(p0 + t / pb) * m + p0 + t % pb];
  __syncthreads();
  if (item >= 2 * rest) return;
  double v[NB];
  if (item < rest) {
    const int j = pe + item;
#pragma unroll
    for (int q = 0; q < NB; ++q) v[q] = q < pb ? F[(int64_t)(p0 + q) * m + j] : 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q < pb) {
        double s = v[q];
#pragma unroll
        for (int r = 0; r < q; ++r) s -= D[q][r] * v[r];
        v[q] = s / D[q][q];
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < pb) F[(int64_t)(p0 + q) * m + j] = v[q];
  } else {
    const int i = pe + (item - rest);
    double *row = F + (int64_t)i * m + p0;
#pragma unroll
    for (int q = 0; q < NB; ++q) v[q] = q < pb ? row[q] : 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q < pb) {
        double s = v[q];
#pragma unroll
        for (int r = 0; r < q; ++r) s -= v[r] * D[r][q];
        v[q] = s;
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < pb) row[q] = v[q];
  }
}

// Batched GEMM update C -= A B over a task list, 64 x 64 output tile per workgroup of 4 waves,
// each wave a 32 x 32 quadrant of 2 x 2 MFMA blocks of 16 x 16.
//   PREC 0: FP64 operands, v_mfma_f64_16x16x4f64, FP64 accumulate;
//   PREC 1: operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32 accumulate;
//   PREC 2: operands rounded to BF16, v_mfma_f32_16x16x32_bf16, FP32 accumulate.
// The accumulated product is subtracted from the FP64 C in every case.
// MFMA 16x16 operand layout (lane l): A row l%16, k-group l/16; B column l%16, k-group l/16;
// result: column l%16, rows as noted at the write-back (checked on gfx950 hardware).
template <int PREC>
struct GemmCfg;
template <>
struct GemmCfg<0> { typedef double T; static constexpr int KT = 16; };
template <>
struct GemmCfg<1> { typedef float T; static constexpr int KT = 16; };
template <>
struct GemmCfg<2> { typedef __bf16 T; static constexpr int KT = 32; };

template <int PREC>
__global__ void __launch_bounds__(256)
k_gemm_update(const FrontDesc *__restrict__ fd, const GemmTask *__restrict__ tasks,
              double *__restrict__ store) {
  typedef typename GemmCfg<PREC>::T T;
  constexpr int KT = GemmCfg<PREC>::KT;
  constexpr int APAD = (PREC == 2) ? 8 : 1;
  __shared__ T As[64][KT + APAD];
  __shared__ T Bs[64][KT + APAD];    // stored transposed: Bs[col][k]
  const GemmTask tk = tasks[blockIdx.x];
  const FrontDesc d = fd[tk.front];
  const int64_t ld = d.m;
  double *F = store + d.store;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename std::conditional<PREC == 0, v4d, v4f>::type Acc;
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;
  const int i0 = tk.i0, j0 = tk.j0;
  for (int q = tk.q0; q < tk.q1; q += KT) {
    // stage A[i0:i0+64, q:q+KT] and B[q:q+KT, j0:j0+64] (zero outside the task)
    for (int t = tid; t < 64 * KT; t += 256) {
      const int r = t / KT, c = t % KT;
      const int gi = i0 + r, gq = q + c;
      double va = (gi < tk.i1 && gq < tk.q1) ? F[gi * ld + gq] : 0.0;
      As[r][c] = (T)va;
    }
    for (int t = tid; t < 64 * KT; t += 256) {
      const int c = t % 64, r = t / 64;
      const int gq = q + r, gj = j0 + c;
      double vb = (gq < tk.q1 && gj < tk.j1) ? F[gq * ld + gj] : 0.0;
      Bs[c][r] = (T)vb;
    }
    __syncthreads();
    if constexpr (PREC == 2) {
      v8bf av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 8; ++e) av[a][e] = As[32 * wr + 16 * a + li][8 * lk + e];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[b][e] = Bs[32 * wc + 16 * b + li][8 * lk + e];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < KT / 4; ++s) {
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[32 * wr + 16 * a + li][4 * s + lk];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[32 * wc + 16 * b + li][4 * s + lk];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            if constexpr (PREC == 0)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 interleaves its result rows (lane l, register r -> row 4r + l/16); the
        // f32 16x16x4 and bf16 16x16x32 forms place them contiguously (row 4(l/16) + r)
        const int gi = i0 + 32 * wr + 16 * a + (PREC == 0 ? 4 * r + lk : 4 * lk + r);
        const int gj = j0 + 32 * wc + 16 * b + li;
        if (gi < tk.i1 && gj < tk.j1) F[gi * ld + gj] -= (double)acc[a][b][r];
      }
}

// ---------------------------------------------------------------------------------------------
// Solves.  One workgroup per front (grid-stride), right-hand sides processed in chunks of `nc`
// columns held in LDS as W[m][nc].
// down sweep (classes 0..H):  TRANS=0: L y = b   (y_p = w_p / L_pp, w_i -= L_ip y_p, i > p)
//                             TRANS=1: U^T z = g (z_p = w_p,        w_j -= U_pj z_p, j > p)
//   The front's RHS block starts as b on its pivots plus its children's contribution blocks;
//   its own contribution block (rows k..m-1) is written to ycb for the parent.
// up sweep (classes H..0):    TRANS=0: U x = y   (x_p = w_p - sum_{j>p} U_pj x_j)
//                             TRANS=1: L^T l = z (l_p = (w_p - sum_{i>p} L_ip l_i) / L_pp)
// ---------------------------------------------------------------------------------------------
template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_down(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list, int nlist,
             const double *__restrict__ store, const int32_t *__restrict__ front_idx,
             const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
             const double *b, double *x, double *__restrict__ ycb, int nrhs, int nc) {
  extern __shared__ double W[];
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int f = list[li];
    const FrontDesc d = fd[f];
    const int m = d.m, k = d.k;
    const int32_t *idx = front_idx + d.idx;
    const int32_t *il = inv_l + d.idx;
    const int32_t *ir = inv_r + d.idx;
    const double *F = store + d.store;
    int64_t rowa = 0, rowb = 0;
    if (d.elem < 0) {
      rowa = fd[d.left].cbrow;
      rowb = fd[d.right].cbrow;
    }
    for (int r0 = 0; r0 < nrhs; r0 += nc) {
      const int nr = min(nc, nrhs - r0);
      for (int t = tid; t < m * nr; t += 256) {
        const int i = t / nr, r = t - (t / nr) * nr;
        double v = i < k ? b[(int64_t)idx[i] * nrhs + r0 + r] : 0.0;
        if (d.elem < 0) {
          const int a = il[i], c = ir[i];
          if (a >= 0) v += ycb[(rowa + a) * nrhs + r0 + r];
          if (c >= 0) v += ycb[(rowb + c) * nrhs + r0 + r];
        }
        W[i * nr + r] = v;
      }
      __syncthreads();
      for (int p = 0; p < k; ++p) {
        const double diag = TRANS ? 1.0 : F[(int64_t)p * m + p];
        const int cnt = (m - p - 1) * nr;
        if (tid < nr) {
          const double yp = TRANS ? W[p * nr + tid] : W[p * nr + tid] / diag;
          x[(int64_t)idx[p] * nrhs + r0 + tid] = yp;
        }
        for (int t = tid; t < cnt; t += 256) {
          const int i = p + 1 + t / nr, r = t - (t / nr) * nr;
          const double yp = TRANS ? W[p * nr + r] : W[p * nr + r] / diag;
          const double c = TRANS ? F[(int64_t)p * m + i] : F[(int64_t)i * m + p];
          W[i * nr + r] -= c * yp;
        }
        __syncthreads();
      }
      for (int t = tid; t < (m - k) * nr; t += 256) {
        const int i = k + t / nr, r = t - (t / nr) * nr;
        ycb[(d.cbrow + i - k) * nrhs + r0 + r] = W[i * nr + r];
      }
      __syncthreads();
    }
  }
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_up(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list, int nlist,
           const double *__restrict__ store, const int32_t *__restrict__ front_idx,
           double *x, int nrhs, int nc) {
  extern __shared__ double W[];
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int f = list[li];
    const FrontDesc d = fd[f];
    const int m = d.m, k = d.k;
    const int32_t *idx = front_idx + d.idx;
    const double *F = store + d.store;
    for (int r0 = 0; r0 < nrhs; r0 += nc) {
      const int nr = min(nc, nrhs - r0);
      for (int t = tid; t < m * nr; t += 256) {
        const int i = t / nr, r = t - (t / nr) * nr;
        W[i * nr + r] = x[(int64_t)idx[i] * nrhs + r0 + r];
      }
      __syncthreads();
      // contribution of the already-final CB unknowns to the pivot rows
      for (int t = tid; t < k * nr; t += 256) {
        const int p = t / nr, r = t - (t / nr) * nr;
        double s = W[p * nr + r];
        for (int j = k; j < m; ++j) {
          const double c = TRANS ? F[(int64_t)j * m + p] : F[(int64_t)p * m + j];
          s -= c * W[j * nr + r];
        }
        W[p * nr + r] = s;
      }
      __syncthreads();
      for (int p = k - 1; p >= 0; --p) {
        const double diag = TRANS ? F[(int64_t)p * m + p] : 1.0;
        if (tid < nr) {
          const double xp = TRANS ? W[p * nr + tid] / diag : W[p * nr + tid];
          x[(int64_t)idx[p] * nrhs + r0 + tid] = xp;
        }
        for (int t = tid; t < p * nr; t += 256) {
          const int q = t / nr, r = t - (t / nr) * nr;
          const double xp = TRANS ? W[p * nr + r] / diag : W[p * nr + r];
          const double c = TRANS ? F[(int64_t)p * m + q] : F[(int64_t)q * m + p];
          W[q * nr + r] -= c * xp;
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Element-by-element operators (FP64).
// ---------------------------------------------------------------------------------------------

// r[v] = b[v] - sum over the (element, local node) pairs of v of K_e[a][:] x[conn_e]; the pairs
// of each node are listed in ascending element order, so the result is deterministic.
__global__ void __launch_bounds__(256)
k_residual(const int64_t *__restrict__ nptr, const int32_t *__restrict__ nelem,
           const int32_t *__restrict__ conn, const double *__restrict__ K, int npe, int64_t n,
           const double *__restrict__ x, const double *__restrict__ b, double *__restrict__ r,
           int nrhs) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * nrhs) return;
  const int64_t v = t / nrhs;
  const int c = (int)(t - v * nrhs);
  double s = 0.0;
  for (int64_t q = nptr[v]; q < nptr[v + 1]; ++q) {
    const int32_t ea = nelem[q];
    const int32_t e = ea / npe, a = ea - (ea / npe) * npe;
    const double *Ke = K + ((int64_t)e * npe + a) * npe;
    const int32_t *ce = conn + (int64_t)e * npe;
    for (int bb = 0; bb < npe; ++bb) s += Ke[bb] * x[(int64_t)ce[bb] * nrhs + c];
  }
  r[t] = b[t] - s;
}

// Per-column partial sums of squares: part[block][c] over rows block*rows_per .. .
__global__ void __launch_bounds__(256)
k_colsq_partial(const double *__restrict__ a, int64_t n, int nrhs, int64_t rows_per,
                double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(n, r0 + rows_per);
  for (int c = 0; c < nrhs; ++c) {
    double s = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
      const double v = a[i * nrhs + c];
      s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nrhs + c] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
k_axpy(double *__restrict__ x, const double *__restrict__ dx, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < len) x[t] += dx[t];
}

// gK[e][a][b] = -sum_r lam[conn_e[a]][r] u[conn_e[b]][r]
__global__ void __launch_bounds__(256)
k_elem_grad(const int32_t *__restrict__ conn, int64_t ne, int npe, const double *__restrict__ lam,
            const double *__restrict__ u, int nrhs, double *__restrict__ gK) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ne * npe * npe) return;
  const int64_t e = t / (npe * npe);
  const int ab = (int)(t - e * npe * npe);
  const int a = ab / npe, bb = ab - (ab / npe) * npe;
  const double *la = lam + (int64_t)conn[e * npe + a] * nrhs;
  const double *ub = u + (int64_t)conn[e * npe + bb] * nrhs;
  double s = 0.0;
  for (int r = 0; r < nrhs; ++r) s += la[r] * ub[r];
  gK[t] = -s;
}

}  // namespace mf
