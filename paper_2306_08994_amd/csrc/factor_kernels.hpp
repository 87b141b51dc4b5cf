// factor_kernels.hpp -- gfx950 kernels of the multifrontal factorization.
//
// Per Foata class, every front is assembled (extend-add of its children's contribution blocks,
// or its element matrix for a leaf) and partially eliminated: for each pivot p the division
// tasks scale row p by the pivot, then every (i, j) > p receives its multiplication and
// subtraction F[i][j] -= F[i][p] U[p][j] (Table 2).  Three routes by front width:
//   tiny   one wave per front, front in LDS, wave-level ordering only;
//   small  one workgroup per front, front in LDS;
//   tiled  front in HBM: extend-add, then panels of NB pivots (diagonal-block LU, the two
//          triangular panel solves, trailing update of the fully summed rows and columns), then
//          the Schur update C22 -= L21 U12 as one MFMA GEMM.
// The panel kernels (diagonal-block LU, panel step, fused per-front panels) are in
// panel_kernels.hpp.
#pragma once

#include "common.hpp"
#include "panel_kernels.hpp"

namespace mf {

// ---------------------------------------------------------------------------------------------
// tiny: one wave per front (m <= kTinyMaxM), four fronts per workgroup, grid-stride over the
// class's wave records.  The record (uniform: scalar loads), then the extend-add maps and every
// entry of both sources, held in registers (U per lane), in one round of loads; then the
// scatter into the LDS front, the k pivot steps and the store of the front.
// ---------------------------------------------------------------------------------------------
constexpr int kTinyMaxM = 32;

__device__ __forceinline__ const double *rec_source(int64_t src, const double *store,
                                                    const double *K) {
  return src >= 0 ? store + src : K + (-1 - src);
}

// Entries t = lane + 64 u (u < U) of an n x n source (row-major, rows ld apart) into v; zero
// where t >= n * n (n = 0: nothing).
template <int U>
__device__ __forceinline__ void stage_source(const double *__restrict__ src, int ld, int n,
                                             int lane, double (&v)[U]) {
  const int nn = n > 0 ? n : 1;
  int r = lane / nn, c = lane - r * nn;
  const int q = 64 / nn, rem = 64 - q * nn;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    v[u] = r < n ? src[r * ld + c] : 0.0;          // 32-bit offsets: n, ld <= kTinyMaxM
    c += rem;
    r += q;
    if (c >= nn) {
      c -= nn;
      ++r;
    }
  }
}

// The staged entries assigned (ADD = false) or added into the LDS front at map[row], map[col].
template <bool ADD, int U>
__device__ __forceinline__ void scatter_staged(const double (&v)[U], int n, const int *map, int ld,
                                               double *sh, int lane) {
  const int nn = n > 0 ? n : 1;
  int r = lane / nn, c = lane - r * nn;
  const int q = 64 / nn, rem = 64 - q * nn;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (r < n) {
      const int dst = map[r] * ld + map[c];
      if (ADD)
        sh[dst] += v[u];
      else
        sh[dst] = v[u];
    }
    c += rem;
    r += q;
    if (c >= nn) {
      c -= nn;
      ++r;
    }
  }
}

// One tiny front, by one wave: the record's maps and both sources staged in registers, the
// scatter into the LDS front sh (rows ld = m | 1 apart; ma / mb: 2 * mmax ints of map scratch),
// the k pivot steps, the store of the front.  U = ceil(mmax^2 / 64): the widest front of the
// launch bounds every source (a child's CB and an element matrix are never wider than the
// front they enter).
template <int U>
__device__ __forceinline__ void tiny_front(const WaveRec r, int lane, double *sh, int *ma,
                                           int *mb, double *store, const int32_t *inv_l,
                                           const int32_t *inv_r, const double *K, int *status) {
  const int m = r.m, k = r.k, ld = m | 1;
  int xa = -1, xb = -1;
  if (lane < m) {
    xa = inv_l[r.idx + lane];
    if (r.n[1] > 0) xb = inv_r[r.idx + lane];
  }
  double va[U], vb[U];
  stage_source<U>(rec_source(r.src[0], store, K), r.ld[0], r.n[0], lane, va);
  stage_source<U>(rec_source(r.src[1], store, K), r.ld[1], r.n[1], lane, vb);
  for (int t = lane; t < m * ld; t += 64) sh[t] = 0.0;
  if (xa >= 0) ma[xa] = lane;
  if (xb >= 0) mb[xb] = lane;
  wave_sync();
  // the left source assigned, then the right one added: each front entry is summed left
  // then right, as in the extend-add of the two children
  scatter_staged<false, U>(va, r.n[0], ma, ld, sh, lane);
  wave_sync();
  scatter_staged<true, U>(vb, r.n[1], mb, ld, sh, lane);
  wave_sync();
  // pivot steps: lane (h, jj) owns column p + 1 + jj of the rows p + 1 + h, p + 3 + h, ...
  // (m <= 32: one column per half-wave lane); its multiplier u = F[p][j] / piv stays in a
  // register, written back to row p by the first half
  const int jj = lane & 31, h = lane >> 5;
  for (int p = 0; p < k; ++p) {
    const double piv = sh[p * ld + p];
    if (!good_pivot(piv)) {
      if (lane == 0) record_bad_pivot(status, r.f, p);
      break;
    }
    const int j = p + 1 + jj;
    if (j < m) {
      const double u = sh[p * ld + j] / piv;
      if (h == 0) sh[p * ld + j] = u;
#pragma unroll 4
      for (int i = p + 1 + h; i < m; i += 2) sh[i * ld + j] -= sh[i * ld + p] * u;
    }
    wave_sync();
  }
  double *out = store + r.store;
  if (jj < m)
    for (int i = h; i < m; i += 2) out[i * m + jj] = sh[i * ld + jj];
  wave_sync();
}

template <int U>
__global__ void __launch_bounds__(256)
k_factor_tiny(const WaveRec *__restrict__ recs, int nrec, double *__restrict__ store,
              const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
              const double *__restrict__ K, int *__restrict__ status, int ldsw, int mmax) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar loads of the record
  double *sh = sm + wv * ldsw;
  int *ma = reinterpret_cast<int *>(sh + (ldsw - mmax));   // 2 * mmax ints after the front
  int *mb = ma + mmax;
  for (int li = blockIdx.x * 4 + wv; li < nrec; li += gridDim.x * 4)
    tiny_front<U>(recs[li], lane, sh, ma, mb, store, inv_l, inv_r, K, status);
}

// ---------------------------------------------------------------------------------------------
// Bottom subtrees: classes 0..ncls-1 of the tiny route in one launch.  A unit is a front of
// class < ncls whose parent lies above that range (or a root), with all its descendants; one
// workgroup takes a unit's fronts class by class, one front per wave, with a workgroup barrier
// between classes.  Every child of a front is in the front's unit and was stored by the same
// workgroup before the barrier, so the barrier between Foata classes (Sec. 3.3) holds inside
// the unit without a launch per class.  Records unit after unit, class after class:
// ptr[u * ncls + c] is the first record of unit u's class c (ptr[nsub * ncls] = the total).
// Each front is the tiny route's arithmetic in the same order, so the results are identical.
// ---------------------------------------------------------------------------------------------
template <int U>
__global__ void __launch_bounds__(256)
k_factor_subtree(const WaveRec *__restrict__ recs, const int32_t *__restrict__ ptr, int nsub,
                 int ncls, double *store, const int32_t *__restrict__ inv_l,
                 const int32_t *__restrict__ inv_r, const double *__restrict__ K,
                 int *__restrict__ status, int ldsw, int mmax) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *sh = sm + wv * ldsw;
  int *ma = reinterpret_cast<int *>(sh + (ldsw - mmax));
  int *mb = ma + mmax;
  for (int u = blockIdx.x; u < nsub; u += gridDim.x) {
    const int32_t *pu = ptr + (int64_t)u * ncls;
    for (int c = 0; c < ncls; ++c) {
      const int a = pu[c], e = pu[c + 1];
      for (int li = a + wv; li < e; li += 4)
        tiny_front<U>(recs[li], lane, sh, ma, mb, store, inv_l, inv_r, K, status);
      __syncthreads();   // the class's fronts stored before the next class gathers them
    }
  }
}

// ---------------------------------------------------------------------------------------------
// small: one workgroup of NT threads per front, the whole front resident in LDS, eliminated in
// panels of SM_NB pivots (Table 2's division, multiplication and subtraction tasks, blocked):
//   1. wave 0 factors the pb x pb diagonal block (register resident, readlane broadcasts);
//   2. one thread per column solves U12 = L11^{-1} A12 (the division tasks of the panel's rows
//      and their updates inside the panel), one thread per row solves L21 = A21 U11^{-1};
//   3. the trailing matrix (the rest of the fully summed part and the contribution block) takes
//      the panel's multiplications and subtractions at once, A22 -= L21 U12, as 16 x 16 blocks
//      of v_mfma_f64_16x16x4f64 with operands and results in LDS.
// Three barriers per panel instead of one per pivot, and one LDS read and write of each trailing
// entry per panel instead of per pivot.  LDS: front (m rows of m|1) | D (NB x NB+1) | rd (NB) |
// extend-add maps (2 m ints).  NT = 512 when a class has few fronts (each front's steps spread
// over eight waves); 256 when it has more fronts than the chip has compute units, so that more
// fronts are resident at once (the kernel's register use allows three waves per SIMD: one
// 512-thread workgroup per compute unit, or three of 256).
// ---------------------------------------------------------------------------------------------
constexpr int SM_THREADS = 512;      // the larger workgroup of the small route
constexpr int SM_NB = 8;

__host__ __device__ inline int64_t small_lds_doubles(int m) {
  return (int64_t)m * (m | 1) + SM_NB * (SM_NB + 1) + SM_NB + m;
}

template <int NT>
__global__ void __launch_bounds__(NT)
k_factor_small(const WaveRec *__restrict__ recs, int nrec, double *__restrict__ store,
               const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
               const double *__restrict__ K, int *__restrict__ status, int mmax) {
  constexpr int NB = SM_NB;
  extern __shared__ double sh[];
  double(*D)[NB + 1] = reinterpret_cast<double(*)[NB + 1]>(sh + (size_t)mmax * (mmax | 1));
  double *rd = sh + (size_t)mmax * (mmax | 1) + NB * (NB + 1);
  int *ma = reinterpret_cast<int *>(rd + NB);   // 2 * mmax ints
  int *mb = ma + mmax;
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  for (int fi = blockIdx.x; fi < nrec; fi += gridDim.x) {
    const WaveRec d = recs[fi];
    const int m = d.m, k = d.k, ld = m | 1;
    const GatherCtx g = rec_gather_ctx(d, store, K);
    if (tid == 0) s_bad = 0;
    scatter_assemble(g, inv_l + d.idx, inv_r + d.idx, m, ld, sh, ma, mb, tid, NT,
                     [] __device__() { __syncthreads(); });
    for (int p0 = 0; p0 < k; p0 += NB) {
      const int pb = min(NB, k - p0), pe = p0 + pb, rest = m - pe;
      // 1. the diagonal block, factored in registers and written back in place
      if (wv == 0 && !wave_diag_lu<NB>(sh + p0 * ld + p0, ld, pb, D, rd, lane, d.f, p0, status))
        if (lane == 0) s_bad = 1;
      __syncthreads();
      if (s_bad) break;                                     // uniform
      // 2. U12 columns (items t < rest) and L21 rows (items from the next multiple of 64, so
      //    that no wave holds both kinds); positions beyond pb meet the identity padding of D
      const int rpad = (rest + 63) & ~63;
      for (int t = tid; t < rpad + rest; t += NT) {
        if (t < rest) {
          double *cp = sh + p0 * ld + pe + t;
          double v[NB];
#pragma unroll
          for (int q = 0; q < NB; ++q) v[q] = cp[min(q, pb - 1) * ld];
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            double a = v[q];
#pragma unroll
            for (int r = 0; r < q; ++r) a -= D[q][r] * v[r];
            v[q] = a * rd[q];
          }
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < pb) cp[q * ld] = v[q];
        } else if (t >= rpad) {
          double *row = sh + (pe + t - rpad) * ld + p0;
          double v[NB];
#pragma unroll
          for (int q = 0; q < NB; ++q) v[q] = row[min(q, pb - 1)];
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            double a = v[q];
#pragma unroll
            for (int r = 0; r < q; ++r) a -= v[r] * D[r][q];
            v[q] = a;
          }
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < pb) row[q] = v[q];
        }
      }
      __syncthreads();
      // 3. A22 -= L21 U12 over the rest x rest trailing matrix, one 16 x 16 block per wave at a
      //    time: A operand lane l = L21[row l%16][q = l/16 + 4s] (negated), B operand lane l =
      //    U12[q = l/16 + 4s][col l%16], result lane l register r at row 4r + l/16, col l%16
      const int nbk = (rest + 15) >> 4;
      for (int blk = wv; blk < nbk * nbk; blk += NT / 64) {
        const int bi = blk / nbk, bj = blk - bi * nbk;
        const int r0 = pe + 16 * bi, c0 = pe + 16 * bj;
        const int col = c0 + li;
        v4d acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 4 * r + lk;
          acc[r] = (row < m && col < m) ? sh[row * ld + col] : 0.0;
        }
        const int arow = r0 + li;
#pragma unroll
        for (int s = 0; s < NB / 4; ++s) {
          const int q = 4 * s + lk;
          const double a = (q < pb && arow < m) ? -sh[arow * ld + p0 + q] : 0.0;
          const double b = (q < pb && col < m) ? sh[(p0 + q) * ld + col] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 4 * r + lk;
          if (row < m && col < m) sh[row * ld + col] = acc[r];
        }
      }
      __syncthreads();
    }
    double *out = store + d.store;
    {
      const int di = NT / m, dj = NT - di * m;
      int i = tid / m, jj = tid - i * m;
      for (int t = tid; t < m * m; t += NT) {
        out[t] = sh[i * ld + jj];
        jj += dj;
        i += di;
        if (jj >= m) {
          jj -= m;
          ++i;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// tiled path
// ---------------------------------------------------------------------------------------------

// Rows i0 .. i1-1 of the extend-add of one front into its storage, by a workgroup of 256
// threads: the front's maps staged in LDS (smaps, 2 m ints), then per column of each thread the
// strip's entries gathered four rows at a time and stored.  Begins and ends with a workgroup
// barrier (smaps may be in use before and is free after).
__device__ __forceinline__ void assemble_rows(const WaveRec &d, int i0, int i1,
                                              double *__restrict__ store,
                                              const int32_t *__restrict__ inv_l,
                                              const int32_t *__restrict__ inv_r,
                                              const double *__restrict__ K, int *smaps) {
  const int m = d.m;
  const int32_t *il = inv_l + d.idx;
  const int32_t *ir = inv_r + d.idx;
  int *sl = smaps, *sr = smaps + m;
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += 256) {
    sl[j] = il[j];
    sr[j] = ir[j];
  }
  __syncthreads();
  const GatherCtx g = rec_gather_ctx(d, store, K);
  double *F = store + d.store;
  for (int r0 = i0; r0 < i1; r0 += 4) {
    for (int j = threadIdx.x; j < m; j += 256) {
      const int lj = sl[j], rj = sr[j];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = min(r0 + u, i1 - 1);
        v[u] = gather_entry(g, sl[i], lj, sr[i], rj);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (r0 + u < i1) F[(int64_t)(r0 + u) * m + j] = v[u];
    }
  }
  __syncthreads();
}

// Extend-add into the front's storage.  grid = (row strips of 4, fronts); the fronts beyond
// gridDim.y are taken grid-stride.
__global__ void __launch_bounds__(256)
k_assemble(const WaveRec *__restrict__ recs, int nrec, double *__restrict__ store,
           const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
           const double *__restrict__ K) {
  extern __shared__ int smaps[];      // the front's column maps: left, then right
  for (int fi = blockIdx.y; fi < nrec; fi += gridDim.y) {
    const WaveRec d = recs[fi];
    const int i0 = blockIdx.x * 4;
    if (i0 >= d.m) continue;            // uniform per workgroup
    assemble_rows(d, i0, min(i0 + 4, d.m), store, inv_l, inv_r, K, smaps);
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

template <int PREC, int TILE>
struct GemmLds {
  typedef typename GemmCfg<PREC>::T T;
  // inner-dimension slab: 32 (a panel update is one slab; a 64 x 64 tile does 32 MFMA k-steps
  // per wave between two barriers)
  static constexpr int KT = 32;
  static constexpr int APAD = (PREC == 2) ? 8 : 1;
  T As[TILE][KT + APAD];
  T Bs[TILE][KT + APAD];        // stored transposed: Bs[col][k]
};

// One tile task of the GEMM update, by a workgroup of 256 threads (4 waves) with its operand
// staging in `sm` (LDS); every slab ends with a workgroup barrier, so sm is free on return.
template <int PREC, int TILE>
__device__ __forceinline__ void gemm_tile(const GemmTask &tk, double *__restrict__ store,
                                          GemmLds<PREC, TILE> &sm) {
  typedef typename GemmCfg<PREC>::T T;
  constexpr int KT = GemmLds<PREC, TILE>::KT;
  constexpr int QB = TILE / 32;            // 16 x 16 MFMA blocks per wave and dimension
  constexpr int HALF = TILE / 2;           // each wave owns a HALF x HALF quadrant
  constexpr int EA = TILE * KT / 256;      // staged elements of A (and of B) per thread
  static_assert(TILE == 32 || TILE == 64, "tile");
  auto &As = sm.As;
  auto &Bs = sm.Bs;
  const int64_t ld = tk.ld;
  double *F = store + tk.store;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename std::conditional<PREC == 0, v4d, v4f>::type Acc;
  Acc acc[QB][QB];
#pragma unroll
  for (int a = 0; a < QB; ++a)
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;
  const int i0 = tk.i0, j0 = tk.j0;
  // A[i0:i0+TILE, q:q+KT] and B[q:q+KT, j0:j0+TILE], zero outside the task; the next slab is
  // loaded into registers while the current one is multiplied
  double ra[EA], rb[EA];
  auto load = [&](int q) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int t = tid + e * 256;
      const int ar = t / KT, ac = t % KT;
      const int gi = i0 + ar, gq = q + ac;
      ra[e] = (gi < tk.i1 && gq < tk.q1) ? F[gi * ld + gq] : 0.0;
      const int bc = t % TILE, br = t / TILE;
      const int gq2 = q + br, gj = j0 + bc;
      rb[e] = (gq2 < tk.q1 && gj < tk.j1) ? F[gq2 * ld + gj] : 0.0;
    }
  };
  // this thread's C entries, read together with the first slab (not after the products)
  double cv[QB][QB][4];
#pragma unroll
  for (int a = 0; a < QB; ++a)
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + HALF * wr + 16 * a + (PREC == 0 ? 4 * r + lk : 4 * lk + r);
        const int gj = j0 + HALF * wc + 16 * b + li;
        cv[a][b][r] = (gi < tk.i1 && gj < tk.j1) ? F[gi * ld + gj] : 0.0;
      }
  if (tk.q0 < tk.q1) load(tk.q0);
  for (int q = tk.q0; q < tk.q1; q += KT) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int t = tid + e * 256;
      As[t / KT][t % KT] = (T)ra[e];
      Bs[t % TILE][t / TILE] = (T)rb[e];
    }
    __syncthreads();
    if (q + KT < tk.q1) load(q + KT);
    if constexpr (PREC == 2) {
      v8bf av[QB], bv[QB];
#pragma unroll
      for (int a = 0; a < QB; ++a)
#pragma unroll
        for (int e = 0; e < 8; ++e) av[a][e] = As[HALF * wr + 16 * a + li][8 * lk + e];
#pragma unroll
      for (int b = 0; b < QB; ++b)
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[b][e] = Bs[HALF * wc + 16 * b + li][8 * lk + e];
#pragma unroll
      for (int a = 0; a < QB; ++a)
#pragma unroll
        for (int b = 0; b < QB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    } else {
      // the operands of S k-steps read from LDS first (reads issued together), then their
      // MFMAs; S bounds the registers the staged operands take (16 / (QB * QB) k-steps)
      constexpr int S = (QB == 1) ? KT / 4 : 4;
#pragma unroll
      for (int s0 = 0; s0 < KT / 4; s0 += S) {
        T av[S][QB], bv[S][QB];
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
          for (int a = 0; a < QB; ++a) av[s][a] = As[HALF * wr + 16 * a + li][4 * (s0 + s) + lk];
#pragma unroll
          for (int b = 0; b < QB; ++b) bv[s][b] = Bs[HALF * wc + 16 * b + li][4 * (s0 + s) + lk];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int a = 0; a < QB; ++a)
#pragma unroll
            for (int b = 0; b < QB; ++b) {
              if constexpr (PREC == 0)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a], bv[s][b], acc[a][b], 0, 0, 0);
              else
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s][a], bv[s][b], acc[a][b], 0, 0, 0);
            }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < QB; ++a)
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 interleaves its result rows (lane l, register r -> row 4r + l/16); the
        // f32 16x16x4 and bf16 16x16x32 forms place them contiguously (row 4(l/16) + r)
        const int gi = i0 + HALF * wr + 16 * a + (PREC == 0 ? 4 * r + lk : 4 * lk + r);
        const int gj = j0 + HALF * wc + 16 * b + li;
        if (gi < tk.i1 && gj < tk.j1) F[gi * ld + gj] = cv[a][b][r] - (double)acc[a][b][r];
      }
}

template <int PREC, int TILE>
__global__ void __launch_bounds__(256)
k_gemm_update(const GemmTask *__restrict__ tasks, double *__restrict__ store) {
  __shared__ GemmLds<PREC, TILE> sm;
  gemm_tile<PREC, TILE>(tasks[blockIdx.x], store, sm);
}

// ---------------------------------------------------------------------------------------------
// Panel step in the look-ahead form (panel width 32): one launch per step does
//   A. per front, the panel p0 .. pe-1.  Its rows and columns -- the diagonal block, the U12
//      columns and the L21 rows -- first take the previous panel's trailing update
//      (F -= L U over the previous 32 pivots, Table 2's multiplications and subtractions of
//      those pivots); then the diagonal block is factored and the columns and rows are solved
//      against it, as in k_panel_trsm;
//   B. the previous panel's trailing update of the rest of the fully summed region (rows and
//      columns from pe on), as GEMM tiles in the workgroups after the A chunks.
// A and B write disjoint entries and read only entries that are final when the launch starts, so
// one launch does the work of a panel launch and an update launch: one launch and two
// inter-kernel gaps less per step on the dependency chain of a front.
// An A chunk is 256 threads: wave 0 stages and factors the diagonal block, waves 1-3 hold 192
// items (item t < rest a U12 column, t in [R, R + rest) an L21 row, R = rest rounded up to 64,
// so that no wave holds both kinds).  Each item wave applies the previous panel's update to its
// 64 items as one small product on MFMA while wave 0 factors: done per item against the staged
// 32 x 32 block, every lane would read all 1024 entries (LDS broadcasts, whose return traffic
// kept that phase longer than the factorization it overlaps).  Two waves per SIMD (the
// launch bound), so that the B tiles keep their occupancy.
// ---------------------------------------------------------------------------------------------
constexpr int LA_NB = 32;
constexpr int LA_ITEMS = 192;

__device__ __host__ inline int lookahead_chunks(int m, int pe) {
  const int rest = m - pe, rpad = (rest + 63) & ~63;
  const int c = (rpad + rest + LA_ITEMS - 1) / LA_ITEMS;
  return c > 1 ? c : 1;
}

template <int TILE>
union LookaheadLds {
  struct {
    double D[LA_NB][LA_NB + 1];     // factored diagonal block (identity padding beyond pb)
    double rd[LA_NB];               // reciprocals of its pivots
    double Dg[LA_NB][LA_NB + 1];    // the diagonal block as loaded, then updated
    double Lp[LA_NB][LA_NB + 1];    // Lp[i][q] = F[p0 + i][p0 - 32 + q]: previous panel's L rows
    double UpT[LA_NB][LA_NB + 1];   // UpT[j][q] = F[p0 - 32 + q][p0 + j]: its U columns
    // per item wave: half of its items' previous-panel entries (64 x 16, padded), then half of
    // the products, on their way between the item layout and the MFMA layout
    double Ws[LA_ITEMS / 64][64 * 17];
  } a;
  GemmLds<0, TILE> g;
};

template <int TILE>
__global__ void __launch_bounds__(256, 2)
k_panel_lookahead(const PanelRec *__restrict__ recs, int nrec, int cmax,
                  const GemmTask *__restrict__ tiles, double *__restrict__ store,
                  int *__restrict__ status, int *__restrict__ arrive) {
  constexpr int NB = LA_NB;
  __shared__ LookaheadLds<TILE> sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t na = (int64_t)nrec * cmax;
  if ((int64_t)blockIdx.x >= na) {                       // B: a tile of the previous update
    gemm_tile<0, TILE>(tiles[blockIdx.x - na], store, sm.g);
    return;
  }
  const int fi = (int)(blockIdx.x / cmax), chunk = (int)(blockIdx.x - (int64_t)fi * cmax);
  const PanelRec d = recs[fi];
  const int m = d.m, p0 = d.p0, pb = min(NB, d.k - p0), pe = p0 + pb;
  const int nact = lookahead_chunks(m, pe);
  if (chunk >= nact) return;                             // idle chunk of a narrower front
  const bool prev = p0 > 0;                              // every panel but the last is NB wide
  const int rest = m - pe, rpad = (rest + 63) & ~63;
  const int i0w = chunk * LA_ITEMS + (wv - 1) * 64;      // first item of this wave (waves 1-3)
  double *F = store + d.store;
  // this thread's item: a U12 column (entries F[p0 + q][j], stride m) or an L21 row (entries
  // F[i][p0 + q], stride 1), at 32-bit element offset io from the front's (uniform) base
  const int item = chunk * LA_ITEMS + tid - 64;
  const bool colitem = wv > 0 && item < rest;
  const bool has = colitem || (wv > 0 && item >= rpad && item < rpad + rest);
  const uint32_t io = colitem ? p0 * m + pe + item : (pe + item - rpad) * m + p0;
  double v[NB];
  // the diagonal block and the previous panel's blocks of this panel, staged in LDS by waves
  // 1-3, every load issued before the first store (rows and columns beyond pb clamped: finite
  // values that the identity padding of the factored block keeps out of the results)
  if (wv > 0) {
    constexpr int U = (NB * NB + LA_ITEMS - 1) / LA_ITEMS;
    double a0[U], a1[U], a2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = tid - 64 + LA_ITEMS * u;
      const int i = t >> 5, j = t & (NB - 1), ic = min(i, pb - 1), jc = min(j, pb - 1);
      if (t < NB * NB) {
        a0[u] = F[(p0 + ic) * m + p0 + jc];
        if (prev) {
          a1[u] = F[(p0 + ic) * m + p0 - NB + j];
          a2[u] = F[(p0 - NB + i) * m + p0 + jc];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = tid - 64 + LA_ITEMS * u;
      const int i = t >> 5, j = t & (NB - 1);
      if (t < NB * NB) {
        sm.a.Dg[i][j] = a0[u];
        if (prev) {
          sm.a.Lp[i][j] = a1[u];
          sm.a.UpT[j][i] = a2[u];
        }
      }
    }
  }
  __syncthreads();
  // every workgroup of the front has its copy of the diagonal block once it is past the barrier
  // above: count it (relaxed, as in k_panel_trsm); the last one stores the factored block
  int arrived = 0;
  if (nact > 1 && tid == 0)
    arrived = __hip_atomic_fetch_add(arrive + d.f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (prev) {
    // the previous panel's update of the diagonal block first (the factorization waits for it),
    // one 16 x 16 block per wave on MFMA: A operand lane l = -Lp[row l%16][q], B operand lane l
    // = U[q][col l%16], q = 4 s + l/16; result lane l register r at row 4r + l/16, column l%16
    const int li = lane & 15, lk = lane >> 4, bi = wv >> 1, bj = wv & 1;
    v4d acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = sm.a.Dg[16 * bi + 4 * r + lk][16 * bj + li];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sm.a.Lp[16 * bi + li][4 * q + lk],
                                                 sm.a.UpT[16 * bj + li][4 * q + lk], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) sm.a.Dg[16 * bi + 4 * r + lk][16 * bj + li] = acc[r];
    __syncthreads();
  }
  if (wv == 0) {
    wave_diag_lu<NB>(&sm.a.Dg[0][0], NB + 1, pb, sm.a.D, sm.a.rd, lane, d.f, p0, status, false);
  } else if (wv > 0 && (i0w < rest || (i0w >= rpad && i0w < rpad + rest))) {
    // while wave 0 factors the block: this item's entries in this panel (v) and in the
    // previous one (w) -- loaded here, after the barriers, which wait for every outstanding
    // load -- and the previous panel's update of them, v[q] -= sum_r Lp[q][r] w[r] for a
    // column, v[q] -= sum_r w[r] U[r][q] for a row.  The wave holds only columns or only rows
    // (i0w: its first item); lanes without an item take part with zeros.
    double w[NB];
    if (colitem) {
#pragma unroll
      for (int q = 0; q < NB; ++q) v[q] = F[io + (uint32_t)(min(q, pb - 1) * m)];
      if (prev) {
#pragma unroll
        for (int q = 0; q < NB; ++q) w[q] = F[io + (uint32_t)((q - NB) * m)];
      }
    } else if (has) {
#pragma unroll
      for (int q = 0; q < NB; ++q) v[q] = F[io + (uint32_t)min(q, pb - 1)];
      if (prev) {
#pragma unroll
        for (int q = 0; q < NB; ++q) w[q] = F[io + (uint32_t)(q - NB)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q) v[q] = w[q] = 0.0;
    }
    if (prev) {
      // the wave's 64 items at once, P = W M^T (W: items x 32 previous-panel entries; M = Lp
      // for columns, UpT for rows, M[q][r]) on MFMA: each lane reads distinct entries of M
      // instead of every lane all 1024 (LDS broadcasts, which bound the product otherwise).
      // A operand lane l = W[16 rb + l%16][4 s + l/16] (staged through Ws, 16 entries of each
      // item at a time), B operand lane l = M[16 cb + l%16][4 s + l/16]; result lane l register
      // t = P[16 rb + 4 t + l/16][16 cb + l%16], staged back through Ws per 16 columns.
      const double(*M)[NB + 1] = i0w < rest ? sm.a.Lp : sm.a.UpT;
      double *Ws = sm.a.Ws[wv - 1];
      const int li = lane & 15, lk = lane >> 4;
      v4d acc[4][2];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int t = 0; t < 16; ++t) Ws[lane * 17 + t] = w[16 * h + t];
        wave_sync();
        double aop[4][4], bop[2][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int ss = 0; ss < 4; ++ss) aop[rb][ss] = Ws[(16 * rb + li) * 17 + 4 * ss + lk];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int ss = 0; ss < 4; ++ss) bop[cb][ss] = M[16 * cb + li][16 * h + 4 * ss + lk];
        wave_sync();                                 // read before the next half overwrites
#pragma unroll
        for (int ss = 0; ss < 4; ++ss)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
              acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[rb][ss], bop[cb][ss],
                                                                 acc[rb][cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int t = 0; t < 4; ++t) Ws[(16 * rb + 4 * t + lk) * 17 + li] = acc[rb][cb][t];
        wave_sync();
#pragma unroll
        for (int t = 0; t < 16; ++t) v[16 * cb + t] -= Ws[lane * 17 + t];
        wave_sync();
      }
    }
  }
  __syncthreads();
  if (wv > 0 && (i0w < rest || (i0w >= rpad && i0w < rpad + rest))) {
    // substitution against the factored block: a column solves L11 u = v (pivots on the
    // diagonal: v[q] = (v[q] - sum_{r<q} D[q][r] v[r]) / D[q][q]), a row solves l U11 = v (unit
    // diagonal: v[q] -= sum_{r<q} v[r] D[r][q]); in two halves of 16, the contribution of the
    // first half to the second taken for the wave's 64 items at once on MFMA (as the previous
    // panel's update above), so that the per-item steps read 240 entries of D instead of 496.
    // Each step reads its entries of D into registers first, the reads issued together, and
    // stores its result at once, so that the stores drain while the later steps compute.
    const bool colw = i0w < rest;
    double dr[NB];
    if (colw) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
#pragma unroll
        for (int r = 0; r < q; ++r) dr[r] = sm.a.D[q][r];
        const double rq = sm.a.rd[q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= dr[r] * v[r];
          s1 -= dr[r + 1] * v[r + 1];
        }
        if ((q - 0) & 1) s0 -= dr[q - 1] * v[q - 1];
        v[q] = (s0 + s1) * rq;
        if (has && q < pb) F[io + (uint32_t)(q * m)] = v[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
#pragma unroll
        for (int r = 0; r < q; ++r) dr[r] = sm.a.D[r][q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= dr[r] * v[r];
          s1 -= dr[r + 1] * v[r + 1];
        }
        if ((q - 0) & 1) s0 -= dr[q - 1] * v[q - 1];
        v[q] = s0 + s1;
        // a row's entries are contiguous: a full panel's in 16-byte pairs
        if (has && (q & 1)) {
          if (pb == NB) {
            *reinterpret_cast<d2u *>(F + io + q - 1) = d2u{v[q - 1], v[q]};
          } else {
            if (q - 1 < pb) F[io + (uint32_t)(q - 1)] = v[q - 1];
            if (q < pb) F[io + (uint32_t)q] = v[q];
          }
        }
      }
    }
    {
      // v[16 + j] -= sum_{r<16} M[j][r] v[r], M[j][r] = D[16 + j][r] (columns) or D[r][16 + j]
      // (rows): A operand lane l = v[r = 4 s + l/16] of item 16 rb + l%16 (staged through Ws),
      // B operand lane l = M[l%16][4 s + l/16]; result lane l register t = item 16 rb + 4 t +
      // l/16, j = l%16
      double *Ws = sm.a.Ws[wv - 1];
      const int li = lane & 15, lk = lane >> 4;
#pragma unroll
      for (int t = 0; t < 16; ++t) Ws[lane * 17 + t] = v[t];
      wave_sync();
      double aop[4][4], bop[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) aop[rb][ss] = Ws[(16 * rb + li) * 17 + 4 * ss + lk];
#pragma unroll
      for (int ss = 0; ss < 4; ++ss)
        bop[ss] = colw ? sm.a.D[16 + li][4 * ss + lk] : sm.a.D[4 * ss + lk][16 + li];
      wave_sync();                                   // read before the products overwrite
      v4d acc[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[rb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ss = 0; ss < 4; ++ss)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[rb][ss], bop[ss], acc[rb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int t = 0; t < 4; ++t) Ws[(16 * rb + 4 * t + lk) * 17 + li] = acc[rb][t];
      wave_sync();
#pragma unroll
      for (int t = 0; t < 16; ++t) v[16 + t] -= Ws[lane * 17 + t];
    }
    if (colw) {
#pragma unroll
      for (int q = 16; q < 32; ++q) {
#pragma unroll
        for (int r = 16; r < q; ++r) dr[r] = sm.a.D[q][r];
        const double rq = sm.a.rd[q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 16; r + 1 < q; r += 2) {
          s0 -= dr[r] * v[r];
          s1 -= dr[r + 1] * v[r + 1];
        }
        if ((q - 16) & 1) s0 -= dr[q - 1] * v[q - 1];
        v[q] = (s0 + s1) * rq;
        if (has && q < pb) F[io + (uint32_t)(q * m)] = v[q];
      }
    } else {
#pragma unroll
      for (int q = 16; q < 32; ++q) {
#pragma unroll
        for (int r = 16; r < q; ++r) dr[r] = sm.a.D[r][q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 16; r + 1 < q; r += 2) {
          s0 -= dr[r] * v[r];
          s1 -= dr[r + 1] * v[r + 1];
        }
        if ((q - 16) & 1) s0 -= dr[q - 1] * v[q - 1];
        v[q] = s0 + s1;
        // a row's entries are contiguous: a full panel's in 16-byte pairs
        if (has && (q & 1)) {
          if (pb == NB) {
            *reinterpret_cast<d2u *>(F + io + q - 1) = d2u{v[q - 1], v[q]};
          } else {
            if (q - 1 < pb) F[io + (uint32_t)(q - 1)] = v[q - 1];
            if (q < pb) F[io + (uint32_t)q] = v[q];
          }
        }
      }
    }
  } else if (wv == 0) {
    // the factored diagonal block: by the only workgroup of the front, or by the one that
    // arrived last (every other one has staged the block by now)
    const int last = __builtin_amdgcn_readlane(arrived, 0) == nact - 1;
    if (nact == 1 || last) {
      store_diag_block<NB>(d, store, sm.a.D, lane);
      if (nact > 1 && lane == 0)
        __hip_atomic_store(arrive + d.f, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace mf
