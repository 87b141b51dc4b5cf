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

// U = ceil(mmax^2 / 64): the class's widest tiny front bounds every source (a child's CB and an
// element matrix are never wider than the front they enter).
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
  for (int li = blockIdx.x * 4 + wv; li < nrec; li += gridDim.x * 4) {
    const WaveRec r = recs[li];
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
    for (int p = 0; p < k; ++p) {
      const double piv = sh[p * ld + p];
      if (!good_pivot(piv)) {
        if (lane == 0) record_bad_pivot(status, r.f, p);
        break;
      }
      for (int j = p + 1 + lane; j < m; j += 64) sh[p * ld + j] = sh[p * ld + j] / piv;
      wave_sync();
      const int rr = m - p - 1;
      for (int t = lane; t < rr * rr; t += 64) {
        const int i = p + 1 + t / rr, j = p + 1 + (t - (t / rr) * rr);
        sh[i * ld + j] -= sh[i * ld + p] * sh[p * ld + j];
      }
      wave_sync();
    }
    double *out = store + r.store;
    for (int t = lane; t < m * m; t += 64) {
      const int i = t / m, j = t - (t / m) * m;
      out[t] = sh[i * ld + j];
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------------------------
// small: one workgroup of SM_THREADS per front, the whole front resident in LDS.  Thread t owns
// column j = t mod m of the rows i = g, g + G, ... with g = t div m and G = SM_THREADS div m
// groups.  At pivot p every owner of column j > p forms U[p][j] = F[p][j] / F[p][p] itself
// (the division task) and subtracts F[i][p] U[p][j] from its rows i > p; the scaled row p is
// stored one step later (nothing reads row p then), so one barrier per pivot orders the steps.
// ---------------------------------------------------------------------------------------------
constexpr int SM_THREADS = 512;

__global__ void __launch_bounds__(SM_THREADS)
k_factor_small(const WaveRec *__restrict__ recs, int nrec, double *__restrict__ store,
               const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
               const double *__restrict__ K, int *__restrict__ status, int mmax) {
  extern __shared__ double sh[];
  int *ma = reinterpret_cast<int *>(sh + (size_t)mmax * (mmax | 1));   // 2 * mmax ints
  int *mb = ma + mmax;
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nrec; li += gridDim.x) {
    const WaveRec d = recs[li];
    const int m = d.m, k = d.k, ld = m | 1;
    const int32_t *il = inv_l + d.idx;
    const int32_t *ir = inv_r + d.idx;
    const GatherCtx g = rec_gather_ctx(d, store, K);
    scatter_assemble(g, il, ir, m, ld, sh, ma, mb, tid, SM_THREADS,
                     [] __device__() { __syncthreads(); });
    const int G = SM_THREADS / m;            // row groups per column (m <= SM_THREADS)
    const int j = tid % m, grp = tid / m;
    const bool owner = grp < G;
    double u_prev = 0.0;
    int p = 0;
    for (; p < k; ++p) {
      const double piv = sh[p * ld + p];
      if (!good_pivot(piv)) {
        if (tid == 0) record_bad_pivot(status, d.f, p);
        break;
      }
      double u = 0.0;
      if (owner && j > p) {
        u = sh[p * ld + j] / piv;
        int i = p + 1 + grp;
        for (; i + G < m; i += 2 * G) {
          const double c0 = sh[i * ld + p], c1 = sh[(i + G) * ld + p];
          sh[i * ld + j] -= c0 * u;
          sh[(i + G) * ld + j] -= c1 * u;
        }
        if (i < m) sh[i * ld + j] -= sh[i * ld + p] * u;
      }
      // deferred store of the scaled row p-1 (its owner group is (p-1) mod G)
      if (owner && p > 0 && j > p - 1 && (p - 1) % G == grp) sh[(p - 1) * ld + j] = u_prev;
      u_prev = u;
      __syncthreads();
    }
    if (owner && p > 0 && p == k && j > p - 1 && (p - 1) % G == grp) sh[(p - 1) * ld + j] = u_prev;
    __syncthreads();
    double *out = store + d.store;
    for (int t = tid; t < m * m; t += SM_THREADS) {
      const int i = t / m, jj = t - (t / m) * m;
      out[t] = sh[i * ld + jj];
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
  // inner-dimension slab: 32 at TILE 32 (a panel update is one slab), else the type's depth
  static constexpr int KT = TILE == 32 ? 32 : GemmCfg<PREC>::KT;
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
      // every operand of the slab read from LDS first (reads issued together), then the MFMAs
      T av[KT / 4][QB], bv[KT / 4][QB];
#pragma unroll
      for (int s = 0; s < KT / 4; ++s) {
#pragma unroll
        for (int a = 0; a < QB; ++a) av[s][a] = As[HALF * wr + 16 * a + li][4 * s + lk];
#pragma unroll
        for (int b = 0; b < QB; ++b) bv[s][b] = Bs[HALF * wc + 16 * b + li][4 * s + lk];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < KT / 4; ++s)
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

}  // namespace mf
