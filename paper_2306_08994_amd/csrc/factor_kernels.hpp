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
#pragma once

#include "common.hpp"

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
k_factor_small(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list, int nlist,
               double *__restrict__ store, const int32_t *__restrict__ inv_l,
               const int32_t *__restrict__ inv_r, const double *__restrict__ K, int npe,
               int *__restrict__ status, int mmax) {
  extern __shared__ double sh[];
  int *ma = reinterpret_cast<int *>(sh + (size_t)mmax * (mmax | 1));   // 2 * mmax ints
  int *mb = ma + mmax;
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int f = list[li];
    const FrontDesc d = fd[f];
    const int m = d.m, k = d.k, ld = m | 1;
    const int32_t *il = inv_l + d.idx;
    const int32_t *ir = inv_r + d.idx;
    const GatherCtx g = gather_ctx(fd, d, store, K, npe);
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
        if (tid == 0) record_bad_pivot(status, f, p);
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

// Extend-add into the front's storage.  grid = (row strips of 4, fronts).
__global__ void __launch_bounds__(256)
k_assemble(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list,
           double *__restrict__ store, const int32_t *__restrict__ inv_l,
           const int32_t *__restrict__ inv_r, const double *__restrict__ K, int npe) {
  extern __shared__ int smaps[];      // the front's column maps: left, then right
  const int f = list[blockIdx.y];
  const FrontDesc d = fd[f];
  const int m = d.m;
  const int i0 = blockIdx.x * 4;
  if (i0 >= m) return;                // uniform per workgroup
  const int32_t *il = inv_l + d.idx;
  const int32_t *ir = inv_r + d.idx;
  int *sl = smaps, *sr = smaps + m;
  for (int j = threadIdx.x; j < m; j += 256) {
    sl[j] = il[j];
    sr[j] = ir[j];
  }
  __syncthreads();
  const GatherCtx g = gather_ctx(fd, d, store, K, npe);
  double *F = store + d.store;
  const int i1 = min(i0 + 4, m);
  for (int i = i0; i < i1; ++i) {
    const int li = sl[i], ri = sr[i];
    for (int j = threadIdx.x; j < m; j += 256)
      F[(int64_t)i * m + j] = gather_entry(g, li, sl[j], ri, sr[j]);
  }
}

// Value of v in lane l of the wave (l uniform across the wave).
__device__ inline double readlane(double v, int l) {
  const unsigned long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffull), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// LU (division tasks scale the pivot row) of the pb x pb diagonal block at F (leading
// dimension m) by one wave, register resident: lane j holds column j of the block, padded with
// the identity beyond pb so that every step runs unconditionally.  At pivot p every lane reads
// the pivot and the multiplier column from lane p (readlane), lane j > p divides its U[p][j]
// and updates its column -- no LDS traffic and no synchronisation inside the block.
// The factored (padded) block is left in LDS D and the pivots' reciprocals in rd (for the panel
// solves), and, if writeback, the pb x pb block in F.  Returns false on a bad pivot (the same
// value on every lane) after recording the first one.
template <int NB>
__device__ __forceinline__ bool wave_diag_lu(double *F, int64_t m, int pb, double (*D)[NB + 1],
                                             double *rd, int lane, int f, int p0, int *status,
                                             bool writeback = true) {
  static_assert(NB <= 64, "one lane per column");
  const bool in = lane < pb;
  const double *src = F + (in ? lane : 0);
  double col[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const double v = src[(int64_t)min(i, pb - 1) * m];
    col[i] = (in && i < pb) ? v : (i == lane ? 1.0 : 0.0);
  }
  int bad = NB;
#pragma unroll
  for (int p = 0; p < NB; ++p) {
    const double piv = readlane(col[p], p);
    if (bad == NB && !good_pivot(piv)) bad = p;
    const bool act = lane > p;
    const double u = act ? col[p] / piv : col[p];
    col[p] = u;
    const double ua = act ? u : 0.0;
#pragma unroll
    for (int i = p + 1; i < NB; ++i) col[i] -= readlane(col[i], p) * ua;
  }
  if (bad < pb && lane == 0) record_bad_pivot(status, f, p0 + bad);
  if (lane < NB) {
#pragma unroll
    for (int i = 0; i < NB; ++i) D[i][lane] = col[i];
  }
  if (writeback && in) {
    if (pb == NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) F[i * m + lane] = col[i];
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < pb) F[i * m + lane] = col[i];
    }
  }
  wave_sync();
  if (lane < NB) rd[lane] = 1.0 / D[lane][lane];
  wave_sync();
  return bad >= pb;
}

// The same as a call (the fused per-front kernel keeps its registers for the panel updates).
template <int NB>
__device__ __noinline__ bool wave_diag_lu_call(double *F, int64_t m, int pb, double (*D)[NB + 1],
                                               double *rd, int lane, int f, int p0, int *status) {
  return wave_diag_lu<NB>(F, m, pb, D, rd, lane, f, p0, status, true);
}

// Panel step of the fronts wider than the fused route: every workgroup factors the pb x pb
// diagonal block at (p0, p0) itself (wave 0, in LDS), then its threads solve against it:
//   U12 = L11^{-1} A12 column by column (rows p0..pe-1, columns pe..m-1),
//   L21 = A21 U11^{-1} row by row       (rows pe..m-1, columns p0..pe-1).
// grid = (item chunks of 256, fronts), at least one chunk; item t < m-pe is a column, else a row.
// Positions beyond pb load clamped (finite) values; the identity padding of D keeps them out of
// the first pb results, and only those are stored.
// The factored diagonal block overwrites the block that the other workgroups of the front read,
// and a workgroup may start only after another has finished (more workgroups than fit on the
// chip at once), so the store is left to the workgroup that arrives last: each workgroup counts
// itself in arrive[f] once its copy is loaded, and the one that sees every other arrival stores
// the block and resets the counter to zero for the next panel step.
template <int NB>
__global__ void __launch_bounds__(256)
k_panel_trsm(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ fronts,
             const int32_t *__restrict__ p0s, double *__restrict__ store,
             int *__restrict__ status, int *__restrict__ arrive) {
  __shared__ double D[NB][NB + 1];
  __shared__ double rd[NB];
  const int f = fronts[blockIdx.y];
  const int p0 = p0s[blockIdx.y];
  const FrontDesc d = fd[f];
  const int m = d.m, pb = min(NB, d.k - p0), pe = p0 + pb;
  const int rest = m - pe;
  const int item = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x > 0 && (int)(blockIdx.x * 256) >= 2 * rest) return;   // idle (uniform)
  double *F = store + d.store;
  // this thread's column (item < rest) or row, loaded before the diagonal block is factored so
  // that the load latency overlaps the factorization
  const bool has = item < 2 * rest, colitem = item < rest;
  double *cp = F + (int64_t)p0 * m + pe + item;
  double *row = F + (int64_t)(pe + item - rest) * m + p0;
  double v[NB];
  if (has) {
    if (colitem) {
#pragma unroll
      for (int q = 0; q < NB; ++q) v[q] = cp[(int64_t)min(q, pb - 1) * m];
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q) v[q] = row[min(q, pb - 1)];
    }
  }
  // workgroups that take part (the others returned above): at least one
  const int nact = max(1, (2 * rest + 255) / 256);
  if (threadIdx.x < 64)
    wave_diag_lu<NB>(F + (int64_t)p0 * m + p0, m, pb, D, rd, threadIdx.x, f, p0, status,
                     nact == 1);
  __syncthreads();
  if (has) {
    if (colitem) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= D[q][r] * v[r];
          s1 -= D[q][r + 1] * v[r + 1];
        }
        if (q & 1) s0 -= D[q][q - 1] * v[q - 1];
        v[q] = (s0 + s1) * rd[q];
      }
      if (pb == NB) {
#pragma unroll
        for (int q = 0; q < NB; ++q) cp[(int64_t)q * m] = v[q];
      } else {
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < pb) cp[(int64_t)q * m] = v[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= v[r] * D[r][q];
          s1 -= v[r + 1] * D[r + 1][q];
        }
        if (q & 1) s0 -= v[q - 1] * D[q - 1][q];
        v[q] = s0 + s1;
      }
      if (pb == NB) {
#pragma unroll
        for (int q = 0; q < NB; ++q) row[q] = v[q];
      } else {
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < pb) row[q] = v[q];
      }
    }
  }
  if (nact > 1 && threadIdx.x < 64) {
    // every thread of this workgroup is past its reads of the diagonal block (the LU consumed
    // them before the barrier); count this workgroup and store the block if it is the last
    int prev = 0;
    if (threadIdx.x == 0)
      prev = __hip_atomic_fetch_add(arrive + f, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    prev = __builtin_amdgcn_readlane(prev, 0);
    if (prev == nact - 1) {
      const int lane = threadIdx.x;
      if (lane < pb) {
        double *dst = F + (int64_t)p0 * m + p0 + lane;
        for (int i = 0; i < pb; ++i) dst[(int64_t)i * m] = D[i][lane];
      }
      if (lane == 0) __hip_atomic_store(arrive + f, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused per-front partial LU of the fully summed rows and columns (fronts up to FP_MAXM wide):
// one workgroup per front runs every panel of NB pivots:
//   1. wave 0 factors the diagonal block in LDS;
//   2. every thread solves L21 rows against U11 (row per thread), keeping them in LDS;
//   3. every thread solves one U12 column against L11 into registers and applies it to its
//      column of the rest of the fully summed region: C[i][j] -= sum_q L21[i][q] U12[q][j],
//      rows i >= pe (all of them for j < k, only the fully summed ones for j >= k).  Lanes run
//      along columns, so every global access of the update is coalesced, and the L21 entries
//      are LDS broadcasts.
// The Schur complement C22 is left to the MFMA GEMM.  LDS: D (NB x NB+1) | L21 panel (m-pe x NB).
// ---------------------------------------------------------------------------------------------
constexpr int FP_THREADS = 512;
constexpr int FP_ROWS = 2;            // rows (and columns) per thread
constexpr int FP_MAXM = 576;          // widest front of this route (LDS and FP_ROWS bound)

template <int NB>
__global__ void __launch_bounds__(FP_THREADS)
k_front_panels(const FrontDesc *__restrict__ fd, const int32_t *__restrict__ list, int nlist,
               double *__restrict__ store, int *__restrict__ status) {
  static_assert(FP_ROWS * FP_THREADS >= FP_MAXM, "rows per thread");
  static_assert(NB % 2 == 0, "two partial sums");
  extern __shared__ double sm[];
  double(*D)[NB + 1] = reinterpret_cast<double(*)[NB + 1]>(sm);
  double *rd = sm + NB * (NB + 1);
  double *Lp = rd + NB;
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int f = list[li];
    const FrontDesc d = fd[f];
    const int m = d.m, k = d.k;
    double *F = store + d.store;
    if (tid == 0) bad = 0;
    for (int p0 = 0; p0 < k; p0 += NB) {
      const int pb = min(NB, k - p0), pe = p0 + pb, rest = m - pe;
      if (wv == 0 && !wave_diag_lu_call<NB>(F + (int64_t)p0 * m + p0, m, pb, D, rd, lane, f, p0, status))
        if (lane == 0) bad = 1;
      __syncthreads();
      if (bad) break;
      // L21 rows pe..m-1:  l = a U11^{-1}
      for (int o = tid; o < rest; o += FP_THREADS) {
        double *row = F + (int64_t)(pe + o) * m + p0;
        double v[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) v[q] = q < pb ? row[q] : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (q < pb) {
            double t = v[q];
#pragma unroll
            for (int r = 0; r < q; ++r) t -= v[r] * D[r][q];
            v[q] = t;
          }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (q < pb) row[q] = v[q];
          Lp[o * NB + q] = v[q];          // zero beyond pb
        }
      }
      __syncthreads();
      // U12 columns pe..m-1:  u = L11^{-1} a, then the column's update
      for (int o = tid; o < rest; o += FP_THREADS) {
        const int j = pe + o;
        double *colp = F + (int64_t)p0 * m + j;
        double u[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) u[q] = q < pb ? colp[(int64_t)q * m] : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (q < pb) {
            double t = u[q];
#pragma unroll
            for (int r = 0; r < q; ++r) t -= D[q][r] * u[r];
            u[q] = t * rd[q];
          }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < pb) colp[(int64_t)q * m] = u[q];
        const int iend = j < k ? m : k;
        double *Cj = F + j;
        // four rows per round: their loads issue together
        int i = pe;
        for (; i + 4 <= iend; i += 4) {
          double c[4], a0[4], a1[4];
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            c[w] = Cj[(int64_t)(i + w) * m];
            a0[w] = 0.0;
            a1[w] = 0.0;
          }
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const double *lr = Lp + (i + w - pe) * NB;
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
              a0[w] += lr[2 * q] * u[2 * q];
              a1[w] += lr[2 * q + 1] * u[2 * q + 1];
            }
          }
#pragma unroll
          for (int w = 0; w < 4; ++w) Cj[(int64_t)(i + w) * m] = c[w] - (a0[w] + a1[w]);
        }
        for (; i < iend; ++i) {
          const double *lr = Lp + (i - pe) * NB;
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int q = 0; q < NB / 2; ++q) {
            a0 += lr[2 * q] * u[2 * q];
            a1 += lr[2 * q + 1] * u[2 * q + 1];
          }
          Cj[(int64_t)i * m] -= a0 + a1;
        }
      }
      __syncthreads();
    }
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
__global__ void __launch_bounds__(256)
k_gemm_update(const FrontDesc *__restrict__ fd, const GemmTask *__restrict__ tasks,
              double *__restrict__ store) {
  typedef typename GemmCfg<PREC>::T T;
  constexpr int KT = GemmCfg<PREC>::KT;
  constexpr int APAD = (PREC == 2) ? 8 : 1;
  constexpr int QB = TILE / 32;            // 16 x 16 MFMA blocks per wave and dimension
  constexpr int HALF = TILE / 2;           // each wave owns a HALF x HALF quadrant
  constexpr int EA = TILE * KT / 256;      // staged elements of A (and of B) per thread
  static_assert(TILE == 32 || TILE == 64, "tile");
  __shared__ T As[TILE][KT + APAD];
  __shared__ T Bs[TILE][KT + APAD];        // stored transposed: Bs[col][k]
  const GemmTask tk = tasks[blockIdx.x];
  const FrontDesc d = fd[tk.front];
  const int64_t ld = d.m;
  double *F = store + d.store;
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
#pragma unroll
      for (int s = 0; s < KT / 4; ++s) {
        T av[QB], bv[QB];
#pragma unroll
        for (int a = 0; a < QB; ++a) av[a] = As[HALF * wr + 16 * a + li][4 * s + lk];
#pragma unroll
        for (int b = 0; b < QB; ++b) bv[b] = Bs[HALF * wc + 16 * b + li][4 * s + lk];
#pragma unroll
        for (int a = 0; a < QB; ++a)
#pragma unroll
          for (int b = 0; b < QB; ++b) {
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
  for (int a = 0; a < QB; ++a)
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 interleaves its result rows (lane l, register r -> row 4r + l/16); the
        // f32 16x16x4 and bf16 16x16x32 forms place them contiguously (row 4(l/16) + r)
        const int gi = i0 + HALF * wr + 16 * a + (PREC == 0 ? 4 * r + lk : 4 * lk + r);
        const int gj = j0 + HALF * wc + 16 * b + li;
        if (gi < tk.i1 && gj < tk.j1) F[gi * ld + gj] -= (double)acc[a][b][r];
      }
}

}  // namespace mf
