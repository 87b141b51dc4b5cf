// panel_kernels.hpp -- gfx950 kernels of the panel factorization of the wide fronts: the
// register-resident LU of a diagonal block by one wave, the panel step of the tiled route
// (diagonal-block LU and the two triangular panel solves, many workgroups per front), and the
// fused route (every panel of a front in one workgroup).  Table 2's division, multiplication and
// subtraction tasks, blocked by panels of NB pivots.
#pragma once

#include "common.hpp"

namespace mf {

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
    // the select is made here: left to the compiler it is sunk to the final stores, which keeps
    // every pivot's lane mask alive in scalar registers and leaves one scalar pair for all the
    // broadcasts below (each broadcast then waits for the previous multiply-add)
    asm volatile("" : "+v"(col[p]));
    const double ua = act ? u : 0.0;
    // the multipliers four at a time, all four live at once (distinct scalar pairs), so that
    // each multiply-add does not wait for the broadcast just before it
#pragma unroll
    for (int i0 = p + 1; i0 < NB; i0 += 4) {
      double mu[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) mu[t] = i0 + t < NB ? readlane(col[i0 + t], p) : 0.0;
      asm volatile("" ::"s"(mu[0]), "s"(mu[1]), "s"(mu[2]), "s"(mu[3]));
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (i0 + t < NB) col[i0 + t] -= mu[t] * ua;
    }
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
// grid = (item chunks of 256, fronts), at least one chunk; with r = m - pe, item t < r is a
// column and item t in [R, R + r) a row, R = r rounded up to a multiple of 64: every wave holds
// only columns or only rows (a wave holding both ran the two substitutions one after the other).
// The host sizes the chunks by the widest front's R + r.
// Positions beyond pb load clamped (finite) values; the identity padding of D keeps them out of
// the first pb results, and only those are stored.
// The factored diagonal block overwrites the block that the other workgroups of the front read,
// and a workgroup may start only after another has finished (more workgroups than fit on the
// chip at once), so the store is left to the workgroup that arrives last: each workgroup counts
// itself in arrive[f] once its copy is loaded, and the one that sees every other arrival stores
// the block and resets the counter to zero for the next panel step.
// Number of 256-item chunks (workgroups) of a panel step of a front: r = m - pe columns, then
// r rows from the next multiple of 64 (at least one chunk).
__device__ __host__ inline int panel_chunks(int m, int pe) {
  const int rest = m - pe, rpad = (rest + 63) & ~63;
  return (rpad + rest + 255) / 256 > 1 ? (rpad + rest + 255) / 256 : 1;
}

// Chunk `chunk` of the panel step (p0 .. pe-1) of one front by a workgroup of 256 threads: the
// loads of its columns / rows, the diagonal-block LU by wave 0 into D / rd (LDS; stored to F
// only if writeback_diag), the two triangular solves and their stores.  Ends after a workgroup
// barrier that follows every thread's reads of D, with the solves' stores issued.
template <int NB>
__device__ __forceinline__ void panel_chunk(const PanelRec &d, int chunk, double *__restrict__ store,
                                            int *__restrict__ status, double (*D)[NB + 1],
                                            double *rd, bool writeback_diag) {
  const int f = d.f, p0 = d.p0;
  const int m = d.m, pb = min(NB, d.k - p0), pe = p0 + pb;
  const int rest = m - pe, rpad = (rest + 63) & ~63;
  const int item = chunk * 256 + threadIdx.x;
  double *F = store + d.store;
  // this thread's column (item < rest) or row, loaded before the diagonal block is factored so
  // that the load latency overlaps the factorization
  const bool colitem = item < rest, has = colitem || (item >= rpad && item < rpad + rest);
  double *cp = F + (int64_t)p0 * m + pe + item;
  double *row = F + (int64_t)(pe + item - rpad) * m + p0;
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
  if (threadIdx.x < 64)
    wave_diag_lu<NB>(F + (int64_t)p0 * m + p0, m, pb, D, rd, threadIdx.x, f, p0, status,
                     writeback_diag);
  __syncthreads();
  if (has) {
    // each step reads its row (column) of D into registers first, the reads issued together,
    // then its products: one LDS round trip per step, overlapped with the previous step
    double dr[NB];
    if (colitem) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
#pragma unroll
        for (int r = 0; r < q; ++r) dr[r] = D[q][r];
        const double rq = rd[q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= dr[r] * v[r];
          s1 -= dr[r + 1] * v[r + 1];
        }
        if (q & 1) s0 -= dr[q - 1] * v[q - 1];
        v[q] = (s0 + s1) * rq;
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
#pragma unroll
        for (int r = 0; r < q; ++r) dr[r] = D[r][q];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = v[q], s1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < q; r += 2) {
          s0 -= v[r] * dr[r];
          s1 -= v[r + 1] * dr[r + 1];
        }
        if (q & 1) s0 -= v[q - 1] * dr[q - 1];
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
  __syncthreads();
}

// The factored pb x pb diagonal block of panel p0 from LDS D into the front (wave 0's lanes).
template <int NB>
__device__ __forceinline__ void store_diag_block(const PanelRec &d, double *__restrict__ store,
                                                 double (*D)[NB + 1], int lane) {
  const int pb = min(NB, d.k - d.p0);
  if (lane < pb) {
    double *dst = store + d.store + (int64_t)d.p0 * d.m + d.p0 + lane;
    for (int i = 0; i < pb; ++i) dst[(int64_t)i * d.m] = D[i][lane];
  }
}

// Panel step of the fronts wider than the fused route: every workgroup factors the pb x pb
// diagonal block at (p0, p0) itself (wave 0, in LDS), then its threads solve against it:
//   U12 = L11^{-1} A12 column by column (rows p0..pe-1, columns pe..m-1),
//   L21 = A21 U11^{-1} row by row       (rows pe..m-1, columns p0..pe-1).
// grid = (item chunks of 256, fronts; fronts beyond gridDim.y grid-stride), at least one chunk;
// with r = m - pe, item t < r is a column and item t in [R, R + r) a row, R = r rounded up to a
// multiple of 64: every wave holds only columns or only rows (a wave holding both ran the two
// substitutions one after the other).  The host sizes the chunks by the widest front's R + r.
// Positions beyond pb load clamped (finite) values; the identity padding of D keeps them out of
// the first pb results, and only those are stored.
// The factored diagonal block overwrites the block that the other workgroups of the front read,
// and a workgroup may start only after another has finished (more workgroups than fit on the
// chip at once), so the store is left to the workgroup that arrives last: each workgroup counts
// itself in arrive[f] once its copy is loaded, and the one that sees every other arrival stores
// the block and resets the counter to zero for the next panel step.
template <int NB>
__global__ void __launch_bounds__(256)
k_panel_trsm(const PanelRec *__restrict__ recs, int nrec, double *__restrict__ store,
             int *__restrict__ status, int *__restrict__ arrive) {
  __shared__ double D[NB][NB + 1];
  __shared__ double rd[NB];
  for (int fi = blockIdx.y; fi < nrec; fi += gridDim.y) {
    const PanelRec d = recs[fi];
    const int nact = panel_chunks(d.m, d.p0 + min(NB, d.k - d.p0));
    if ((int)blockIdx.x >= nact) continue;   // idle chunk of a narrower front (uniform)
    panel_chunk<NB>(d, blockIdx.x, store, status, D, rd, nact == 1);
    if (nact > 1 && threadIdx.x < 64) {
      // every thread of this workgroup is past its reads of the diagonal block (the LU consumed
      // them before the barrier); count this workgroup and store the block if it is the last.
      // Relaxed: the only order needed is each workgroup's reads (complete, their values used
      // before the barrier) before the last one's stores (issued only after the count returned),
      // and no data passes through the counter -- an acquire/release here would write back and
      // invalidate the whole L2 around every increment.
      int prev = 0;
      if (threadIdx.x == 0)
        prev = __hip_atomic_fetch_add(arrive + d.f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      prev = __builtin_amdgcn_readlane(prev, 0);
      if (prev == nact - 1) {
        store_diag_block<NB>(d, store, D, threadIdx.x);
        if (threadIdx.x == 0)
          __hip_atomic_store(arrive + d.f, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
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

}  // namespace mf
