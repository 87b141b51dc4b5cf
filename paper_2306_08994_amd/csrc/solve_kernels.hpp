// solve_kernels.hpp -- gfx950 kernels of the substitution sweeps over the elimination tree, and
// the element-by-element operators (residual, adjoint element gradient).
//
// A = L U in elimination order (L carries the pivots, U has a unit diagonal).  The down sweep
// runs classes 0..H and the up sweep classes H..0 (leaves to root, then root to leaves).
//   down, TRANS=0: L y = b    y_p = w_p / L_pp,  w_i -= L_ip y_p        (i > p)
// (the division by a pivot is applied as a multiplication by its reciprocal, computed once)
//   down, TRANS=1: U^T z = g  z_p = w_p,         w_j -= U_pj z_p        (j > p)
//   up,   TRANS=0: U x = y    x_p = w_p,         w_q -= U_qp x_p        (q < p)
//   up,   TRANS=1: L^T l = z  l_p = w_p / L_pp,  w_q -= L_pq l_p        (q < p)
// A front's right-hand-side block W (m x nc columns, in LDS) starts, in the down sweep, as b on
// its pivots plus its children's contribution blocks (extend-add, like the factor); its own
// contribution block (rows k..m-1) goes to `ycb` for its parent, and its pivots' values to x.
// In the up sweep W holds the down-sweep values on the pivots and final values on the CB rows
// (pivots of ancestors); the CB part is applied first, then the pivots in reverse order.
// Coefficient accessors on the front storage F (m x m row-major):
//   down: cd(i, p) = TRANS ? U_pi = F[p][i] : L_ip = F[i][p];  diag TRANS ? 1 : F[p][p]
//   up:   cu(q, p) = TRANS ? L_pq = F[p][q] : U_qp = F[q][p];  diag TRANS ? F[p][p] : 1
#pragma once

#include "common.hpp"

namespace mf {

// ---------------------------------------------------------------------------------------------
// One wave per front (fronts of width <= 64), four fronts per workgroup.  Lane i owns row i of
// the front for every global access (coefficients, gathers, results), so each lane issues its
// loads back to back; pivots are eliminated one at a time in LDS with wave-level ordering.
// LDS per wave: ldsw doubles = W (mmax x nc) + coefficients (cdoubles) + reciprocals (64).
// ---------------------------------------------------------------------------------------------
constexpr int kWaveRows = 64;

// Loads n values v[u] = src[u * stride], u < n, eight independent loads at a time, into
// dst[u * dstride] (LDS).
// Right-hand-side columns gathered per batch: the loads of a batch are issued together before
// any of them is used (a loop of load-then-store waits for every load in turn).
constexpr int kRhsBatch = 8;

__device__ inline void copy_strided(const double *__restrict__ src, int64_t stride, int n,
                                    double *dst, int dstride) {
  for (int u0 = 0; u0 < n; u0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = u0 + u < n ? src[(int64_t)(u0 + u) * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (u0 + u < n) dst[(u0 + u) * dstride] = v[u];
  }
}

// The down sweep of one front by one wave: W (mmax x nc), C (mmax rows of cld) and rdv (64)
// are the wave's LDS.
template <bool TRANS>
__device__ __forceinline__ void down_wave_front(const WaveRec d, int lane, double *W, double *C,
                                                double *rdv, const double *store,
                                                const int32_t *front_idx, const int32_t *inv_l,
                                                const int32_t *inv_r, const double *b, double *x,
                                                double *ycb, int nrhs, int nc, int cld) {
  const int m = d.m, k = d.k;
  const double *F = store + d.store;
  // children that pass a contribution block (a pass-through leaf passes none)
  const bool use_a = d.ycb[0] >= 0, use_c = d.ycb[1] >= 0;
  const int i = lane;                               // this lane's row
  int64_t gi = 0;
  int xa = -1, xc = -1;
  if (i < m) {
    gi = front_idx[d.idx + i];
    if (use_a) xa = inv_l[d.idx + i];
    if (use_c) xc = inv_r[d.idx + i];
    const int np = min(i + 1, k);
    if (TRANS)
      copy_strided(F + i, m, np, C + i * cld, 1);            // U[p][i], p <= i
    else
      copy_strided(F + (int64_t)i * m, 1, np, C + i * cld, 1);   // L[i][p], p <= i
  }
  wave_sync();
  if (i < k) rdv[i] = TRANS ? 1.0 : 1.0 / C[i * cld + i];
  for (int r0 = 0; r0 < nrhs; r0 += nc) {
    const int nr = min(nc, nrhs - r0);
    if (i < m)
      for (int rb = 0; rb < nr; rb += kRhsBatch) {     // loads of a batch in flight together
        double v[kRhsBatch];
#pragma unroll
        for (int u = 0; u < kRhsBatch; ++u) {
          const int r = rb + u;
          v[u] = 0.0;
          if (r < nr) {
            if (i < k) v[u] = b[gi * nrhs + r0 + r];
            if (xa >= 0) v[u] += ycb[(d.ycb[0] + xa) * nrhs + r0 + r];
            if (xc >= 0) v[u] += ycb[(d.ycb[1] + xc) * nrhs + r0 + r];
          }
        }
#pragma unroll
        for (int u = 0; u < kRhsBatch; ++u)
          if (rb + u < nr) W[i * nr + rb + u] = v[u];
      }
    wave_sync();
    // lane (la, lr): right-hand sides lr, lr + 64, ... of the rows la, la + rs, ... (rs rows
    // per pass; one row and several sides per lane when nr >= 64)
    const int rs = nr >= 64 ? 1 : 64 / nr, la = nr >= 64 ? 0 : lane / nr, lr = lane - la * nr;
    const bool act = la < rs;
    for (int p = 0; p < k; ++p) {
      if (act)
        for (int c = lr; c < nr; c += 64) {
          const double wp = W[p * nr + c] * rdv[p];
          for (int ii = p + 1 + la; ii < m; ii += rs) W[ii * nr + c] -= C[ii * cld + p] * wp;
        }
      wave_sync();
    }
    // pivot rows: y = w / L_pp (row p is final after step p); CB rows: the contribution block
    if (i < k)
      for (int r = 0; r < nr; ++r) x[gi * nrhs + r0 + r] = W[i * nr + r] * rdv[i];
    else if (i < m)
      for (int r = 0; r < nr; ++r) ycb[(d.cbrow + i - k) * nrhs + r0 + r] = W[i * nr + r];
    wave_sync();
  }
}

// The up sweep of one front by one wave (LDS as in down_wave_front; C column-major here).
template <bool TRANS>
__device__ __forceinline__ void up_wave_front(const WaveRec d, int lane, double *W, double *C,
                                              double *rdv, const double *store,
                                              const int32_t *front_idx, double *x, int nrhs,
                                              int nc, int cld) {
  const int m = d.m, k = d.k;
  const double *F = store + d.store;
  const int j = lane;                               // this lane's row / column
  int64_t gj = 0;
  if (j < m) {
    gj = front_idx[d.idx + j];
    const int nq = min(j + 1, k);
    if (TRANS)
      copy_strided(F + (int64_t)j * m, 1, nq, C + j * cld, 1);   // L[j][q], q <= j
    else
      copy_strided(F + j, m, nq, C + j * cld, 1);                // U[q][j], q <= j
  }
  wave_sync();
  if (j < k) rdv[j] = TRANS ? 1.0 / C[j * cld + j] : 1.0;
  for (int r0 = 0; r0 < nrhs; r0 += nc) {
    const int nr = min(nc, nrhs - r0);
    if (j < m)
      for (int rb = 0; rb < nr; rb += kRhsBatch) {
        double v[kRhsBatch];
#pragma unroll
        for (int u = 0; u < kRhsBatch; ++u) v[u] = rb + u < nr ? x[gj * nrhs + r0 + rb + u] : 0.0;
#pragma unroll
        for (int u = 0; u < kRhsBatch; ++u)
          if (rb + u < nr) W[j * nr + rb + u] = v[u];
      }
    wave_sync();
    // lane (la, lr): right-hand sides lr, lr + 64, ... of the rows la, la + rs, ... (rs rows
    // per pass; one row and several sides per lane when nr >= 64)
    const int rs = nr >= 64 ? 1 : 64 / nr, la = nr >= 64 ? 0 : lane / nr, lr = lane - la * nr;
    const bool act = la < rs;
    // the already-final CB unknowns applied to the pivot rows
    if (act)
      for (int p = la; p < k; p += rs)
        for (int c = lr; c < nr; c += 64) {
          double s = 0.0;
          for (int jj = k; jj < m; ++jj) s += C[jj * cld + p] * W[jj * nr + c];
          W[p * nr + c] -= s;
        }
    wave_sync();
    for (int p = k - 1; p >= 0; --p) {
      if (act)
        for (int c = lr; c < nr; c += 64) {
          const double wp = W[p * nr + c] * rdv[p];
          for (int q = la; q < p; q += rs) W[q * nr + c] -= C[p * cld + q] * wp;
        }
      wave_sync();
    }
    if (j < k)
      for (int r = 0; r < nr; ++r) x[gj * nrhs + r0 + r] = W[j * nr + r] * rdv[j];
    wave_sync();
  }
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_down_wave(const WaveRec *__restrict__ recs, int nrec,
                  const double *__restrict__ store, const int32_t *__restrict__ front_idx,
                  const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
                  const double *b, double *x, double *__restrict__ ycb, int nrhs, int nc,
                  int mmax, int cld, int ldsw) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  double *W = sm + wv * ldsw;
  double *C = W + mmax * nc;       // C[i * cld + p] = cd(i, p), p <= i, p < k
  double *rdv = C + mmax * cld;    // reciprocal of each pivot's diagonal coefficient
  for (int li = blockIdx.x * 4 + wv; li < nrec; li += gridDim.x * 4)
    down_wave_front<TRANS>(recs[li], lane, W, C, rdv, store, front_idx, inv_l, inv_r, b, x, ycb,
                           nrhs, nc, cld);
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_up_wave(const WaveRec *__restrict__ recs, int nrec,
                const double *__restrict__ store, const int32_t *__restrict__ front_idx,
                double *x, int nrhs, int nc, int mmax, int cld, int ldsw) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  double *W = sm + wv * ldsw;
  double *C = W + mmax * nc;       // C[j * cld + q] = cu(q, j), q <= j, q < k  (column-major)
  double *rdv = C + mmax * cld;
  for (int li = blockIdx.x * 4 + wv; li < nrec; li += gridDim.x * 4)
    up_wave_front<TRANS>(recs[li], lane, W, C, rdv, store, front_idx, x, nrhs, nc, cld);
}

// ---------------------------------------------------------------------------------------------
// Bottom subtrees of the wave route in one launch per sweep (units and record order as for
// k_factor_subtree): the down sweep takes a unit's classes 0..ncls-1 in turn, the up sweep
// ncls-1..0, one front per wave, a workgroup barrier between classes.  The contribution blocks
// a front gathers (down) and the ancestor values it reads (up) were written by this workgroup
// before the barrier or by an earlier launch.  Per front the wave route's arithmetic, so the
// results are identical to the per-class launches.
// ---------------------------------------------------------------------------------------------
template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_down_subtree(const WaveRec *__restrict__ recs, const int32_t *__restrict__ ptr,
                     int nsub, int ncls, const double *__restrict__ store,
                     const int32_t *__restrict__ front_idx, const int32_t *__restrict__ inv_l,
                     const int32_t *__restrict__ inv_r, const double *b, double *x, double *ycb,
                     int nrhs, int nc, int mmax, int cld, int ldsw) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *W = sm + wv * ldsw;
  double *C = W + mmax * nc;
  double *rdv = C + mmax * cld;
  for (int u = blockIdx.x; u < nsub; u += gridDim.x) {
    const int32_t *pu = ptr + (int64_t)u * ncls;
    for (int c = 0; c < ncls; ++c) {
      const int a = pu[c], e = pu[c + 1];
      for (int li = a + wv; li < e; li += 4)
        down_wave_front<TRANS>(recs[li], lane, W, C, rdv, store, front_idx, inv_l, inv_r, b, x,
                               ycb, nrhs, nc, cld);
      __syncthreads();   // the class's contribution blocks written before the next class
    }
  }
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_solve_up_subtree(const WaveRec *__restrict__ recs, const int32_t *__restrict__ ptr, int nsub,
                   int ncls, const double *__restrict__ store,
                   const int32_t *__restrict__ front_idx, double *x, int nrhs, int nc, int mmax,
                   int cld, int ldsw) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *W = sm + wv * ldsw;
  double *C = W + mmax * nc;
  double *rdv = C + mmax * cld;
  for (int u = blockIdx.x; u < nsub; u += gridDim.x) {
    const int32_t *pu = ptr + (int64_t)u * ncls;
    for (int c = ncls - 1; c >= 0; --c) {
      const int a = pu[c], e = pu[c + 1];
      for (int li = a + wv; li < e; li += 4)
        up_wave_front<TRANS>(recs[li], lane, W, C, rdv, store, front_idx, x, nrhs, nc, cld);
      __syncthreads();   // the class's values written before its children read them
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Inverses of the NBS x NBS diagonal blocks of L and U of every front that the block solves
// handle, computed once after the factorization, so that a block solve applies a diagonal block
// as one matrix-vector product instead of NBS dependent substitution steps.  For a front f with
// k > 0, dinv + dinv_off[f] holds ceil(k / NBS) pairs of NBS x NBS row-major blocks: inv(L_BB)
// (lower, pivots on the diagonal), then inv(U_BB) (unit upper); a ragged last block is padded
// with the identity.  A workgroup takes four (front, block) tasks at a time: each wave stages
// one block in LDS, then the even waves form the columns of inv(L_BB) by forward substitution
// and the odd waves those of inv(U_BB) by back substitution, NBS lanes per block (two blocks
// per wave), each column in registers.
// ---------------------------------------------------------------------------------------------
constexpr int NBS = 32;
static_assert(2 * NBS == 64, "one wave forms both inverses of a block");

__global__ void __launch_bounds__(256)
k_diag_inverse(const FrontDesc *__restrict__ fd, const int2 *__restrict__ tasks, int ntasks,
               const double *__restrict__ store, const int64_t *__restrict__ dinv_off,
               double *__restrict__ dinv) {
  __shared__ double Bs[4][NBS][NBS + 1];
  __shared__ double Rs[4][NBS];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  // the task this lane substitutes for (of the group's four): waves 0, 1 take tasks 0 and 1
  // (lanes 0..NBS-1, NBS..2NBS-1), waves 2, 3 tasks 2 and 3; even waves form inv(L), odd waves
  // inv(U), so no wave runs both substitutions one after the other.  LDS bases in vector
  // registers (threadIdx-derived): every block entry is an immediate offset from them.
  const int tl = ((threadIdx.x >> 6) & ~1) + (lane >> 5);
  const bool upper = wv & 1;
  double(*Bw)[NBS + 1] = Bs[threadIdx.x >> 6];
  double(*B)[NBS + 1] = Bs[tl];
  const double *rdg = Rs[tl];
  const int j = lane & (NBS - 1);
  static_assert(2 * NBS == 64, "two blocks per wave");
  for (int g0 = blockIdx.x * 4; g0 < ntasks; g0 += gridDim.x * 4) {   // uniform
    // wave w stages task g0 + w: the block's 16 entries per lane loaded together, then stored
    if (g0 + wv < ntasks) {
      const int2 tk = tasks[g0 + wv];
      const FrontDesc d = fd[tk.x];
      const int p0 = tk.y, pb = min(NBS, d.k - p0);
      const double *F = store + d.store + (int64_t)p0 * d.m + p0;
      double v[NBS * NBS / 64];
#pragma unroll
      for (int u = 0; u < NBS * NBS / 64; ++u) {
        const int e = lane + 64 * u, i = e / NBS, c = e % NBS;
        v[u] = (i < pb && c < pb) ? F[(int64_t)i * d.m + c] : (i == c ? 1.0 : 0.0);
      }
#pragma unroll
      for (int u = 0; u < NBS * NBS / 64; ++u) {
        const int e = lane + 64 * u;
        Bw[e / NBS][e % NBS] = v[u];
      }
      wave_sync();
      if (lane < NBS) Rs[wv][lane] = 1.0 / Bw[lane][lane];   // the pivots' reciprocals
    }
    __syncthreads();
    const bool act = g0 + tl < ntasks;
    int2 tko = make_int2(0, 0);
    int64_t off = 0;
    if (act) {
      tko = tasks[g0 + tl];
      off = dinv_off[tko.x];
    }
    // substitutions with two partial sums per row (half the dependent chain of one sum); each
    // row of the block is read from LDS into registers as a whole (its reads issued together)
    // before its products, so a row costs one LDS round trip rather than one per entry
    double z[NBS];
    double br[NBS];
    if (!upper) {
#pragma unroll
      for (int i = 0; i < NBS; ++i) {          // L z = e_j
#pragma unroll
        for (int p = 0; p < i; ++p) br[p] = B[i][p];
        __builtin_amdgcn_sched_barrier(0);     // the row's reads are issued before its products
        double s0 = (i == j) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int p = 0; p + 1 < i; p += 2) {
          s0 -= br[p] * z[p];
          s1 -= br[p + 1] * z[p + 1];
        }
        if (i & 1) s0 -= br[i - 1] * z[i - 1];
        z[i] = (s0 + s1) * rdg[i];
      }
    } else {
#pragma unroll
      for (int i = NBS - 1; i >= 0; --i) {     // U z = e_j, unit diagonal
#pragma unroll
        for (int p = i + 1; p < NBS; ++p) br[p] = B[i][p];
        __builtin_amdgcn_sched_barrier(0);
        double s0 = (i == j) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int p = i + 1; p + 1 < NBS; p += 2) {
          s0 -= br[p] * z[p];
          s1 -= br[p + 1] * z[p + 1];
        }
        if ((NBS - 1 - i) & 1) s0 -= br[NBS - 1] * z[NBS - 1];
        z[i] = s0 + s1;
      }
    }
    if (act) {
      double *out = dinv + off + (int64_t)(tko.y / NBS) * 2 * NBS * NBS + (upper ? NBS * NBS : 0);
#pragma unroll
      for (int i = 0; i < NBS; ++i) out[i * NBS + j] = z[i];
    }
    __syncthreads();                           // the blocks are restaged by the next group
  }
}

// ---------------------------------------------------------------------------------------------
// One workgroup per front (fronts wider than the wave route), pivots in blocks of NBS.  Per
// block: the inverse of the diagonal block (staged in LDS) gives the block's unknowns in one
// matrix-vector product, thread (q, r) forming row q for right-hand side r; then the remaining
// rows take the block's contribution.  Coefficients of the remaining rows are read in tiles of
// kTileRows x NBS, each tile loaded cooperatively so that the lanes of a load run along
// contiguous memory (along a row of F without TRANS, along a column with TRANS), staged in LDS
// and applied row per thread; the next tile (and the next block's inverse and first tile) is
// loaded while the current one is applied.
// Inner loops run over all NBS positions without bound checks: loads clamp their index into the
// front (a clamped value only ever meets a zero), W carries NBS zero rows after row m-1, the
// inverse of a ragged block is identity-padded and Y's unused rows are zero.
// LDS, right-hand side major (a column r of W is contiguous, so block offsets are immediates):
// W (nc columns of ldw >= m + NBS, ldw odd) | M (NBS x NBS+1, the block inverse) |
// T (kTileRows x NBS+1 coefficient tile) | Y (nc x NBS).
// ---------------------------------------------------------------------------------------------
constexpr int kTileRows = 128;
constexpr int kTileLoads = kTileRows * NBS / 256;
__host__ __device__ constexpr int block_solve_fixed_doubles() {
  return NBS * (NBS + 1) + kTileRows * (NBS + 1);
}
// doubles of LDS per right-hand-side column for up to rmax rows of W: W column + Y column
__host__ __device__ constexpr int block_solve_col_doubles(int rmax) { return ((rmax + NBS) | 1) + NBS; }

constexpr int kInvPerThread = NBS * NBS / 256;

// The inverse a sweep applies for the diagonal block starting at pivot p0, read in memory order
// (coalesced): down: TRANS ? inv(U)^T : inv(L); up: TRANS ? inv(L)^T : inv(U).
template <bool TRANS, bool UP>
__device__ inline void load_block_inverse(const double *dv, int p0, int tid, double *v) {
  const double *M = dv + (int64_t)(p0 / NBS) * 2 * NBS * NBS + ((UP != TRANS) ? NBS * NBS : 0);
#pragma unroll
  for (int u = 0; u < kInvPerThread; ++u) v[u] = M[tid + 256 * u];
}
// ... and stored into LDS as Ms[q][p] = entry (q, p) of the applied matrix.
template <bool TRANS>
__device__ inline void store_block_inverse(const double *v, int tid, double *Ms) {
#pragma unroll
  for (int u = 0; u < kInvPerThread; ++u) {
    const int e = tid + 256 * u, a = e / NBS, c = e % NBS;
    if (TRANS)
      Ms[c * (NBS + 1) + a] = v[u];
    else
      Ms[a * (NBS + 1) + c] = v[u];
  }
}

// Tile element u of this thread: row i (of kTileRows) and column p (of NBS).  Without TRANS a
// load's lanes run along a row (32 consecutive columns), with TRANS along the rows.
template <bool TRANS>
__device__ inline void tile_pos(int tid, int u, int &i, int &p) {
  const int e = tid + 256 * u;
  if (TRANS) {
    i = e % kTileRows;
    p = e / kTileRows;
  } else {
    i = e / NBS;
    p = e % NBS;
  }
}

// Coefficients C(rb + i, c0 + p) of either sweep (cd and cu are the same access:
// TRANS ? F[col][row] : F[row][col]), rows clamped below r_hi and columns below m.
template <bool TRANS>
__device__ inline void tile_load(const double *F, int m, int rb, int r_hi, int c0, int tid,
                                 double *v) {
#pragma unroll
  for (int u = 0; u < kTileLoads; ++u) {
    int i, p;
    tile_pos<TRANS>(tid, u, i, p);
    const int row = min(rb + i, r_hi - 1), col = min(c0 + p, m - 1);
    v[u] = TRANS ? F[(int64_t)col * m + row] : F[(int64_t)row * m + col];
  }
}
template <bool TRANS>
__device__ inline void tile_store(const double *v, int tid, double *T) {
#pragma unroll
  for (int u = 0; u < kTileLoads; ++u) {
    int i, p;
    tile_pos<TRANS>(tid, u, i, p);
    T[i * (NBS + 1) + p] = v[u];
  }
}

// W[r][rb + i] -= sum_p T[i][p] X[r][p] for the kTileRows rows of a staged tile (rows at or
// beyond r_hi skipped) and the nr right-hand sides, on the matrix cores: wave w takes rows
// 32 w.. as two 16-row blocks, right-hand sides in blocks of 16 (v_mfma_f64_16x16x4f64: A lane
// l = row l%16, k l/16; B lane l = column l%16, k l/16; result lane l, register r = row
// 4r + l/16, column l%16).
__device__ inline void tile_apply_mfma(const double *T, const double *X, int ldx, double *W,
                                       int ldw, int rb, int r_hi, int nr, int tid) {
  static_assert(kTileRows == 128 && NBS % 4 == 0, "four waves of 32 rows");
  const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  for (int cb = 0; cb < nr; cb += 16) {
    v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    const int col = cb + li;
    // every operand of the block's products read from LDS first (reads issued together), then
    // the dependent MFMA chain -- not one LDS round trip per product
    double bv[NBS / 4], av[2][NBS / 4];
#pragma unroll
    for (int s = 0; s < NBS / 4; ++s) {
      bv[s] = col < nr ? X[col * ldx + 4 * s + lk] : 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a][s] = T[(32 * wv + 16 * a + li) * (NBS + 1) + 4 * s + lk];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < NBS / 4; ++s)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][s], bv[s], acc[a], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + 32 * wv + 16 * a + 4 * r + lk;
        if (row < r_hi && col < nr) W[col * ldw + row] -= acc[a][r];
      }
  }
}

// W[r][row] -= sum_p C(row, c0 + p) X[r][p] for rows [r_lo, r_hi) and column blocks c0 in
// [c_lo, c_hi) (step NBS), X of block c0 at xf(c0) with column stride ldx.  `pre` holds the
// first tile (r_lo, c_lo), loaded by the caller.  Ends with a barrier.
template <bool TRANS, typename XF>
__device__ inline void rect_update(const double *F, int m, int r_lo, int r_hi, int c_lo, int c_hi,
                                   XF xf, int ldx, double *W, int ldw, int nr, double *T,
                                   int tid, double *pre) {
  for (int c0 = c_lo; c0 < c_hi; c0 += NBS) {
    const double *X = xf(c0);
    for (int rb = r_lo; rb < r_hi; rb += kTileRows) {
      tile_store<TRANS>(pre, tid, T);
      int nrb = rb + kTileRows, nc0 = c0;
      if (nrb >= r_hi) {
        nrb = r_lo;
        nc0 = c0 + NBS;
      }
      if (nc0 < c_hi) tile_load<TRANS>(F, m, nrb, r_hi, nc0, tid, pre);
      __syncthreads();
      tile_apply_mfma(T, X, ldx, W, ldw, rb, r_hi, nr, tid);
      __syncthreads();
    }
  }
}

// Y[r][q] = sum_p M[q][p] W[r][p0 + p] for q < pb, 0 for pb <= q < NBS, on the matrix cores:
// (wave, 16-column block) pairs over the two 16-row blocks of M and the nr right-hand sides.
__device__ inline void block_matvec(const double *Ms, const double *W, int ldw, double *Y, int p0,
                                    int pb, int nr, int tid) {
  const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int a = wv & 1;                      // row block of M
  for (int cb = 16 * (wv >> 1); cb < nr; cb += 32) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    const int col = cb + li;
    double bv[NBS / 4], av[NBS / 4];          // operands first, then the MFMA chain
#pragma unroll
    for (int s = 0; s < NBS / 4; ++s) {
      bv[s] = col < nr ? W[col * ldw + p0 + 4 * s + lk] : 0.0;
      av[s] = Ms[(16 * a + li) * (NBS + 1) + 4 * s + lk];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < NBS / 4; ++s)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 16 * a + 4 * r + lk;
      if (col < nr) Y[col * NBS + q] = q < pb ? acc[r] : 0.0;
    }
  }
}

// FULL = true: the whole front in one workgroup (rows [0, m): the pivots' triangle, then the
// contribution rows in the same block loop; up: the contribution columns applied first).
// FULL = false: the pivots' triangle only; the rectangular part runs in k_solve_rect (after
// this kernel in the down sweep, before it in the up sweep).
template <bool TRANS, bool FULL>
__global__ void __launch_bounds__(256)
k_solve_down_block(const WaveRec *__restrict__ recs, int nrec,
                   const double *__restrict__ store, const int32_t *__restrict__ front_idx,
                   const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
                   const double *b, double *x, double *__restrict__ ycb, int nrhs, int nc,
                   int rmax, const double *__restrict__ dinv) {
  extern __shared__ double sm[];
  const int ldw = (rmax + NBS) | 1;
  double *W = sm;
  double *Ms = W + ldw * nc;
  double *T = Ms + NBS * (NBS + 1);
  double *Y = T + kTileRows * (NBS + 1);
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nrec; li += gridDim.x) {
    const WaveRec d = recs[li];
    const int m = d.m, k = d.k;
    const int rows = FULL ? m : k;          // rows this kernel solves for
    if (rows == 0) continue;
    const int32_t *idx = front_idx + d.idx;
    const int32_t *il = inv_l + d.idx;
    const int32_t *ir = inv_r + d.idx;
    const double *F = store + d.store;
    const double *dv = k > 0 ? dinv + d.dinv : nullptr;
    // children that pass a contribution block (a pass-through leaf passes none)
    const bool use_a = d.ycb[0] >= 0, use_c = d.ycb[1] >= 0;
    for (int r0 = 0; r0 < nrhs; r0 += nc) {
      const int nr = min(nc, nrhs - r0);
      double mv[kInvPerThread], pre[kTileLoads];
      if (k > 0) {
        load_block_inverse<TRANS, false>(dv, 0, tid, mv);
        const int pe = min(NBS, k);
        if (pe < rows) tile_load<TRANS>(F, m, pe, rows, 0, tid, pre);
      }
      for (int i = tid; i < rows; i += 256) {
        const int64_t gi = idx[i];
        const int x0 = use_a ? il[i] : -1, y0 = use_c ? ir[i] : -1;
        for (int rb = 0; rb < nr; rb += kRhsBatch) {     // loads of a batch in flight together
          double v[kRhsBatch];
#pragma unroll
          for (int u = 0; u < kRhsBatch; ++u) {
            const int r = rb + u;
            v[u] = 0.0;
            if (r < nr) {
              if (i < k) v[u] = b[gi * nrhs + r0 + r];
              if (x0 >= 0) v[u] += ycb[(d.ycb[0] + x0) * nrhs + r0 + r];
              if (y0 >= 0) v[u] += ycb[(d.ycb[1] + y0) * nrhs + r0 + r];
            }
          }
#pragma unroll
          for (int u = 0; u < kRhsBatch; ++u)
            if (rb + u < nr) W[(rb + u) * ldw + i] = v[u];
        }
      }
      for (int t = tid; t < NBS * nr; t += 256) W[(t / NBS) * ldw + rows + t % NBS] = 0.0;
      if (k > 0) store_block_inverse<TRANS>(mv, tid, Ms);
      for (int p0 = 0; p0 < k; p0 += NBS) {
        const int pb = min(NBS, k - p0), pe = p0 + pb;
        __syncthreads();            // rows p0.. of W final, Ms holds this block's inverse
        block_matvec(Ms, W, ldw, Y, p0, pb, nr, tid);
        const bool more = pe < k;
        if (more) load_block_inverse<TRANS, false>(dv, pe, tid, mv);
        __syncthreads();            // Y complete, every read of Ms and of rows p0..pe-1 done
        for (int t = tid; t < pb * nr; t += 256) {
          const int r = t / pb, q = t - (t / pb) * pb;
          W[r * ldw + p0 + q] = Y[r * NBS + q];
        }
        if (pe < rows)
          rect_update<TRANS>(F, m, pe, rows, p0, p0 + 1, [&](int) { return (const double *)Y; },
                             NBS, W, ldw, nr, T, tid, pre);
        if (more) {
          store_block_inverse<TRANS>(mv, tid, Ms);
          const int pen = pe + min(NBS, k - pe);
          if (pen < rows) tile_load<TRANS>(F, m, pen, rows, pe, tid, pre);
        }
      }
      __syncthreads();
      for (int i = tid; i < rows; i += 256) {
        if (i < k) {
          const int64_t gi = idx[i];
          for (int r = 0; r < nr; ++r) x[gi * nrhs + r0 + r] = W[r * ldw + i];
        } else {
          for (int r = 0; r < nr; ++r) ycb[(d.cbrow + i - k) * nrhs + r0 + r] = W[r * ldw + i];
        }
      }
      __syncthreads();
    }
  }
}

template <bool TRANS, bool FULL>
__global__ void __launch_bounds__(256)
k_solve_up_block(const WaveRec *__restrict__ recs, int nrec,
                 const double *__restrict__ store, const int32_t *__restrict__ front_idx,
                 double *x, int nrhs, int nc, int rmax, const double *__restrict__ dinv) {
  extern __shared__ double sm[];
  const int ldw = (rmax + NBS) | 1;
  double *W = sm;
  double *Ms = W + ldw * nc;
  double *T = Ms + NBS * (NBS + 1);
  double *Y = T + kTileRows * (NBS + 1);
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nrec; li += gridDim.x) {
    const WaveRec d = recs[li];
    const int m = d.m, k = d.k;
    if (k == 0) continue;
    const int rows = FULL ? m : k;          // rows of W: the pivots (+ the CB values if FULL)
    const int32_t *idx = front_idx + d.idx;
    const double *F = store + d.store;
    const double *dv = dinv + d.dinv;
    const int plast = ((k - 1) / NBS) * NBS;
    const bool cb = FULL && k < m;
    for (int r0 = 0; r0 < nrhs; r0 += nc) {
      const int nr = min(nc, nrhs - r0);
      double mv[kInvPerThread], pre[kTileLoads];
      load_block_inverse<TRANS, true>(dv, plast, tid, mv);
      if (cb)
        tile_load<TRANS>(F, m, 0, k, k, tid, pre);
      else if (plast > 0)
        tile_load<TRANS>(F, m, 0, plast, plast, tid, pre);
      for (int i = tid; i < rows; i += 256) {
        const int64_t gi = idx[i];
        for (int rb = 0; rb < nr; rb += kRhsBatch) {
          double v[kRhsBatch];
#pragma unroll
          for (int u = 0; u < kRhsBatch; ++u) v[u] = rb + u < nr ? x[gi * nrhs + r0 + rb + u] : 0.0;
#pragma unroll
          for (int u = 0; u < kRhsBatch; ++u)
            if (rb + u < nr) W[(rb + u) * ldw + i] = v[u];
        }
      }
      for (int t = tid; t < NBS * nr; t += 256) W[(t / NBS) * ldw + rows + t % NBS] = 0.0;
      if (cb) {
        // the already-final CB unknowns applied to the pivot rows (columns beyond m meet W's
        // zero rows)
        rect_update<TRANS>(F, m, 0, k, k, m, [&](int c0) { return (const double *)(W + c0); },
                           ldw, W, ldw, nr, T, tid, pre);
        if (plast > 0) tile_load<TRANS>(F, m, 0, plast, plast, tid, pre);
      }
      store_block_inverse<TRANS>(mv, tid, Ms);
      for (int p0 = plast; p0 >= 0; p0 -= NBS) {
        const int pb = min(NBS, k - p0);
        __syncthreads();            // rows p0.. of W final, Ms holds this block's inverse
        block_matvec(Ms, W, ldw, Y, p0, pb, nr, tid);
        const bool more = p0 > 0;
        if (more) load_block_inverse<TRANS, true>(dv, p0 - NBS, tid, mv);
        __syncthreads();            // Y complete, every read of Ms and of rows p0.. done
        for (int t = tid; t < pb * nr; t += 256) {
          const int r = t / pb, q = t - (t / pb) * pb;
          W[r * ldw + p0 + q] = Y[r * NBS + q];
        }
        if (more) {
          rect_update<TRANS>(F, m, 0, p0, p0, p0 + 1, [&](int) { return (const double *)Y; },
                             NBS, W, ldw, nr, T, tid, pre);
          store_block_inverse<TRANS>(mv, tid, Ms);
          if (p0 - NBS > 0) tile_load<TRANS>(F, m, 0, p0 - NBS, p0 - NBS, tid, pre);
        }
      }
      __syncthreads();
      for (int p = tid; p < k; p += 256) {
        const int64_t gp = idx[p];
        for (int r = 0; r < nr; ++r) x[gp * nrhs + r0 + r] = W[r * ldw + p];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Chunked triangle solves (no transposition) of fronts with many pivots.  The one-workgroup
// block solve walks a front's whole triangle of L or U, k^2/2 coefficients through one CU (the
// 1,089-pivot root of the 3D workload: 4.7 MB, over 300 us per sweep).  Here the triangle is
// cut into chunks of kChunkPiv pivots (see chunk_pivots), one launch per chunk, one workgroup per 128-row tile of
// the pivot rows the chunk updates (below it in the down sweep, above it in the up sweep) and
// one "writer" workgroup per front: every workgroup solves the chunk's own small triangle
// redundantly from its diagonal-block inverses, then the tile workgroups apply the chunk's
// columns to their rows.  The pivot rows' right-hand sides live between launches in a
// workspace (row wrow + i of the front's pivot i, nrhs values per row), staged by
// k_solve_chunk_stage from b and the children's contribution blocks (down) or from x (up); a
// launch reads chunk and tile rows of the workspace and writes only its tile rows there and
// the chunk's solution into x, so no workgroup reads what another writes in the same launch.
// Task (int4): wave record, first pivot of the chunk, first row of the tile (-1: the writer),
// the front's first workspace row.
// ---------------------------------------------------------------------------------------------
constexpr int kChunkPiv = 4 * NBS;
constexpr int kChunkMax = kChunkPiv + NBS;       // a remainder of up to NBS joins the last chunk
constexpr int kChunkRows = kChunkMax + kTileRows + NBS;     // LDS rows: chunk, tile, zero rows
constexpr int kChunkLd = kChunkRows | 1;
// Pivots of the chunk starting at p0 of a front with k pivots (chunks of kChunkPiv from 0, the
// last one taking a remainder of up to NBS more).
__host__ __device__ inline int chunk_pivots(int k, int p0) {
  return k - p0 <= kChunkMax ? k - p0 : kChunkPiv;
}
__host__ __device__ constexpr int chunk_solve_fixed_doubles() {
  return NBS * (NBS + 1) + 2 * kTileRows * (NBS + 1);
}
__host__ __device__ constexpr int chunk_solve_col_doubles() { return kChunkLd + NBS; }

// F[row][col] for rows rb.. (clamped below r_hi) and the NBS columns c0.. (clamped below c_hi),
// in the layout of tile_load<false>.
__device__ inline void ctile_load(const double *F, int m, int rb, int r_hi, int c0, int c_hi,
                                  int tid, double *v) {
#pragma unroll
  for (int u = 0; u < kTileLoads; ++u) {
    int i, p;
    tile_pos<false>(tid, u, i, p);
    const int row = min(rb + i, r_hi - 1), col = min(c0 + p, c_hi - 1);
    v[u] = F[(int64_t)row * m + col];
  }
}

// Stage the pivot rows [row0, row0 + rows) of a front into the workspace: down, b plus the
// children's contribution blocks; up, x.  Task (int4): wave record, row0, rows (<= 256), wrow.
template <bool UP>
__global__ void __launch_bounds__(256)
k_solve_chunk_stage(const WaveRec *__restrict__ recs, const int4 *__restrict__ tasks,
                    const int32_t *__restrict__ front_idx, const int32_t *__restrict__ inv_l,
                    const int32_t *__restrict__ inv_r, const double *b, const double *x,
                    const double *ycb, double *wsp, int nrhs) {
  const int4 tk = tasks[blockIdx.x];
  const WaveRec d = recs[tk.x];
  const int i = tk.y + (int)threadIdx.x;
  if ((int)threadIdx.x >= tk.z) return;
  const int64_t gi = front_idx[d.idx + i];
  const int xa = !UP && d.ycb[0] >= 0 ? inv_l[d.idx + i] : -1;
  const int xc = !UP && d.ycb[1] >= 0 ? inv_r[d.idx + i] : -1;
  double *out = wsp + ((int64_t)tk.w + i) * nrhs;
  for (int rb = 0; rb < nrhs; rb += kRhsBatch) {       // loads of a batch in flight together
    double v[kRhsBatch];
#pragma unroll
    for (int u = 0; u < kRhsBatch; ++u) {
      const int r = rb + u;
      v[u] = 0.0;
      if (r < nrhs) {
        if (UP) {
          v[u] = x[gi * nrhs + r];
        } else {
          v[u] = b[gi * nrhs + r];
          if (xa >= 0) v[u] += ycb[(d.ycb[0] + xa) * nrhs + r];
          if (xc >= 0) v[u] += ycb[(d.ycb[1] + xc) * nrhs + r];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kRhsBatch; ++u)
      if (rb + u < nrhs) out[rb + u] = v[u];
  }
}

// One chunk of a front (see above): W in LDS holds the chunk's rows [0, kChunkPiv), the tile's
// rows [kChunkPiv, kChunkPiv + kTileRows) and NBS zero rows, for nr right-hand sides.
template <bool UP>
__global__ void __launch_bounds__(256)
k_solve_chunk(const WaveRec *__restrict__ recs, const int4 *__restrict__ tasks,
              const double *__restrict__ store, const int32_t *__restrict__ front_idx, double *x,
              double *wsp, int nrhs, int nc, const double *__restrict__ dinv) {
  extern __shared__ double sm[];
  constexpr int PC = kChunkMax, ld = kChunkLd;
  double *W = sm;
  double *Ms = W + ld * nc;
  double *T1 = Ms + NBS * (NBS + 1);            // coefficients of the chunk rows a block updates
  double *T2 = T1 + kTileRows * (NBS + 1);      // ... and of the tile rows
  double *Y = T2 + kTileRows * (NBS + 1);
  const int tid = threadIdx.x;
  const int4 tk = tasks[blockIdx.x];
  const WaveRec d = recs[tk.x];
  const int m = d.m, k = d.k, p0 = tk.y, rt0 = tk.z;
  const int64_t wrow = tk.w;
  const int pc = chunk_pivots(k, p0);                    // the chunk's pivots
  const int tr = rt0 < 0 ? 0 : (UP ? min(kTileRows, p0 - rt0) : min(kTileRows, k - rt0));
  const double *F = store + d.store;
  const double *dv = dinv + d.dinv;
  const int nblk = (pc + NBS - 1) / NBS;
  // block bi of the chunk in processing order: first pivot (in the chunk), pivots, and the
  // chunk rows it updates (down: below it, up: above it)
  auto blk = [&](int bi, int &qb, int &pb, int &ulo, int &uhi) {
    qb = UP ? (nblk - 1 - bi) * NBS : bi * NBS;
    pb = min(NBS, pc - qb);
    ulo = UP ? 0 : qb + pb;
    uhi = UP ? qb : pc;
  };
  // the coefficients of a block (its inverse, its chunk-row and tile-row tiles) do not depend on
  // the values: block bi + 1's are loaded while block bi is applied
  double mv[kInvPerThread], cv[kTileLoads], tv[kTileLoads];
  auto load_blk = [&](int bi) {
    int qb, pb, ulo, uhi;
    blk(bi, qb, pb, ulo, uhi);
    load_block_inverse<false, UP>(dv, p0 + qb, tid, mv);
    if (uhi > ulo) ctile_load(F, m, p0 + ulo, p0 + uhi, p0 + qb, p0 + qb + pb, tid, cv);
    if (tr > 0) ctile_load(F, m, rt0, rt0 + tr, p0 + qb, p0 + qb + pb, tid, tv);
  };
  for (int r0 = 0; r0 < nrhs; r0 += nc) {
    const int nr = min(nc, nrhs - r0);
    load_blk(0);
    // chunk rows, tile rows, zeros (row index fastest: a constant divisor)
    for (int t0 = tid; t0 < kChunkRows * nr; t0 += 256 * kRhsBatch) {
      double v[kRhsBatch];
#pragma unroll
      for (int u = 0; u < kRhsBatch; ++u) {
        const int t = t0 + 256 * u, r = t / kChunkRows, i = t - r * kChunkRows;
        v[u] = 0.0;
        if (r < nr) {
          if (i < pc)
            v[u] = wsp[(wrow + p0 + i) * nrhs + r0 + r];
          else if (i >= PC && i < PC + tr)
            v[u] = wsp[(wrow + rt0 + i - PC) * nrhs + r0 + r];
        }
      }
#pragma unroll
      for (int u = 0; u < kRhsBatch; ++u) {
        const int t = t0 + 256 * u, r = t / kChunkRows, i = t - r * kChunkRows;
        if (r < nr) W[r * ld + i] = v[u];
      }
    }
    // the chunk's triangle block by block, each block's columns applied to the chunk rows and
    // the tile rows it updates right away
    for (int bi = 0; bi < nblk; ++bi) {
      int qb, pb, ulo, uhi;
      blk(bi, qb, pb, ulo, uhi);
      __syncthreads();            // W's rows of this block final; Ms, T1, T2, Y free
      store_block_inverse<false>(mv, tid, Ms);
      if (uhi > ulo) tile_store<false>(cv, tid, T1);
      if (tr > 0) tile_store<false>(tv, tid, T2);
      if (bi + 1 < nblk) load_blk(bi + 1);
      __syncthreads();
      block_matvec(Ms, W, ld, Y, qb, pb, nr, tid);
      __syncthreads();            // Y complete
      for (int t = tid; t < NBS * nr; t += 256) {
        const int r = t / NBS, q = t - (t / NBS) * NBS;
        W[r * ld + qb + q] = Y[r * NBS + q];                // zero beyond pb
      }
      if (uhi > ulo) tile_apply_mfma(T1, Y, NBS, W, ld, ulo, uhi, nr, tid);
      if (tr > 0) tile_apply_mfma(T2, Y, NBS, W, ld, PC, PC + tr, nr, tid);
    }
    __syncthreads();
    if (rt0 < 0) {
      const int32_t *idx = front_idx + d.idx + p0;
      for (int i = tid; i < pc; i += 256) {
        const int64_t gi = idx[i];
        for (int r = 0; r < nr; ++r) x[gi * nrhs + r0 + r] = W[r * ld + i];
      }
    } else {
      for (int i = tid; i < tr; i += 256)
        for (int r = 0; r < nr; ++r) wsp[(wrow + rt0 + i) * nrhs + r0 + r] = W[r * ld + PC + i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// The rectangular part of a wide front's sweep, off the front's sequential block path and
// spread over many workgroups:
//   down: the contribution-block rows i in [k, m):  ycb_i = w_i - sum_{p < k} cd(i, p) y_p
//         (w_i gathered from the children's contribution blocks, y_p = x[idx[p]] as the
//         triangle kernel of the same class left it);
//   up:   the pivot rows i in [0, k):  x[idx[i]] -= sum_{p in [k, m)} cu(i, p) x[idx[p]]
//         (before the triangle kernel of the class).
// cd and cu are the same access (TRANS ? F[p][i] : F[i][p]).  A task is a slab of up to 64
// output rows of one front; wave w takes 16 of them and computes them on the matrix cores
// (v_mfma_f64_16x16x4f64, right-hand sides as the 16 columns of B), each lane holding its
// A-operand coefficients of a group of kRectCols columns in registers, so all loads of a group
// are in flight at once; the input values of the group sit in LDS.  The values the result is
// combined with (children's contributions down, the pivots' values up) are loaded at the start.
// Right-hand sides in chunks of 16.  LDS: V (16 x kRectCols + 4).
// ---------------------------------------------------------------------------------------------
constexpr int kRectCols = 256;   // columns per group (64 MFMA steps of 4)
static_assert(kRectCols == 256, "one staged column per thread of the rectangular kernel");
constexpr int kRectRows = 64;    // output rows per task (4 waves x 16)
constexpr int kRectRowsQ = 16;   // output rows per task of the quarter form
constexpr int kRectLdv = kRectCols + 4;

// Q (quarter form, for classes with too few tasks of kRectRows to spread over the chip): a task
// is a slab of 16 rows, and wave w multiplies the w-th quarter (16 MFMA steps) of every column
// group; the four partial products are added in wave order through LDS (after V: 4 x 64 x 4
// doubles) and wave 0 stores.
template <bool TRANS, bool UP, bool Q = false>
__global__ void __launch_bounds__(256)
k_solve_rect(const WaveRec *__restrict__ recs, const int4 *__restrict__ tasks,
             const double *__restrict__ store, const int32_t *__restrict__ front_idx,
             const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r, double *x,
             double *ycb, int nrhs) {
  extern __shared__ double sm[];
  double *V = sm;
  const int4 tk = tasks[blockIdx.x];
  const WaveRec d = recs[tk.x];
  const int m = d.m, k = d.k, row0 = tk.y, rows = tk.z;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int plo = UP ? k : 0, phi = UP ? m : k;
  const double *F = store + d.store;
  const int32_t *idx = front_idx + d.idx;
  const int wrow = Q ? 0 : 16 * wv;                          // this wave's first output row
  const int arow = row0 + min(wrow + li, rows - 1);          // this lane's A-operand row
  constexpr int NS = Q ? kRectCols / 16 : kRectCols / 4;     // MFMA steps per wave and group
  const int s0 = Q ? 16 * wv : 0;                            // this wave's first step
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = min(16, nrhs - r0), col = li;
    // the values the product is combined with, for this lane's four result entries
    double base[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = wrow + 4 * r + lk, row = row0 + orow;
      base[r] = 0.0;
      if (orow < rows && col < nr) {
        if (UP) {
          base[r] = x[(int64_t)idx[row] * nrhs + r0 + col];
        } else {
          // children that pass a contribution block (none for a leaf or a pass-through leaf)
          const int xa = d.ycb[0] >= 0 ? inv_l[d.idx + row] : -1;
          const int xc = d.ycb[1] >= 0 ? inv_r[d.idx + row] : -1;
          if (xa >= 0) base[r] += ycb[(d.ycb[0] + xa) * nrhs + r0 + col];
          if (xc >= 0) base[r] += ycb[(d.ycb[1] + xc) * nrhs + r0 + col];
        }
      }
    }
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = plo; c0 < phi; c0 += kRectCols) {
      // MFMA steps of 4 columns that hold data in this group (the last group is usually
      // partial): chunks of 16 steps beyond them are neither loaded nor multiplied
      const int nst = min(kRectCols / 4, (phi - c0 + 3) / 4);
      double av[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int p = min(c0 + 4 * (s0 + s) + lk, phi - 1);
        av[s] = 0.0;
        if (((s0 + s) & ~15) < nst) av[s] = TRANS ? F[(int64_t)p * m + arow] : F[(int64_t)arow * m + p];
      }
      // thread t stages column p = c0 + t of the group (kRectCols = 256 threads): its 16
      // right-hand-side values, one contiguous row of x, loaded together
      const int pv = c0 + tid;
      const int64_t gp = pv < phi ? idx[pv] : 0;
      double vv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) vv[r] = (pv < phi && r < nr) ? x[gp * nrhs + r0 + r] : 0.0;
      __syncthreads();          // the previous group's V is no longer read
#pragma unroll
      for (int r = 0; r < 16; ++r) V[r * kRectLdv + tid] = vv[r];
      __syncthreads();
      // the B operands in chunks of 16 steps, each chunk's reads issued together (and
      // overlapping the previous chunk's products), then its MFMA chain
#pragma unroll
      for (int c = 0; c < NS; c += 16) {
        if (s0 + c >= nst) break;      // wave-uniform
        double vb[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) vb[u] = V[col * kRectLdv + 4 * (s0 + c + u) + lk];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 16; ++u)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c + u], vb[u], acc, 0, 0, 0);
      }
    }
    if constexpr (Q) {
      double *Red = V + 16 * kRectLdv;
#pragma unroll
      for (int r = 0; r < 4; ++r) Red[(wv * 64 + lane) * 4 + r] = acc[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[r] = ((Red[lane * 4 + r] + Red[(64 + lane) * 4 + r]) + Red[(128 + lane) * 4 + r]) +
                 Red[(192 + lane) * 4 + r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = wrow + 4 * r + lk, row = row0 + orow;
      if ((!Q || wv == 0) && orow < rows && col < nr) {
        if (UP)
          x[(int64_t)idx[row] * nrhs + r0 + col] = base[r] - acc[r];
        else
          ycb[(d.cbrow + row - k) * nrhs + r0 + col] = base[r] - acc[r];
      }
    }
    __syncthreads();            // V is rewritten by the next chunk
  }
}

// ---------------------------------------------------------------------------------------------
// Element-by-element operators (FP64).
// ---------------------------------------------------------------------------------------------

// r[v] = b[v] - sum over the (element, local node) pairs of v of K_e[a][:] x[conn_e]; the pairs
// of each node are listed in ascending element order, so the result is deterministic.
// part (may be null; requires nrhs | 256): the block's column sums of r^2, part[block][c] over
// the block's 256 / nrhs nodes, added in a fixed order.
__global__ void __launch_bounds__(256)
k_residual(const int64_t *__restrict__ nptr, const int32_t *__restrict__ nelem,
           const int32_t *__restrict__ conn, const double *__restrict__ K, int npe, int64_t n,
           const double *__restrict__ x, const double *__restrict__ b, double *__restrict__ r,
           int nrhs, double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rv = 0.0;
  if (t < n * nrhs) {
    const int64_t v = t / nrhs;
    const int c = (int)(t - v * nrhs);
    // the same sum in the same order, with the loads of a batch of (element, node) pairs and
    // of eight element columns issued together rather than one dependent chain per term
    double s = 0.0;
    const int64_t q0 = nptr[v], nq = nptr[v + 1] - q0;
    for (int64_t qb = 0; qb < nq; qb += 4) {
      int32_t ea[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ea[u] = qb + u < nq ? nelem[q0 + qb + u] : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (qb + u >= nq) break;
        const int32_t e = ea[u] / npe, a = ea[u] - (ea[u] / npe) * npe;
        const double *Ke = K + ((int64_t)e * npe + a) * npe;
        const int32_t *ce = conn + (int64_t)e * npe;
        for (int b0 = 0; b0 < npe; b0 += 8) {
          double kv[8], xv[8];
#pragma unroll
          for (int w = 0; w < 8; ++w) {
            const bool in = b0 + w < npe;
            kv[w] = in ? Ke[b0 + w] : 0.0;
            xv[w] = in ? x[(int64_t)ce[b0 + w] * nrhs + c] : 0.0;
          }
#pragma unroll
          for (int w = 0; w < 8; ++w)
            if (b0 + w < npe) s += kv[w] * xv[w];
        }
      }
    }
    rv = b[t] - s;
    r[t] = rv;
  }
  if (!part) return;                  // uniform
  red[threadIdx.x] = rv * rv;
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    double q = 0.0;
    for (int j = threadIdx.x; j < 256; j += nrhs) q += red[j];
    part[(int64_t)blockIdx.x * nrhs + threadIdx.x] = q;
  }
}

// The column sums of the partial sums of squares of the residual (and of b, bblocks > 0),
// written with the factorization's status words (status non-null) straight into mapped host
// memory: out[c] = sum over blocks of rpart[block][c], out[nrhs + c] the same of bpart.  One
// workgroup per column and vector; each thread adds its blocks in ascending order, then a fixed
// tree adds the threads: deterministic.  Each workgroup makes its writes visible to the host
// and counts itself in *count; the last one resets the count and writes seq to *seq_out, after
// which every value is readable by a host that sees seq.
__global__ void __launch_bounds__(256)
k_norm_publish(const double *__restrict__ rpart, int64_t rblocks,
               const double *__restrict__ bpart, int64_t bblocks, int nrhs,
               const int *__restrict__ status, double *out, int *out_status, int *count,
               int *seq_out, int seq) {
  __shared__ double red[256];
  const int c = blockIdx.x % nrhs;
  const bool isb = (int)blockIdx.x >= nrhs;
  const double *part = isb ? bpart : rpart;
  const int64_t nb = isb ? bblocks : rblocks;
  double s = 0.0;
  for (int64_t bl = threadIdx.x; bl < nb; bl += 256) s += part[bl * nrhs + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x] = red[0];
    if (blockIdx.x == 0 && status)
      for (int w = 0; w < kStatusWords; ++w) out_status[w] = status[w];
    __threadfence_system();
    __builtin_amdgcn_s_waitcnt(0);       // this block's values in memory before it is counted
    if (atomicAdd(count, 1) == (int)gridDim.x - 1) {
      *count = 0;
      __threadfence_system();
      __builtin_amdgcn_s_waitcnt(0);     // the write-back complete before the sequence number
      __hip_atomic_store(seq_out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Per-column partial sums of squares: part[block][c] over rows block*rows_per .. .
// When nrhs divides 256, the block walks its rows x columns range in flat order, 256 entries per
// round: every thread keeps one column (its index mod nrhs) and all loads are contiguous; the
// per-thread sums of a column are then added in a fixed order, so the result is deterministic.
// Otherwise one column after another.
__device__ __forceinline__ void colsq_block(const double *__restrict__ a, int64_t n, int nrhs,
                                            int64_t rows_per, double *__restrict__ part,
                                            double *red) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(n, r0 + rows_per);
  if (256 % nrhs == 0) {
    double s = 0.0;
    for (int64_t i = r0 * nrhs + threadIdx.x; i < r1 * nrhs; i += 256) {
      const double v = a[i];
      s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < nrhs) {
      double t = 0.0;
      for (int j = threadIdx.x; j < 256; j += nrhs) t += red[j];
      part[(int64_t)blockIdx.x * nrhs + threadIdx.x] = t;
    }
    return;
  }
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
k_colsq_partial(const double *__restrict__ a, int64_t n, int nrhs, int64_t rows_per,
                double *__restrict__ part) {
  __shared__ double red[256];
  colsq_block(a, n, nrhs, rows_per, part, red);
}

// The first launch of a combined factorization and solve: b's partial column sums of squares
// (as k_colsq_partial) and the clearing of the status words and of the persistent class
// launches' counters (as k_clear_status_counters), in one launch instead of two.
__global__ void __launch_bounds__(256)
k_refine_prologue(const double *__restrict__ b, int64_t n, int nrhs, int64_t rows_per,
                  double *__restrict__ part, int *__restrict__ st, int *__restrict__ cnt,
                  int64_t ncnt) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < kStatusWords) st[i] = 0;
  for (int64_t j = i; j < ncnt; j += (int64_t)gridDim.x * 256) cnt[j] = 0;
  colsq_block(b, n, nrhs, rows_per, part, red);
}

__global__ void __launch_bounds__(256)
k_axpy(double *__restrict__ x, const double *__restrict__ dx, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < len) x[t] += dx[t];
}

// Krylov kernels of the refinement with GMRES (FP64, [n][nrhs] blocks, one Krylov basis per
// right-hand side): partial column dots of w with nv basis vectors, a linear combination of basis
// vectors added to a block, and a column scaling.

// part[(blk * nv + i) * nrhs + c] = sum over the rows of block blk of V_i[row][c] * w[row][c];
// grid (row blocks of rows_per, nv).
__global__ void __launch_bounds__(256)
k_coldots_partial(const double *__restrict__ V, int64_t vstride, const double *__restrict__ w,
                  int64_t n, int nrhs, int64_t rows_per, double *__restrict__ part) {
  __shared__ double red[256];
  const int nv = gridDim.y, i = blockIdx.y;
  const double *a = V + (int64_t)i * vstride;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(n, r0 + rows_per);
  double *out = part + ((int64_t)blockIdx.x * nv + i) * nrhs;
  if (256 % nrhs == 0) {
    double s = 0.0;
    for (int64_t e = r0 * nrhs + threadIdx.x; e < r1 * nrhs; e += 256) s += a[e] * w[e];
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < nrhs) {
      double t = 0.0;
      for (int j = threadIdx.x; j < 256; j += nrhs) t += red[j];
      out[threadIdx.x] = t;
    }
    return;
  }
  for (int c = 0; c < nrhs; ++c) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) s += a[r * nrhs + c] * w[r * nrhs + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

// y[row][c] += sum_{i < nv} coef[i * nrhs + c] * V_i[row][c]
__global__ void __launch_bounds__(256)
k_combine(double *__restrict__ y, const double *__restrict__ V, int64_t vstride, int nv,
          const double *__restrict__ coef, int64_t n, int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nrhs) return;
  const int c = (int)(e % nrhs);
  double s = y[e];
  for (int i = 0; i < nv; ++i) s += coef[i * nrhs + c] * V[(int64_t)i * vstride + e];
  y[e] = s;
}

// dst[row][c] = scale[c] * src[row][c]
__global__ void __launch_bounds__(256)
k_scale_cols(double *__restrict__ dst, const double *__restrict__ src,
             const double *__restrict__ scale, int64_t n, int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nrhs) return;
  dst[e] = scale[e % nrhs] * src[e];
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
