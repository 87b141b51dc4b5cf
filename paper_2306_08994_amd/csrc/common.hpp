// common.hpp -- device-side helpers shared by the factor and solve kernels.
//
// Storage: every front f owns an m x m row-major FP64 block at store + desc[f].store.  After the
// front is factored it holds, in place,
//   L (pivots on the diagonal)  at rows p..m-1 of columns p < k,
//   U (unit diagonal, implicit) at columns p+1..m-1 of rows p < k,
//   the Schur complement (contribution block, CB) in rows and columns k..m-1,
// i.e. the result of the division / multiplication / subtraction tasks of Table 2 applied to
// the assembled front.  A parent reads its children's CBs straight from their storage.
// A leaf without pivots is never stored: its CB is its element matrix, and the parent's
// extend-add map addresses the element matrix directly.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <type_traits>

#include "plan.hpp"

namespace mf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
// two consecutive doubles at any 8-byte-aligned address: one 16-byte access (the memory
// system takes accesses that are not naturally aligned)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

constexpr int kStatusWords = 4;   // [0] bad-pivot flag, [1] front, [2] pivot, [3] wait abort

__device__ inline void record_bad_pivot(int *st, int f, int p) {
  if (atomicCAS(st, 0, 1) == 0) {
    st[1] = f;
    st[2] = p;
  }
}

__device__ inline bool good_pivot(double v) { return v != 0.0 && __builtin_isfinite(v); }

// Orders the LDS traffic of one wave: every LDS access the wave issued before is complete and
// visible to the accesses it issues after (a wave executes in lockstep, so no s_barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__global__ void k_clear_status(int *st) {
  if (threadIdx.x < kStatusWords) st[threadIdx.x] = 0;
}

// Clears the status block and n counters (the persistent class launches' tickets and progress
// counters) at the start of a factorization: a kernel, so that captured graphs replay it.
__global__ void k_clear_status_counters(int *st, int *cnt, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < kStatusWords) st[i] = 0;
  for (int64_t j = i; j < n; j += (int64_t)gridDim.x * blockDim.x) cnt[j] = 0;
}

// Sources of the extend-add of one front: its element matrix (a leaf), or its two children's
// contribution blocks (left first, then right), each with its leading dimension.
struct GatherCtx {
  const double *ke;   // element matrix of a leaf front, else null
  const double *ca, *cb;
  int la, lb, npe;
  int na, nb;         // contribution-block sizes of the two sources (a leaf: npe, 0)
};

// Extend-add sources of a front from its wave record: a leaf (no second source) reads its
// element matrix.
__device__ inline GatherCtx rec_gather_ctx(const WaveRec &r, const double *__restrict__ store,
                                           const double *__restrict__ K) {
  GatherCtx g;
  const double *s0 = r.src[0] >= 0 ? store + r.src[0] : K + (-1 - r.src[0]);
  const double *s1 = r.src[1] >= 0 ? store + r.src[1] : K + (-1 - r.src[1]);
  g.npe = r.ld[0];
  g.ke = r.n[1] > 0 ? nullptr : s0;
  g.ca = s0;
  g.la = r.ld[0];
  g.na = r.n[0];
  g.cb = r.n[1] > 0 ? s1 : nullptr;
  g.lb = r.ld[1];
  g.nb = r.n[1];
  return g;
}

// Entry (i, j) of the assembled front from the maps of rows i and j: for a leaf, li/lj are
// local element nodes; otherwise li/lj (ri/rj) index the left (right) child's CB, -1 = absent.
__device__ inline double gather_entry(const GatherCtx &g, int li, int lj, int ri, int rj) {
  if (g.ke) return g.ke[li * g.npe + lj];
  double v = 0.0;
  if ((li | lj) >= 0) v += g.ca[(int64_t)li * g.la + lj];
  if ((ri | rj) >= 0) v += g.cb[(int64_t)ri * g.lb + rj];
  return v;
}

// One source of the extend-add: its n x n block (leading dimension lda, contiguous rows) is
// assigned (ADD = false) or added into the LDS front at rows/columns map[.].  Loads are issued
// in batches of four independent reads before their LDS writes, so a thread keeps several
// memory round trips in flight.
template <bool ADD>
__device__ inline void scatter_source(const double *__restrict__ src, int lda, int n,
                                      const int *map, int ld, double *sh, int t0, int nt) {
  const int nn = n * n;
  if (nn == 0) return;
  // (r, c) of entry t, advanced by nt entries per step without a division
  const int dr = nt / n, dc = nt - dr * n;
  int r = t0 / n, c = t0 - r * n;
  for (int tb = t0; tb < nn; tb += 4 * nt) {
    double v[4];
    int dst[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = tb + u * nt;
      dst[u] = -1;
      v[u] = 0.0;
      if (t < nn) {
        v[u] = src[(int64_t)r * lda + c];
        dst[u] = map[r] * ld + map[c];
      }
      c += dc;
      r += dr;
      if (c >= n) {
        c -= n;
        ++r;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (dst[u] >= 0) {
        if (ADD)
          sh[dst[u]] += v[u];
        else
          sh[dst[u]] = v[u];
      }
  }
}

// Extend-add into an LDS front (row stride ld) by scattering the sources' contiguous rows:
// zero, then the left source assigned, then the right source added -- the same order of
// additions as summing the entries of each front position left then right.  `sync` orders
// LDS between the phases (a workgroup barrier or a wave-level fence); ma/mb are int scratch
// of at least na/nb entries.
template <typename Sync>
__device__ inline void scatter_assemble(const GatherCtx &g, const int32_t *__restrict__ il,
                                        const int32_t *__restrict__ ir, int m, int ld, double *sh,
                                        int *ma, int *mb, int t0, int nt, Sync sync) {
  for (int t = t0; t < m * ld; t += nt) sh[t] = 0.0;
  for (int i = t0; i < m; i += nt) {
    const int x = il[i];
    if (x >= 0) ma[x] = i;
    if (!g.ke) {
      const int y = ir[i];
      if (y >= 0) mb[y] = i;
    }
  }
  sync();
  scatter_source<false>(g.ca, g.la, g.na, ma, ld, sh, t0, nt);
  sync();
  if (!g.ke) scatter_source<true>(g.cb, g.lb, g.nb, mb, ld, sh, t0, nt);
  sync();
}

}  // namespace mf
