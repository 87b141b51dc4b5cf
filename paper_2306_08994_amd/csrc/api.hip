// api.hip -- C ABI of libmf (declared in include/mf.h): device plan upload, the per-class launch
// schedule of the factorization (Sec. 3.3: Foata classes run in order, fronts inside a class
// run concurrently), the substitution sweeps, refinement and the adjoint helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(MF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

struct StepDev {
  int64_t fronts = 0, p0 = 0, n = 0;
  int64_t update = 0, n_update = 0;
  int64_t trsm_items = 0;
};

struct LevelDev {
  int64_t small = 0, n_small = 0;
  int32_t small_max_m = 0;
  int64_t large = 0, n_large = 0;
  int32_t large_max_m = 0;
  int64_t all = 0, n_all = 0;
  int32_t max_m = 0;
  std::vector<StepDev> steps;
  int64_t schur = 0, n_schur = 0;
};

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

}  // namespace

struct mf_plan {
  mf::HostPlan hp;
  mf::Tuning tune;
  int device = -1;
  bool uploaded = false;
  bool factored = false;
  int max_shared = 65536;
  mf::FrontDesc *d_desc = nullptr;
  int32_t *d_front_idx = nullptr, *d_inv_l = nullptr, *d_inv_r = nullptr, *d_conn = nullptr;
  int64_t *d_nptr = nullptr;
  int32_t *d_nelem = nullptr;
  int32_t *d_lists = nullptr;
  mf::GemmTask *d_tasks = nullptr;
  double *d_store = nullptr;
  int *d_status = nullptr;
  int *h_status = nullptr;
  double *d_ycb = nullptr;
  size_t ycb_cap = 0;
  double *d_work = nullptr;
  size_t work_cap = 0;
  double *h_part = nullptr;
  size_t part_cap = 0;
  std::vector<LevelDev> lv;

  ~mf_plan() {
    dfree(d_desc);
    dfree(d_front_idx);
    dfree(d_inv_l);
    dfree(d_inv_r);
    dfree(d_conn);
    dfree(d_nptr);
    dfree(d_nelem);
    dfree(d_lists);
    dfree(d_tasks);
    dfree(d_store);
    dfree(d_status);
    dfree(d_ycb);
    dfree(d_work);
    if (h_status) (void)hipHostFree(h_status);
    if (h_part) (void)hipHostFree(h_part);
  }
};

namespace {

template <typename T>
int upload(T *&dst, const std::vector<T> &src) {
  dfree(dst);
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  HIPCHK(hipMalloc((void **)&dst, bytes));
  if (!src.empty()) HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return MF_OK;
}

int ensure_uploaded(mf_plan *P) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (P->uploaded) {
    if (dev != P->device)
      return fail(MF_EINVAL, "plan was uploaded to device " + std::to_string(P->device) +
                                 " but the current device is " + std::to_string(dev));
    return MF_OK;
  }
  P->device = dev;
  HIPCHK(hipDeviceGetAttribute(&P->max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  mf::HostPlan &H = P->hp;
  // widest front whose padded square fits in one workgroup's LDS
  int32_t mm = 1;
  while ((int64_t)(mm + 1) * ((mm + 1) | 1) * 8 <= P->max_shared) ++mm;
  P->tune.small_max_m = std::min<int32_t>(P->tune.small_max_m, mm);
  mf::build_schedule(H, P->tune);
  // flatten the schedule
  std::vector<int32_t> lists;
  std::vector<mf::GemmTask> tasks;
  P->lv.assign(H.levels.size(), LevelDev());
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const mf::LevelSchedule &S = H.levels[l];
    LevelDev &D = P->lv[l];
    D.small = (int64_t)lists.size();
    D.n_small = (int64_t)S.small.size();
    D.small_max_m = S.small_max_m;
    lists.insert(lists.end(), S.small.begin(), S.small.end());
    D.large = (int64_t)lists.size();
    D.n_large = (int64_t)S.large.size();
    D.large_max_m = S.large_max_m;
    lists.insert(lists.end(), S.large.begin(), S.large.end());
    D.all = (int64_t)lists.size();
    D.n_all = (int64_t)S.all.size();
    D.max_m = S.max_m;
    lists.insert(lists.end(), S.all.begin(), S.all.end());
    for (const mf::PanelStep &st : S.steps) {
      StepDev sd;
      sd.n = (int64_t)st.fronts.size();
      sd.fronts = (int64_t)lists.size();
      lists.insert(lists.end(), st.fronts.begin(), st.fronts.end());
      sd.p0 = (int64_t)lists.size();
      lists.insert(lists.end(), st.p0.begin(), st.p0.end());
      sd.update = (int64_t)tasks.size();
      sd.n_update = (int64_t)st.update.size();
      tasks.insert(tasks.end(), st.update.begin(), st.update.end());
      sd.trsm_items = st.trsm_items;
      D.steps.push_back(sd);
    }
    D.schur = (int64_t)tasks.size();
    D.n_schur = (int64_t)S.schur.size();
    tasks.insert(tasks.end(), S.schur.begin(), S.schur.end());
  }
  // node -> (element, local node) pairs in ascending element order, for the residual
  std::vector<int64_t> nptr(H.n + 1, 0);
  for (int64_t q = 0; q < H.n_elem * H.npe; ++q) nptr[H.conn[q] + 1]++;
  for (int64_t v = 0; v < H.n; ++v) nptr[v + 1] += nptr[v];
  std::vector<int32_t> nelem(H.n_elem * H.npe);
  {
    std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
    for (int64_t q = 0; q < H.n_elem * H.npe; ++q) nelem[fill[H.conn[q]]++] = (int32_t)q;
  }
  int rc;
  if ((rc = upload(P->d_desc, H.desc)) || (rc = upload(P->d_front_idx, H.front_idx)) ||
      (rc = upload(P->d_inv_l, H.inv_l)) || (rc = upload(P->d_inv_r, H.inv_r)) ||
      (rc = upload(P->d_conn, H.conn)) || (rc = upload(P->d_nptr, nptr)) ||
      (rc = upload(P->d_nelem, nelem)) || (rc = upload(P->d_lists, lists)) ||
      (rc = upload(P->d_tasks, tasks)))
    return rc;
  dfree(P->d_store);
  if (hipMalloc((void **)&P->d_store, std::max<int64_t>(1, H.store_doubles) * sizeof(double)) != hipSuccess)
    return fail(MF_ENOMEM, "cannot allocate " + std::to_string(H.store_doubles * 8) +
                               " bytes of factor storage");
  if (!P->d_status) HIPCHK(hipMalloc((void **)&P->d_status, mf::kStatusWords * sizeof(int)));
  if (!P->h_status)
    HIPCHK(hipHostMalloc((void **)&P->h_status, mf::kStatusWords * sizeof(int), hipHostMallocDefault));
  // raise the dynamic-LDS limit of the kernels that size LDS per launch (best effort)
  const void *dyn[] = {(const void *)mf::k_factor_small<256>, (const void *)mf::k_solve_down<false>,
                       (const void *)mf::k_solve_down<true>, (const void *)mf::k_solve_up<false>,
                       (const void *)mf::k_solve_up<true>};
  for (const void *fn : dyn)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_shared);
  (void)hipGetLastError();
  P->uploaded = true;
  return MF_OK;
}

int grow(double *&buf, size_t &cap, size_t doubles) {
  if (cap >= doubles && buf) return MF_OK;
  dfree(buf);
  cap = 0;
  if (hipMalloc((void **)&buf, std::max<size_t>(doubles, 1) * sizeof(double)) != hipSuccess)
    return fail(MF_ENOMEM, "cannot allocate " + std::to_string(doubles * 8) + " bytes of workspace");
  cap = doubles;
  return MF_OK;
}

int launch_factor(mf_plan *P, const double *K, int prec, hipStream_t s) {
  const mf::HostPlan &H = P->hp;
  hipLaunchKernelGGL(mf::k_clear_status, dim3(1), dim3(64), 0, s, P->d_status);
  for (size_t l = 0; l < P->lv.size(); ++l) {
    const LevelDev &D = P->lv[l];
    if (D.n_small) {
      const int m = D.small_max_m;
      const size_t lds = (size_t)m * (m | 1) * sizeof(double);
      const int grid = (int)std::min<int64_t>(D.n_small, 16384);
      hipLaunchKernelGGL(mf::k_factor_small<256>, dim3(grid), dim3(256), lds, s, P->d_desc,
                         P->d_lists + D.small, (int)D.n_small, P->d_store, P->d_inv_l, P->d_inv_r,
                         K, H.npe, P->d_status);
    }
    if (D.n_large) {
      hipLaunchKernelGGL(mf::k_assemble, dim3((D.large_max_m + 3) / 4, (unsigned)D.n_large),
                         dim3(256), 0, s, P->d_desc, P->d_lists + D.large, P->d_store, P->d_inv_l,
                         P->d_inv_r, K, H.npe);
      for (const StepDev &st : D.steps) {
        const dim3 gd((unsigned)st.n), gt((unsigned)((st.trsm_items + 255) / 256), (unsigned)st.n);
        const int32_t *fr = P->d_lists + st.fronts, *p0 = P->d_lists + st.p0;
        switch (P->tune.nb) {
          case 16:
            hipLaunchKernelGGL(mf::k_panel_diag<16>, gd, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store, P->d_status);
            if (st.trsm_items > 0)
              hipLaunchKernelGGL(mf::k_panel_trsm<16>, gt, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store);
            break;
          case 64:
            hipLaunchKernelGGL(mf::k_panel_diag<64>, gd, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store, P->d_status);
            if (st.trsm_items > 0)
              hipLaunchKernelGGL(mf::k_panel_trsm<64>, gt, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store);
            break;
          default:
            hipLaunchKernelGGL(mf::k_panel_diag<32>, gd, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store, P->d_status);
            if (st.trsm_items > 0)
              hipLaunchKernelGGL(mf::k_panel_trsm<32>, gt, dim3(256), 0, s, P->d_desc, fr, p0, P->d_store);
        }
        if (st.n_update)
          hipLaunchKernelGGL(mf::k_gemm_update<0>, dim3((unsigned)st.n_update), dim3(256), 0, s,
                             P->d_desc, P->d_tasks + st.update, P->d_store);
      }
      if (D.n_schur) {
        const mf::GemmTask *t = P->d_tasks + D.schur;
        if (prec == MF_SCHUR_FP32)
          hipLaunchKernelGGL(mf::k_gemm_update<1>, dim3((unsigned)D.n_schur), dim3(256), 0, s,
                             P->d_desc, t, P->d_store);
        else if (prec == MF_SCHUR_BF16)
          hipLaunchKernelGGL(mf::k_gemm_update<2>, dim3((unsigned)D.n_schur), dim3(256), 0, s,
                             P->d_desc, t, P->d_store);
        else
          hipLaunchKernelGGL(mf::k_gemm_update<0>, dim3((unsigned)D.n_schur), dim3(256), 0, s,
                             P->d_desc, t, P->d_store);
      }
    }
  }
  HIPCHK(hipGetLastError());
  return MF_OK;
}

int chunk_for(const mf_plan *P, int32_t max_m, int32_t nrhs) {
  int nc = 1;
  while (nc * 2 <= nrhs && (int64_t)max_m * nc * 2 * 8 <= P->max_shared) nc *= 2;
  return nc;
}

int launch_solve(const mf_plan *P, const double *b, double *x, int32_t nrhs, bool trans,
                 hipStream_t s) {
  const int gridcap = 8192;
  for (size_t l = 0; l < P->lv.size(); ++l) {
    const LevelDev &D = P->lv[l];
    if (!D.n_all) continue;
    const int nc = chunk_for(P, D.max_m, nrhs);
    const size_t lds = (size_t)D.max_m * nc * sizeof(double);
    const int grid = (int)std::min<int64_t>(D.n_all, gridcap);
    if (trans)
      hipLaunchKernelGGL(mf::k_solve_down<true>, dim3(grid), dim3(256), lds, s, P->d_desc,
                         P->d_lists + D.all, (int)D.n_all, P->d_store, P->d_front_idx, P->d_inv_l,
                         P->d_inv_r, b, x, P->d_ycb, nrhs, nc);
    else
      hipLaunchKernelGGL(mf::k_solve_down<false>, dim3(grid), dim3(256), lds, s, P->d_desc,
                         P->d_lists + D.all, (int)D.n_all, P->d_store, P->d_front_idx, P->d_inv_l,
                         P->d_inv_r, b, x, P->d_ycb, nrhs, nc);
  }
  for (size_t l = P->lv.size(); l-- > 0;) {
    const LevelDev &D = P->lv[l];
    if (!D.n_all) continue;
    const int nc = chunk_for(P, D.max_m, nrhs);
    const size_t lds = (size_t)D.max_m * nc * sizeof(double);
    const int grid = (int)std::min<int64_t>(D.n_all, gridcap);
    if (trans)
      hipLaunchKernelGGL(mf::k_solve_up<true>, dim3(grid), dim3(256), lds, s, P->d_desc,
                         P->d_lists + D.all, (int)D.n_all, P->d_store, P->d_front_idx, x, nrhs, nc);
    else
      hipLaunchKernelGGL(mf::k_solve_up<false>, dim3(grid), dim3(256), lds, s, P->d_desc,
                         P->d_lists + D.all, (int)D.n_all, P->d_store, P->d_front_idx, x, nrhs, nc);
  }
  HIPCHK(hipGetLastError());
  return MF_OK;
}

// max over columns of ||a_c||_2 / ||ref_c||_2 (ref may be null: plain norms returned in out)
int col_norms(mf_plan *P, const double *a, int64_t n, int32_t nrhs, hipStream_t s,
              std::vector<double> &out) {
  const int64_t rows_per = 4096;
  const int64_t blocks = std::max<int64_t>(1, (n + rows_per - 1) / rows_per);
  const size_t need = (size_t)blocks * nrhs;
  if (P->part_cap < need) {
    if (P->h_part) (void)hipHostFree(P->h_part);
    P->h_part = nullptr;
    P->part_cap = 0;
    HIPCHK(hipHostMalloc((void **)&P->h_part, need * sizeof(double), hipHostMallocDefault));
    P->part_cap = need;
  }
  // partials live at the tail of the work buffer
  double *dpart = P->d_work + 2 * (size_t)n * nrhs;
  hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)blocks), dim3(256), 0, s, a, n, nrhs,
                     rows_per, dpart);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(P->h_part, dpart, need * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out.assign(nrhs, 0.0);
  for (int64_t bl = 0; bl < blocks; ++bl)
    for (int c = 0; c < nrhs; ++c) out[c] += P->h_part[bl * nrhs + c];
  for (int c = 0; c < nrhs; ++c) out[c] = std::sqrt(out[c]);
  return MF_OK;
}

}  // namespace

extern "C" {

const char *mf_last_error(void) { return g_err.c_str(); }

int mf_analyse(int32_t n_mesh, const mf_mesh *meshes, mf_plan **out) {
  if (!out) return fail(MF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_mesh < 1 || !meshes) return fail(MF_EINVAL, "need n_mesh >= 1 and a mesh array");
  std::vector<int32_t> dims(n_mesh), npes(n_mesh);
  std::vector<int64_t> nn(n_mesh), ne(n_mesh);
  std::vector<const int32_t *> conns(n_mesh), ijks(n_mesh);
  for (int32_t i = 0; i < n_mesh; ++i) {
    dims[i] = meshes[i].dim;
    npes[i] = meshes[i].npe;
    nn[i] = meshes[i].n_nodes;
    ne[i] = meshes[i].n_elem;
    conns[i] = meshes[i].conn;
    ijks[i] = meshes[i].elem_ijk;
  }
  mf_plan *P = new (std::nothrow) mf_plan();
  if (!P) return fail(MF_ENOMEM, "cannot allocate plan");
  std::string err;
  try {
    err = mf::analyse(n_mesh, dims.data(), npes.data(), nn.data(), ne.data(), conns.data(),
                      ijks.data(), P->hp);
  } catch (const std::bad_alloc &) {
    delete P;
    return fail(MF_ENOMEM, "host allocation failed during analysis");
  }
  if (!err.empty()) {
    delete P;
    return fail(MF_EINVAL, err);
  }
  *out = P;
  return MF_OK;
}

int mf_plan_info(const mf_plan *P, mf_info *o) {
  if (!P || !o) return fail(MF_EINVAL, "null argument");
  const mf::HostPlan &H = P->hp;
  o->n = H.n;
  o->n_elem = H.n_elem;
  o->n_fronts = H.F;
  o->sum_m = (int64_t)H.front_idx.size();
  o->sum_mk = H.sum_mk;
  o->store_doubles = H.store_doubles;
  o->n_mesh = H.n_mesh;
  o->dim = H.dim;
  o->npe = H.npe;
  o->height = H.height;
  o->max_m = H.max_m;
  o->max_k = H.max_k;
  o->factor_flops = H.factor_flops;
  o->solve_flops_per_rhs = H.solve_flops;
  o->sum_cb2 = H.sum_cb2;
  return MF_OK;
}

int mf_plan_export_tree(const mf_plan *P, int32_t *parent, int32_t *level, int64_t *front_ptr,
                        int32_t *front_idx, int32_t *npiv, int64_t *leaf_elem) {
  if (!P) return fail(MF_EINVAL, "null plan");
  const mf::HostPlan &H = P->hp;
  if (parent) std::memcpy(parent, H.parent.data(), H.F * sizeof(int32_t));
  if (level) std::memcpy(level, H.level.data(), H.F * sizeof(int32_t));
  if (front_ptr) std::memcpy(front_ptr, H.front_ptr.data(), (H.F + 1) * sizeof(int64_t));
  if (front_idx) std::memcpy(front_idx, H.front_idx.data(), H.front_idx.size() * sizeof(int32_t));
  if (npiv) std::memcpy(npiv, H.npiv.data(), H.F * sizeof(int32_t));
  if (leaf_elem) std::memcpy(leaf_elem, H.leaf_elem.data(), H.F * sizeof(int64_t));
  return MF_OK;
}

int mf_set_tuning(mf_plan *P, int32_t small_max_m, int32_t nb) {
  if (!P) return fail(MF_EINVAL, "null plan");
  if (small_max_m < 0) return fail(MF_EINVAL, "small_max_m must be >= 0");
  if (nb != 0 && nb != 16 && nb != 32 && nb != 64) return fail(MF_EINVAL, "nb must be 16, 32 or 64");
  if (small_max_m > 0) P->tune.small_max_m = small_max_m;
  if (nb > 0) P->tune.nb = nb;
  P->uploaded = false;      // the schedule is rebuilt at the next device call
  P->factored = false;
  return MF_OK;
}

int mf_factor(mf_plan *P, const double *elem_mats, int32_t precision, void *hip_stream) {
  if (!P || !elem_mats) return fail(MF_EINVAL, "null plan or element matrices");
  if (precision != MF_FP64 && precision != MF_SCHUR_FP32 && precision != MF_SCHUR_BF16)
    return fail(MF_EINVAL, "unknown precision " + std::to_string(precision));
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  P->factored = false;
  if ((rc = launch_factor(P, elem_mats, precision, s))) return rc;
  HIPCHK(hipMemcpyAsync(P->h_status, P->d_status, mf::kStatusWords * sizeof(int),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (P->h_status[0])
    return fail(MF_EZERO_PIVOT, "zero or non-finite pivot in front " + std::to_string(P->h_status[1]) +
                                    ", pivot " + std::to_string(P->h_status[2]));
  P->factored = true;
  return MF_OK;
}

int mf_solve(const mf_plan *Pc, const double *b, double *x, int32_t nrhs, int32_t transpose,
             void *hip_stream) {
  mf_plan *P = const_cast<mf_plan *>(Pc);
  if (!P || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  if (transpose != 0 && transpose != 1) return fail(MF_EINVAL, "transpose must be 0 or 1");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  int rc;
  if ((rc = grow(P->d_ycb, P->ycb_cap, (size_t)std::max<int64_t>(1, P->hp.sum_c) * nrhs))) return rc;
  return launch_solve(P, b, x, nrhs, transpose != 0, (hipStream_t)hip_stream);
}

int mf_residual(const mf_plan *P, const double *elem_mats, const double *x, const double *b,
                double *r, int32_t nrhs, void *hip_stream) {
  if (!P || !elem_mats || !x || !b || !r) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  int rc = ensure_uploaded(const_cast<mf_plan *>(P));
  if (rc) return rc;
  const mf::HostPlan &H = P->hp;
  const int64_t tot = H.n * nrhs;
  hipLaunchKernelGGL(mf::k_residual, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, P->d_nptr, P->d_nelem, P->d_conn, elem_mats, H.npe,
                     H.n, x, b, r, nrhs);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

int mf_refine(const mf_plan *Pc, const double *elem_mats, const double *b, double *x,
              int32_t nrhs, double tol, int32_t max_it, int32_t *its, double *relres,
              void *hip_stream) {
  mf_plan *P = const_cast<mf_plan *>(Pc);
  if (!P || !elem_mats || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1 || max_it < 0 || !(tol >= 0)) return fail(MF_EINVAL, "bad nrhs, max_it or tol");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n = P->hp.n;
  const size_t nn = (size_t)n * nrhs;
  const size_t parts = (size_t)std::max<int64_t>(1, (n + 4095) / 4096) * nrhs;
  int rc;
  if ((rc = grow(P->d_work, P->work_cap, 2 * nn + parts))) return rc;
  double *r = P->d_work, *dx = P->d_work + nn;
  if ((rc = mf_solve(P, b, x, nrhs, 0, hip_stream))) return rc;
  std::vector<double> bn, rn;
  if ((rc = col_norms(P, b, n, nrhs, s, bn))) return rc;
  double rr = 0.0;
  for (int32_t it = 0;; ++it) {
    if ((rc = mf_residual(P, elem_mats, x, b, r, nrhs, hip_stream))) return rc;
    if ((rc = col_norms(P, r, n, nrhs, s, rn))) return rc;
    rr = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double q = bn[c] > 0 ? rn[c] / bn[c] : (rn[c] > 0 ? INFINITY : 0.0);
      rr = std::max(rr, std::isnan(q) ? INFINITY : q);
    }
    if (its) *its = it;
    if (relres) *relres = rr;
    if (rr <= tol) return MF_OK;
    if (it >= max_it) break;
    if ((rc = mf_solve(P, r, dx, nrhs, 0, hip_stream))) return rc;
    hipLaunchKernelGGL(mf::k_axpy, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, x, dx,
                       (int64_t)nn);
    HIPCHK(hipGetLastError());
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "refinement stopped after %d corrections at relres %.3e > tol %.3e",
                max_it, rr, tol);
  return fail(MF_ENOCONV, buf);
}

int mf_elem_grad(const mf_plan *P, const double *lam, const double *u, int32_t nrhs, double *gK,
                 void *hip_stream) {
  if (!P || !lam || !u || !gK) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  int rc = ensure_uploaded(const_cast<mf_plan *>(P));
  if (rc) return rc;
  const mf::HostPlan &H = P->hp;
  const int64_t tot = H.n_elem * H.npe * H.npe;
  hipLaunchKernelGGL(mf::k_elem_grad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, P->d_conn, H.n_elem, H.npe, lam, u, nrhs, gK);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

int mf_export_factors(const mf_plan *P, double *L, double *U) {
  if (!P || !L || !U) return fail(MF_EINVAL, "null argument");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  const mf::HostPlan &H = P->hp;
  std::vector<double> st;
  try {
    st.resize(H.store_doubles);
  } catch (const std::bad_alloc &) {
    return fail(MF_ENOMEM, "cannot allocate host copy of the factors");
  }
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(st.data(), P->d_store, H.store_doubles * sizeof(double), hipMemcpyDeviceToHost));
  int64_t off = 0;
  for (int64_t f = 0; f < H.F; ++f) {
    const mf::FrontDesc &d = H.desc[f];
    const double *Fm = st.data() + d.store;
    double *Lf = L + off, *Uf = U + off;
    for (int32_t i = 0; i < d.m; ++i)
      for (int32_t p = 0; p < d.k; ++p) {
        Lf[(int64_t)i * d.k + p] = i >= p ? Fm[(int64_t)i * d.m + p] : 0.0;
        Uf[(int64_t)p * d.m + i] = i > p ? Fm[(int64_t)p * d.m + i] : (i == p ? 1.0 : 0.0);
      }
    off += (int64_t)d.m * d.k;
  }
  return MF_OK;
}

void mf_destroy(mf_plan *P) { delete P; }

}  // extern "C"
