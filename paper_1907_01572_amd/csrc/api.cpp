// C ABI of the hpdg library: contexts, mesh upload, apply / smooth / V-cycle / solve.
//
// Solver structure (arXiv:1907.01572): flexible CG (Alg. 2) preconditioned by a V-cycle
// (Alg. 3) over the stored level hierarchy, Chebyshev smoothing (Alg. 4) with spectral
// bounds from CG (Alg. 5, computed once per level), exact FP64 coarse solve.  Every
// step runs in the kernels of kernels.hip, stream-ordered; the host only sequences
// launches and reads one residual norm per Krylov iteration.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstdio>
#include <limits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/hpdg.h"
#include "device.hpp"
#include "setup.hpp"
#include "schwarz.hpp"

using namespace hpdg;

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) throw Error(HPDG_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct hpdg_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::vector<hpdg_mesh*> meshes;
  std::mutex mu;  // guards used and meshes (a solve server uploads from several threads)
};

namespace {

template <typename T>
struct DevLevel {
  ElemInfo* einfo = nullptr;
  MortarInfo* minfo = nullptr;
  int* fmlist = nullptr;
  T* vgeo = nullptr;
  T* mgeo = nullptr;
  T* dinv = nullptr;
  TransferInfo* tinfo = nullptr;  // prolongation from level + 1 into this level
  int* cstart = nullptr;
  int* clist = nullptr;
  T *f = nullptr, *v = nullptr, *t = nullptr, *p = nullptr;
  long long* poff = nullptr;  // element-block Jacobi: offsets of the packed inverse blocks
  T* binv = nullptr;           // packed lower triangles of the inverse blocks
  long long* boff16 = nullptr;  // offsets of the full bf16 blocks (FP32 levels)
  uint16_t* binv16 = nullptr;   // full bf16 copies of the inverse blocks (FP32 levels)
  int* belems = nullptr;      // element ids grouped by (n, q) (elements of the element kernel)
  int* felems = nullptr;      // element-centric apply: element ids grouped by n
  int* telems = nullptr;      // elements whose face traces the mortar kernel reads
  FaceLink* flink = nullptr;  // element-centric apply, group order: face records (6 per element),
  long long* fe_off = nullptr;  // dof offsets, face-trace offsets and the diagonal metric (3 per element)
  long long* fe_toff = nullptr;
  T* fe_g = nullptr;
  T* fcoef = nullptr;         // face coefficient tuples
  // mass term (Newton linearisation): w det J c at the GL points, the diagonal of A
  T* mcoef = nullptr;
  T* diag = nullptr;
  MortarTask* mtask = nullptr;
  T* trace = nullptr;  // face traces (written before each apply)
  T* slot = nullptr;   // lifted face terms (written by the mortar kernel before each element kernel)
  T* trace2 = nullptr;  // block smoothing: the next step's traces, written by the fused step
  double* nl_alpha = nullptr;  // alpha and w det J beta at the GL points (FP64 levels only)
  double* nl_wbeta = nullptr;
};

}  // namespace

struct hpdg_mesh {
  hpdg_ctx* ctx = nullptr;
  MacroMesh mm;
  DiscParams dp;
  OpTable tab;
  std::vector<LevelHost> H;
  bool has_f32 = false;
  // device
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  size_t bytes = 0;
  int* tab_off = nullptr;
  int *dg_off = nullptr, *w_off = nullptr, *dface_off = nullptr, *gl_off = nullptr;
  double* tab64 = nullptr;
  float* tab32 = nullptr;
  std::vector<DevLevel<double>> L64;
  std::vector<DevLevel<float>> L32;
  double* Ainv64 = nullptr;  // explicit inverse of the coarsest operator (FP64 in every precision mode)
  int ncoarse = 0;
  // smoother
  std::vector<double> lam;
  hpdg_smoother_params sp{4, 15, 20.0, HPDG_SMOOTH_POINT, 0, 0, 0, 2};
  bool smoother_ready = false;
  rocblas_handle blas = nullptr;  // batched Cholesky of the element blocks (setup only)
  // nonlinear source (Newton)
  bool mass_on = true;            // false: applies leave out the mass term (the residual's A u)
  bool bf16_blocks = false;       // FP32 V-cycle reads the bf16 inverse blocks (HPDG_PREC_MIXED_BF16)
  std::vector<double> nl_key;     // kind and parameters of the source the GL tables hold
  int nl_kind = 0;                // HPDG_NL_* of that source
  int* bad = nullptr;             // device flag: 1 + alpha u <= 0 somewhere
  int* host_bad = nullptr;        // pinned
  double *nl_b = nullptr, *nl_rhs = nullptr, *nl_delta = nullptr;  // Newton: R, -R, correction
  // Krylov work
  double *r = nullptr, *vv = nullptr, *w = nullptr, *d = nullptr, *q = nullptr;
  double *partials = nullptr, *sc = nullptr;
  double* host_sc = nullptr;  // pinned
  // kernel timing: HIP events around every timing_every-th operator apply and block-smoother
  // step of each (kind, level, precision)
  bool timing = false;
  int timing_every = 1;
  long long timing_count[HPDG_TIMING_KINDS][32][2] = {};
  struct Timed {
    hipEvent_t a, b;
    int kind, level, prec;
    double bytes;
  };
  struct Acc {
    double ms = 0, bytes = 0;
    long long calls = 0;
  };
  std::vector<long long> block_scalars = std::vector<long long>(32, 0);  // packed inverse-block scalars per level
  std::vector<long long> block_full_scalars = std::vector<long long>(32, 0);  // full-block scalars per level
  double* gm_V = nullptr;  // FGMRES basis (gm_m + 1 level-0 vectors) and directions (gm_m)
  double* gm_Z = nullptr;
  int gm_m = 0;
  int max_levels = 32;     // cap on the hierarchy depth given at upload
  int block_retries = 0;   // block factorisations repeated after a failed attempt
  int coarse_retries = 0;  // coarse factorisations repeated after a failed attempt
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  // side stream of the apply (default priority): the element kernel's buckets run there beside
  // the element-centric groups; created on first use
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  Acc acc[HPDG_TIMING_KINDS][32][2];
  // a posteriori estimator: the point data of one problem on level 0 (rebuilt when the problem
  // changes) and the per-element / per-mortar parts
  struct EstCache {
    std::vector<double> key;  // rhs kind and parameters (empty: not built)
    EstVolume ev{};
    EstFace ef{};
    MortarTask* tasks = nullptr;
    long long n_tasks = 0;
    double* vpart = nullptr;
    std::vector<void*> ptrs;
    long long alg_bytes = 0, vpoints = 0, mpoints = 0;  // of one estimate (hpdg_mesh_info)
  } est;
  std::unique_ptr<MacroMesh> est_grid;  // the estimator's fiducial grid (null: the physical one)
  // macros and level-0 cells on the device (the right-hand side's volume part maps its points
  // there); uploaded on first use
  Macro* dmacros = nullptr;
  Cell* dcells = nullptr;
  // additive Schwarz smoother, per smoothed level (FP64): subdomain entries (global dofs), the
  // rows of W_s A_ss^-1 of the weighted entries, the local corrections and, per dof, the
  // corrections that sum into it
  struct SchwarzDev {
    int n_sub = 0, max_m = 0, max_nw = 0, overlap = 0;
    int* gidx = nullptr;
    long long *goff = nullptr, *woff = nullptr, *moff = nullptr;
    double* minv = nullptr;
    double* d = nullptr;
    float* minv32 = nullptr;  // FP32 copies for the FP32 V-cycle (meshes with FP32 levels), own stride
    float* d32 = nullptr;
    long long* moff32 = nullptr;
    long long* ptr = nullptr;
    int* list = nullptr;
    long long minv_scalars = 0, entries = 0;
    double alg_bytes = 0, alg_bytes32 = 0;  // of one launch of the local solves
    const double* rows(double*) const { return minv; }
    const float* rows(float*) const { return minv32; }
    double* corr(double*) const { return d; }
    float* corr(float*) const { return d32; }
    const long long* offs(double*) const { return moff; }
    const long long* offs(float*) const { return moff32; }
  };
  std::vector<SchwarzDev> sw;

  template <typename T>
  T* alloc(size_t count) {
    size_t b = count * sizeof(T);
    if (b == 0) b = sizeof(T);
    {
      std::lock_guard<std::mutex> lock(ctx->mu);
      if (ctx->budget && ctx->used + b > ctx->budget) throw Error(HPDG_ERR_OOM, "HBM budget exceeded");
      ctx->used += b;
    }
    void* ptr = nullptr;
    if (hipMalloc(&ptr, b) != hipSuccess) {
      std::lock_guard<std::mutex> lock(ctx->mu);
      ctx->used -= b;
      throw Error(HPDG_ERR_OOM, "hipMalloc failed");
    }
    allocs.push_back(ptr);
    alloc_bytes.push_back(b);
    bytes += b;
    return static_cast<T*>(ptr);
  }
  // free one allocation made by alloc() before the mesh is destroyed (setup temporaries)
  void release(void* ptr) {
    for (size_t i = 0; i < allocs.size(); ++i) {
      if (allocs[i] != ptr) continue;
      (void)hipFree(ptr);
      const size_t b = alloc_bytes[i];
      allocs.erase(allocs.begin() + i);
      alloc_bytes.erase(alloc_bytes.begin() + i);
      bytes -= b;
      std::lock_guard<std::mutex> lock(ctx->mu);
      ctx->used -= std::min(ctx->used, b);
      return;
    }
  }
  template <typename T, typename S>
  T* upload(const std::vector<S>& v, hipStream_t s) {
    T* ptr = alloc<T>(v.size());
    if (!v.empty()) {
      std::vector<T> tmp(v.begin(), v.end());
      HIPCHK(hipMemcpyAsync(ptr, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return ptr;
  }
  template <typename T>
  T* upload_raw(const std::vector<T>& v, hipStream_t s) {
    T* ptr = alloc<T>(v.size());
    if (!v.empty()) {
      HIPCHK(hipMemcpyAsync(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return ptr;
  }
  ~hpdg_mesh() {
    for (auto& ev : pending) {
      (void)hipEventDestroy(ev.a);
      (void)hipEventDestroy(ev.b);
    }
    for (auto ev : event_pool) (void)hipEventDestroy(ev);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (side) (void)hipStreamDestroy(side);
    for (void* ptr : allocs) (void)hipFree(ptr);
    if (host_sc) (void)hipHostFree(host_sc);
    if (host_bad) (void)hipHostFree(host_bad);
    if (blas) rocblas_destroy_handle(blas);
    if (ctx) {
      std::lock_guard<std::mutex> lock(ctx->mu);
      ctx->used -= std::min(ctx->used, bytes);
    }
  }

  int nlevels() const { return int(H.size()); }

  TabView tabview() const { return TabView{tab_off, dg_off, w_off, dface_off, gl_off}; }

  template <typename T>
  LevelView<T> view(int l) const;
  template <typename T>
  TransferView<T> tview(int l) const;  // between level l (fine) and l + 1
  template <typename T>
  DevLevel<T>& lev(int l);
  template <typename T>
  const T* table() const;
};

template <>
DevLevel<double>& hpdg_mesh::lev<double>(int l) { return L64[l]; }
template <>
DevLevel<float>& hpdg_mesh::lev<float>(int l) { return L32[l]; }
template <>
const double* hpdg_mesh::table<double>() const { return tab64; }
template <>
const float* hpdg_mesh::table<float>() const { return tab32; }

template <typename T>
LevelView<T> hpdg_mesh::view(int l) const {
  const LevelHost& h = H[l];
  const DevLevel<T>& d = const_cast<hpdg_mesh*>(this)->lev<T>(l);
  LevelView<T> v;
  v.einfo = d.einfo;
  v.minfo = d.minfo;
  v.fmlist = d.fmlist;
  v.mtask = d.mtask;
  v.n_mtask = (long long)h.mtask.size();
  v.vgeo = d.vgeo;
  v.mgeo = d.mgeo;
  v.mcoef = mass_on ? d.mcoef : nullptr;
  v.flink = d.flink;
  v.fe_off = d.fe_off;
  v.fe_toff = d.fe_toff;
  v.fe_g = d.fe_g;
  v.fe_id = d.felems;
  v.fcoef = d.fcoef;
  v.trace = d.trace;
  v.slot = d.slot;
  v.tab = table<T>();
  v.tv = tabview();
  v.n_elem = (long long)h.cells.size();
  v.nmax = h.nmax;
  v.qmax = h.qmax;
  v.qmmax = std::max(h.qmmax, 1);
  v.self_only = 0;
  return v;
}

template <typename T>
TransferView<T> hpdg_mesh::tview(int l) const {
  const DevLevel<T>& d = const_cast<hpdg_mesh*>(this)->lev<T>(l);
  TransferView<T> v;
  v.tinfo = d.tinfo;
  v.cstart = d.cstart;
  v.clist = d.clist;
  v.tab = table<T>();
  v.tv = tabview();
  v.n_fine = (long long)H[l].cells.size();
  v.n_coarse = (long long)H[l + 1].cells.size();
  v.nmax = std::max(H[l].nmax, H[l + 1].nmax);
  return v;
}

namespace {

// message of the last failed call of the calling thread (the server's worker threads and the
// caller's threads do not overwrite each other's messages)
thread_local std::string t_last_error = "no error";

int fail(hpdg_ctx* ctx, int code, const std::string& msg) {
  (void)ctx;
  t_last_error = msg.empty() ? "error " + std::to_string(code) : msg;
  return code;
}

template <typename F>
int guarded(hpdg_ctx* ctx, F&& f) {
  try {
    f();
    return HPDG_OK;
  } catch (const Error& e) {
    return fail(ctx, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, HPDG_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, HPDG_ERR_INVALID_ARG, e.what());
  }
}

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

template <typename T>
void build_device_level(hpdg_mesh* M, int l, hipStream_t s) {
  LevelHost& h = M->H[l];
  DevLevel<T>& d = M->lev<T>(l);
  d.einfo = M->upload_raw(h.einfo, s);
  d.minfo = M->upload_raw(h.minfo, s);
  d.fmlist = M->upload_raw(h.fmlist, s);
  d.mtask = M->upload_raw(h.mtask, s);
  d.belems = M->upload_raw(h.bucket_elems, s);
  d.felems = M->upload_raw(h.fast_elems, s);
  d.telems = M->upload_raw(h.trace_elems, s);
  d.flink = M->upload_raw(h.flink, s);
  d.fe_off = M->upload_raw(h.fast_off, s);
  d.fe_toff = M->upload_raw(h.fast_toff, s);
  d.fe_g = M->upload<T>(h.fast_g, s);
  d.fcoef = M->upload<T>(h.fcoef, s);
  d.vgeo = M->upload<T>(h.vgeo, s);
  d.mgeo = M->upload<T>(h.mgeo, s);
  std::vector<double> dinv(h.diag.size());
  for (size_t i = 0; i < dinv.size(); ++i) dinv[i] = 1.0 / h.diag[i];
  d.dinv = M->upload<T>(dinv, s);
  if (l + 1 < M->nlevels()) {
    d.tinfo = M->upload_raw(h.tinfo, s);
    d.cstart = M->upload_raw(h.cstart, s);
    d.clist = M->upload_raw(h.clist, s);
  }
  if (h.nmq > 0) {
    d.mcoef = M->alloc<T>(size_t(h.nmq));
    launch_fill<T>(h.nmq, T(0), d.mcoef, s);
    d.diag = M->upload<T>(h.diag, s);
  }
  d.trace = M->alloc<T>(size_t(h.ntrace));
  d.slot = M->alloc<T>(size_t(h.nslot));
  const size_t n = size_t(h.ndof);
  d.f = M->alloc<T>(n);
  d.v = M->alloc<T>(n);
  d.t = M->alloc<T>(n);
  d.p = M->alloc<T>(n);
}

// ---- kernel timing ----------------------------------------------------------------
hipEvent_t take_event(hpdg_mesh* M) {
  if (!M->event_pool.empty()) {
    hipEvent_t e = M->event_pool.back();
    M->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// run f() between two events on s when timing is enabled
template <typename F>
void timed(hpdg_mesh* M, int kind, int level, int prec, double bytes, hipStream_t s, F&& f) {
  if (!M->timing || level >= 32 || (M->timing_count[kind][level][prec]++ % M->timing_every) != 0) {
    f();
    return;
  }
  hipEvent_t a = take_event(M);
  HIPCHK(hipEventRecord(a, s));
  f();
  hipEvent_t b = take_event(M);
  HIPCHK(hipEventRecord(b, s));
  M->pending.push_back({a, b, kind, level, prec, bytes});
}

void collect_timing(hpdg_mesh* M) {
  for (auto& t : M->pending) {
    HIPCHK(hipEventSynchronize(t.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
    hpdg_mesh::Acc& a = M->acc[t.kind][t.level][t.prec];
    a.ms += ms;
    a.bytes += t.bytes;
    a.calls += 1;
    M->event_pool.push_back(t.a);
    M->event_pool.push_back(t.b);
  }
  M->pending.clear();
}

// algorithmic bytes of one apply of level l: x read and y written once, the stored metric once,
// the records once (element records of the element kernel's elements, the element-centric
// records of the others, mortar tasks)
double apply_bytes(const hpdg_mesh* M, int l, size_t scalar) {
  const LevelHost& h = M->H[l];
  return double(scalar) * (2.0 * double(h.ndof) + double(h.vgeo.size()) + double(h.mgeo.size()) +
                           double(h.fcoef.size()) + double(h.fast_g.size())) +
         double(h.bucket_elems.size() * sizeof(ElemInfo) + h.mtask.size() * sizeof(MortarTask) +
                h.fast_elems.size() * (6 * sizeof(FaceLink) + sizeof(long long)));
}

// group b of level l's element-centric apply
template <typename T>
FastBucket<T> fast_bucket(const hpdg_mesh* M, int l, size_t b) {
  const LevelHost& h = M->H[l];
  const int n = h.fast_n[b];
  const T* tb = M->table<T>();
  return FastBucket<T>{n, h.fast_nx[b], h.fast_start[b], h.fast_start[b + 1] - h.fast_start[b],
                       tb + M->tab.index(OpTable::MASS1, n, n), tb + M->tab.index(OpTable::STIFF1, n, n),
                       tb + M->tab.dface_off[n]};
}

// y = A_l x through the view V (whose trace and slot buffers are used): the face traces that the
// mortar kernel reads and the mortar kernel (faces left to it), then the element-centric apply of
// the fast elements and the element kernel of the others
// run slow(ss) on the mesh's side stream and fast(s) on s, both after the work enqueued on s so
// far, s continuing after both (when the level has work of both kinds; else both on s)
template <typename FS, typename FF>
void side_by_side(hpdg_mesh* M, bool both, hipStream_t s, FS&& slow, FF&& fast) {
  if (!both) {
    slow(s);
    fast(s);
    return;
  }
  if (!M->side) {
    HIPCHK(hipStreamCreateWithFlags(&M->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&M->fork_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&M->join_ev, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(M->fork_ev, s));
  HIPCHK(hipStreamWaitEvent(M->side, M->fork_ev, 0));
  slow(M->side);
  HIPCHK(hipEventRecord(M->join_ev, M->side));
  fast(s);
  HIPCHK(hipStreamWaitEvent(s, M->join_ev, 0));
}

// y = A_l x through the view V; ``overlap``: the element kernel's buckets on the side stream
template <typename T>
void level_apply(hpdg_mesh* M, int l, const LevelView<T>& V, const T* x, T* y, hipStream_t s, bool overlap = true) {
  const LevelHost& h = M->H[l];
  DevLevel<T>& d = M->lev<T>(l);
  if (!h.mtask.empty()) {
    launch_traces<T>(V, x, s, d.telems, (long long)h.trace_elems.size());
    launch_faces<T>(V, s);
  }
  side_by_side(
      M, overlap && !h.fast_n.empty() && !h.bucket_n.empty(), s,
      [&](hipStream_t ss) {
        for (size_t b = 0; b < h.bucket_n.size(); ++b)
          launch_apply_bucket<T>(V, h.bucket_n[b], h.bucket_q[b], d.belems + h.bucket_start[b],
                                 h.bucket_start[b + 1] - h.bucket_start[b], x, y, ss);
      },
      [&](hipStream_t ss) {
        for (size_t b = h.fast_n.size(); b-- > 0;) launch_fast_apply<T>(V, fast_bucket<T>(M, l, b), x, y, ss);
      });
}

template <typename T>
void apply_level(hpdg_mesh* M, int l, const T* x, T* y, hipStream_t s) {
  const int prec = sizeof(T) == 4 ? HPDG_F32 : HPDG_F64;
  const LevelView<T> V = M->view<T>(l);
  timed(M, HPDG_TIMING_APPLY, l, prec, M->timing ? apply_bytes(M, l, sizeof(T)) : 0.0, s,
        [&] { level_apply<T>(M, l, V, x, y, s); });
}

// the apply of level l with the face traces and the face slots in the caller-free scratch
// ``trace`` and ``slot`` (no timing, no allocation)
template <typename T>
void apply_level_scratch(hpdg_mesh* M, int l, const T* x, T* y, T* trace, T* slot, hipStream_t s) {
  LevelView<T> V = M->view<T>(l);
  V.trace = trace;
  V.slot = slot;
  level_apply<T>(M, l, V, x, y, s, false);
}

// Alg. schwarz_smoother on level l (FP64, or FP32 with the FP32 copies of the stored rows):
// n_iter times r = b - A x, x += sum_s R_s^T W_s A_ss^-1 R_s r (zero: x == 0 on entry, so the
// first residual is b)
template <typename T>
void schwarz_smooth(hpdg_mesh* M, int l, const T* b, T* x, int n_iter, bool zero, hipStream_t s) {
  const hpdg_mesh::SchwarzDev& w = M->sw.at(size_t(l));
  if (!w.minv) throw Error(HPDG_ERR_INVALID_ARG, "Schwarz smoother not set up on this level");
  const T* rows = w.rows(static_cast<T*>(nullptr));
  T* corr = w.corr(static_cast<T*>(nullptr));
  if (!rows) throw Error(HPDG_ERR_UNSUPPORTED, "FP32 Schwarz smoothing needs a mesh built with FP32 levels");
  DevLevel<T>& d = M->lev<T>(l);
  const long long n = M->H[l].ndof;
  const int prec = sizeof(T) == 4 ? HPDG_F32 : HPDG_F64;
  for (int k = 0; k < n_iter; ++k) {
    const T* r = b;
    if (!(zero && k == 0)) {
      apply_level<T>(M, l, x, d.t, s);
      launch_axpby<T>(n, T(1), b, T(-1), d.t, s);  // t = b - A x
      r = d.t;
    }
    timed(M, HPDG_TIMING_SCHWARZ, l, prec, sizeof(T) == 4 ? w.alg_bytes32 : w.alg_bytes, s, [&] {
      launch_schwarz_local<T>(w.n_sub, w.max_m, w.max_nw, r, w.gidx, w.goff, w.woff, w.offs(static_cast<T*>(nullptr)),
                              rows, corr, s);
    });
    launch_schwarz_scatter<T>(n, w.ptr, w.list, corr, x, s);
  }
}

// Alg. 4 with frozen lambda on level l: x <- x + Chebyshev correction (zero: x == 0 on entry)
template <typename T>
void smooth_level(hpdg_mesh* M, int l, const T* b, T* x, int n_iter, bool zero, hipStream_t s) {
  if (M->sp.scaling == HPDG_SMOOTH_SCHWARZ) {
    schwarz_smooth<T>(M, l, b, x, n_iter, zero, s);
    return;
  }
  DevLevel<T>& d = M->lev<T>(l);
  const long long n = M->H[l].ndof;
  const double lmax = M->lam[l];
  const double lmin = lmax / M->sp.Lambda;
  const double c = 0.5 * (lmax - lmin), dd = 0.5 * (lmax + lmin);
  double alpha = 0;
  const T* dinv = M->sp.scaling == HPDG_SMOOTH_POINT ? d.dinv : nullptr;
  const bool block = M->sp.scaling == HPDG_SMOOTH_BLOCK;
  const bool bf16 = std::is_same<T, float>::value && M->bf16_blocks && d.binv16;
  const LevelHost& h = M->H[l];
  const bool has_fast = !h.fast_n.empty();
  // levels without element-centric elements: the element kernel's fused step (block or point)
  bool fuse = !has_fast && ((block && !bf16) || dinv) && !M->sp.unfused && !h.bucket_n.empty();
  for (size_t bk = 0; fuse && bk < h.bucket_n.size(); ++bk)
    fuse = apply_block_fusable(h.bucket_n[bk], h.bucket_q[bk]);
  // levels with element-centric elements: fused point-Jacobi steps that write the new iterate to
  // the other of two vectors (x and the level's temporary), since neighbours read x during the
  // launch; the level's other elements take the element kernel's fused step with the same output
  bool fuse_ec = has_fast && dinv && !M->sp.unfused;
  for (size_t bk = 0; fuse_ec && bk < h.bucket_n.size(); ++bk)
    fuse_ec = apply_block_fusable(h.bucket_n[bk], h.bucket_q[bk]);
  const int prec = sizeof(T) == 4 ? HPDG_F32 : HPDG_F64;
  if (fuse_ec) {
    const int fused = n_iter - (zero ? 1 : 0);
    T* buf[2] = {x, d.t};
    int cur = 0;  // buf[cur] holds the iterate; the last fused step writes buf[0] = x
    LevelView<T> V = M->view<T>(l);
    for (int k = 1; k <= n_iter; ++k) {
      if (k == 1)
        alpha = 1.0 / dd;
      else if (k == 2)
        alpha = 2.0 * dd / (2.0 * dd * dd - c * c);
      else
        alpha = 1.0 / (dd - alpha * c * c / 4.0);
      const double beta = alpha * dd - 1.0;
      if (zero && k == 1) {
        // x = 0: p = alpha dinv b, iterate p, placed so that the remaining steps end in x
        cur = fused % 2;
        launch_cheb_update<T>(n, b, nullptr, dinv, d.p, x, T(alpha), T(beta), 1, s, buf[cur]);
        continue;
      }
      const double bytes = M->timing ? apply_bytes(M, l, sizeof(T)) - double(sizeof(T)) * double(n) +
                                           double(sizeof(T)) * double(n) * (1 + 1 + (k == 1 ? 1 : 2) + 1)
                                     : 0.0;
      T* xi = buf[cur];
      T* xo = buf[1 - cur];
      const FastStep<T> st{dinv, b, d.p, xo, T(alpha), T(beta), k == 1 ? 1 : 0};
      const BlockStep<T> bs{dinv, d.poff, d.binv, b, d.p, xi, nullptr, T(alpha), T(beta), k == 1 ? 1 : 0, xo};
      timed(M, HPDG_TIMING_SMOOTH, l, prec, bytes, s, [&] {
        if (!h.mtask.empty()) {
          launch_traces<T>(V, xi, s, d.telems, (long long)h.trace_elems.size());
          launch_faces<T>(V, s);
        }
        side_by_side(
            M, !h.bucket_n.empty(), s,
            [&](hipStream_t ss) {
              for (size_t bk = 0; bk < h.bucket_n.size(); ++bk)
                launch_apply_block_cheb<T>(V, h.bucket_n[bk], h.bucket_q[bk], d.belems + h.bucket_start[bk],
                                           h.bucket_start[bk + 1] - h.bucket_start[bk], xi, bs, ss);
            },
            [&](hipStream_t ss) {
              for (size_t bk = h.fast_n.size(); bk-- > 0;)
                launch_fast_cheb<T>(V, fast_bucket<T>(M, l, bk), xi, st, ss);
            });
      });
      cur = 1 - cur;
    }
    if (cur != 0) launch_copy<T>(n, buf[cur], x, s);
    return;
  }
  // fused steps write the traces of their result for the next fused step, alternating between
  // the level's two trace buffers (a step reads one while its neighbours' new traces go to the
  // other); ``cur`` holds the traces of x when they are current, else null
  T* cur = nullptr;
  for (int k = 1; k <= n_iter; ++k) {
    if (k == 1)
      alpha = 1.0 / dd;
    else if (k == 2)
      alpha = 2.0 * dd / (2.0 * dd * dd - c * c);
    else
      alpha = 1.0 / (dd - alpha * c * c / 4.0);
    const double beta = alpha * dd - 1.0;
    if (fuse && !(zero && k == 1)) {
      // the apply without its y write; packed blocks (or the inverse diagonal), b, p (read after the
      // first step, written), x written
      const double scaling = double(sizeof(T)) * (dinv ? double(n) : double(M->block_scalars[l]));
      const double bytes = M->timing ? apply_bytes(M, l, sizeof(T)) - double(sizeof(T)) * double(n) + scaling +
                                           double(sizeof(T)) * double(n) * (1 + (k == 1 ? 1 : 2) + 1)
                                     : 0.0;
      LevelView<T> V = M->view<T>(l);
      if (!cur) {
        launch_traces<T>(V, x, s);
        cur = d.trace;
      }
      V.trace = cur;
      T* next = k < n_iter ? (cur == d.trace ? d.trace2 : d.trace) : nullptr;
      const BlockStep<T> bs{dinv, d.poff, d.binv, b, d.p, x, next, T(alpha), T(beta), k == 1 ? 1 : 0, nullptr};
      timed(M, HPDG_TIMING_SMOOTH, l, prec, bytes, s, [&] {
        launch_faces<T>(V, s);
        for (size_t bk = 0; bk < h.bucket_n.size(); ++bk)
          launch_apply_block_cheb<T>(V, h.bucket_n[bk], h.bucket_q[bk], M->lev<T>(l).belems + h.bucket_start[bk],
                                     h.bucket_start[bk + 1] - h.bucket_start[bk], x, bs, s);
      });
      cur = next;
      continue;
    }
    cur = nullptr;
    const T* Ax = nullptr;
    if (!(zero && k == 1)) {
      apply_level<T>(M, l, x, d.t, s);
      Ax = d.t;
    }
    if (block) {
      // inverse blocks, b, Ax (when given), p (read after the first step, written), x (read, written)
      const double vec = double(n) * (1 + (Ax ? 1 : 0) + (k == 1 ? 1 : 2) + 2);
      const double stored = bf16 ? 2.0 * double(M->block_full_scalars[l]) : double(sizeof(T)) * double(M->block_scalars[l]);
      const double bytes = M->timing ? stored + double(sizeof(T)) * vec : 0.0;
      timed(M, HPDG_TIMING_BLOCK, l, prec, bytes, s, [&] {
        if constexpr (std::is_same<T, float>::value) {
          if (bf16) {
            launch_block_cheb_bf16(M->view<float>(l), d.boff16, d.binv16, b, Ax, d.p, x, float(alpha), float(beta),
                                   k == 1 ? 1 : 0, s);
            return;
          }
        }
        launch_block_cheb<T, T>(M->view<T>(l), d.poff, d.binv, b, Ax, d.p, x, T(alpha), T(beta), k == 1 ? 1 : 0,
                                s);
      });
    } else
      launch_cheb_update<T>(n, b, Ax, dinv, d.p, x, T(alpha), T(beta), k == 1 ? 1 : 0, s);
  }
}

// exact coarse solve v = A_L^-1 f through the FP64 inverse; FP32 vectors (mixed V-cycle) are
// widened to FP64 for the mat-vec and rounded back, so the coarse solve itself stays FP64
template <typename T>
void coarse_solve(hpdg_mesh* M, const T* f, T* v, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    launch_dense_matvec<double>(M->ncoarse, M->Ainv64, f, v, s);
  } else {
    DevLevel<double>& d = M->lev<double>(M->nlevels() - 1);
    launch_convert_f2d(M->ncoarse, f, d.f, s);
    launch_dense_matvec<double>(M->ncoarse, M->Ainv64, d.f, d.v, s);
    launch_convert_d2f(M->ncoarse, d.v, v, s);
  }
}

// Alg. 3: z = V(r) on level-0 vectors of type T
template <typename T>
void vcycle(hpdg_mesh* M, const T* r0, T* z0, hipStream_t s) {
  const int L = M->nlevels() - 1;
  auto nc = [&](int l) { return l > 0 && M->sp.n_cheb_coarse > 0 ? M->sp.n_cheb_coarse : M->sp.n_cheb; };
  std::vector<const T*> f(L + 1);
  std::vector<T*> v(L + 1);
  for (int l = 0; l <= L; ++l) {
    f[l] = l == 0 ? r0 : M->lev<T>(l).f;
    v[l] = l == 0 ? z0 : M->lev<T>(l).v;
  }
  for (int l = 0; l < L; ++l) {
    DevLevel<T>& d = M->lev<T>(l);
    const long long n = M->H[l].ndof;
    launch_fill<T>(n, T(0), v[l], s);
    smooth_level<T>(M, l, f[l], v[l], nc(l), true, s);
    apply_level<T>(M, l, v[l], d.t, s);
    launch_axpby<T>(n, T(1), f[l], T(-1), d.t, s);  // t = f - A v
    launch_restrict<T>(M->tview<T>(l), d.t, M->lev<T>(l + 1).f, s);
  }
  coarse_solve<T>(M, f[L], v[L], s);
  if (L == 0) return;
  for (int l = L - 1; l >= 0; --l) {
    launch_prolong_add<T>(M->tview<T>(l), v[l + 1], v[l], s);
    smooth_level<T>(M, l, f[l], v[l], nc(l), false, s);
  }
}

// host-side dot (synchronising); used at setup and by PCG
double dot_sync(hpdg_mesh* M, long long n, const double* a, const double* b, hipStream_t s) {
  launch_dot(n, a, b, M->partials, M->sc + 12, s);
  HIPCHK(hipMemcpyAsync(M->host_sc + 12, M->sc + 12, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return M->host_sc[12];
}

uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Alg. 5 on level l (FP64): returns the Gershgorin bound of the Lanczos tridiagonal
double cg_bound(hpdg_mesh* M, int l, int n_eigs, uint64_t seed, hipStream_t s) {
  DevLevel<double>& d = M->lev<double>(l);
  const long long n = M->H[l].ndof;
  std::vector<double> b(n);
  uint64_t st = seed;
  for (long long i = 0; i < n; ++i) b[i] = double(splitmix64(st) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
  // preconditioned CG with the smoother's M (x0 = 0): r = f, z = v, p = p, A p = t
  HIPCHK(hipMemcpyAsync(d.f, b.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  auto precond = [&](const double* r, double* z) {
    if (M->sp.scaling == HPDG_SMOOTH_POINT)
      launch_scale<double>(n, d.dinv, r, z, s);
    else if (M->sp.scaling == HPDG_SMOOTH_BLOCK)
      launch_block_apply<double, double>(M->view<double>(l), d.poff, d.binv, r, z, s);
    else
      launch_copy<double>(n, r, z, s);
  };
  precond(d.f, d.v);
  launch_copy<double>(n, d.v, d.p, s);
  double rz = dot_sync(M, n, d.f, d.v, s);
  std::vector<double> al, be;
  for (int k = 0; k < n_eigs; ++k) {
    apply_level<double>(M, l, d.p, d.t, s);
    const double pAp = dot_sync(M, n, d.p, d.t, s);
    const double alpha = rz / pAp;
    launch_axpby<double>(n, -alpha, d.t, 1.0, d.f, s);  // r -= alpha A p
    precond(d.f, d.v);
    const double rz2 = dot_sync(M, n, d.f, d.v, s);
    const double beta = rz2 / rz;
    al.push_back(alpha);
    be.push_back(beta);
    launch_axpby<double>(n, 1.0, d.v, beta, d.p, s);  // p = z + beta p
    rz = rz2;
    if (!(rz > 0)) break;
  }
  const int k = int(al.size());
  double bound = 0;
  for (int i = 0; i < k; ++i) {
    const double diag = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
    const double lo = i > 0 ? std::sqrt(be[i - 1]) / al[i - 1] : 0.0;
    const double hi = i + 1 < k ? std::sqrt(be[i]) / al[i] : 0.0;
    bound = std::max(bound, diag + lo + hi);
  }
  return bound;
}

void factor_blocks(hpdg_mesh* M, int l, const LevelView<double>& V, const std::vector<long long>& boff,
                   const long long* dboff, double* B, hipStream_t s);
std::string diagnose_block(hpdg_mesh* M, int l, const LevelView<double>& V, const std::vector<long long>& boff,
                           const long long* dboff, double* B, long long e, hipStream_t s);

// a batched element-block factorisation reported a non-positive pivot in element ``elem``
struct BlockFailure : Error {
  long long elem;
  BlockFailure(const std::string& m, long long e) : Error(HPDG_ERR_BREAKDOWN, m), elem(e) {}
};

// element-block Jacobi: A_ee of every element of level l (column j of all blocks from one
// apply with neighbours taken as zero), their inverses by batched Cholesky (rocSOLVER), and
// the lower triangles of the inverses packed (FP64, and FP32 for FP32 levels; the bf16 copies
// for FP32 levels are full blocks, read row per thread). The full FP64 blocks exist during
// setup only.
void build_blocks(hpdg_mesh* M, int l, hipStream_t s) {
  DevLevel<double>& d = M->lev<double>(l);
  if (d.binv) return;
  const LevelHost& h = M->H[l];
  const size_t E = h.cells.size();
  std::vector<long long> boff(E + 1, 0), poff(E + 1, 0);
  for (size_t e = 0; e < E; ++e) {
    const long long N = (long long)h.einfo[e].n * h.einfo[e].n * h.einfo[e].n;
    boff[e + 1] = boff[e] + N * N;
    poff[e + 1] = poff[e] + N * (N + 1) / 2;
  }
  M->block_scalars[l] = poff[E];
  M->block_full_scalars[l] = boff[E];
  long long* dboff = M->upload_raw(boff, s);
  double* B = M->alloc<double>(size_t(boff[E]));
  LevelView<double> V = M->view<double>(l);
  V.self_only = 1;
  // A failed factorisation is retried once from a fresh gather (the blocks are SPD: a
  // failure that does not repeat is not a property of the operator); a repeated one is an error.
  // Each failure is reported on stderr with a host check of the re-gathered block, which tells
  // bad block data (not SPD on the host) from a failed device factorisation (SPD on the host),
  // and counted (hpdg_mesh_info.block_retries).
  for (int attempt = 0;; ++attempt) {
    try {
      factor_blocks(M, l, V, boff, dboff, B, s);
      break;
    } catch (const BlockFailure& err) {
      const std::string diag = diagnose_block(M, l, V, boff, dboff, B, err.elem, s);
      std::fprintf(stderr, "hpdg: %s; %s\n", err.what(), diag.c_str());
      if (attempt >= 1) throw Error(HPDG_ERR_BREAKDOWN, std::string(err.what()) + "; " + diag);
      M->block_retries += 1;
    }
  }
  d.poff = M->upload_raw(poff, s);
  d.binv = M->alloc<double>(size_t(poff[E]));
  launch_pack_blocks<double>(V, dboff, B, d.poff, d.binv, s);
  if (M->has_f32) {
    DevLevel<float>& d32 = M->lev<float>(l);
    d32.poff = d.poff;
    d32.binv = M->alloc<float>(size_t(poff[E]));
    launch_pack_blocks<float>(V, dboff, B, d.poff, d32.binv, s);
    d32.boff16 = dboff;
    d32.binv16 = M->alloc<uint16_t>(size_t(boff[E]));
    launch_blocks_bf16_full(V, dboff, B, d32.binv16, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  M->release(B);
  if (!M->has_f32) M->release(dboff);
}

// gather the element blocks of level l: column j of every block from one self-only apply
void gather_blocks(hpdg_mesh* M, int l, const LevelView<double>& V, const long long* dboff, double* B,
                   hipStream_t s) {
  DevLevel<double>& d = M->lev<double>(l);
  const LevelHost& h = M->H[l];
  launch_fill<double>(h.ndof, 0.0, d.f, s);
  const int nmax3 = h.nmax * h.nmax * h.nmax;
  for (int j = 0; j < nmax3; ++j) {
    launch_set_unit<double>(V, j, 1.0, d.f, s);
    level_apply<double>(M, l, V, d.f, d.t, s);
    launch_gather_column<double>(V, j, d.t, dboff, B, s);
    launch_set_unit<double>(V, j, 0.0, d.f, s);
  }
}

// after a failed factorisation of element e's block: gather the blocks again, copy e's to the
// host and factorise it there (plain Cholesky); returns a one-line finding
std::string diagnose_block(hpdg_mesh* M, int l, const LevelView<double>& V, const std::vector<long long>& boff,
                           const long long* dboff, double* B, long long e, hipStream_t s) {
  if (e < 0 || e + 1 >= (long long)boff.size()) return "no element to check";
  try {
    gather_blocks(M, l, V, dboff, B, s);
    const long long N2 = boff[e + 1] - boff[e];
    const int N = int(std::llround(std::sqrt(double(N2))));
    std::vector<double> A(static_cast<size_t>(N2));
    HIPCHK(hipMemcpyAsync(A.data(), B + boff[e], size_t(N2) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double asym = 0, scale = 0;
    for (int i = 0; i < N; ++i) {
      scale = std::max(scale, std::fabs(A[size_t(i) * N + i]));
      for (int j = 0; j < i; ++j) asym = std::max(asym, std::fabs(A[size_t(i) * N + j] - A[size_t(j) * N + i]));
    }
    // in-place lower Cholesky of the symmetric part
    double minpiv = std::numeric_limits<double>::infinity();
    int fail_at = -1;
    for (int j = 0; j < N && fail_at < 0; ++j) {
      double dj = A[size_t(j) * N + j];
      for (int k = 0; k < j; ++k) dj -= A[size_t(j) * N + k] * A[size_t(j) * N + k];
      minpiv = std::min(minpiv, dj);
      if (!(dj > 0)) {
        fail_at = j;
        break;
      }
      const double ljj = std::sqrt(dj);
      A[size_t(j) * N + j] = ljj;
      for (int i = j + 1; i < N; ++i) {
        double v = 0.5 * (A[size_t(i) * N + j] + A[size_t(j) * N + i]);
        for (int k = 0; k < j; ++k) v -= A[size_t(i) * N + k] * A[size_t(j) * N + k];
        A[size_t(i) * N + j] = v / ljj;
      }
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "re-gathered block of element %lld (N %d): host Cholesky %s (smallest pivot %.3e, "
                  "largest diagonal %.3e, asymmetry %.3e)",
                  e, N, fail_at < 0 ? "succeeds" : ("fails at column " + std::to_string(fail_at)).c_str(), minpiv,
                  scale, asym);
    return buf;
  } catch (const std::exception& x) {
    return std::string("the check of the re-gathered block failed: ") + x.what();
  }
}

// gather the element blocks of level l, check them, and replace them by their inverses
// (batched Cholesky + inverse, rocSOLVER)
void factor_blocks(hpdg_mesh* M, int l, const LevelView<double>& V, const std::vector<long long>& boff,
                   const long long* dboff, double* B, hipStream_t s) {
  DevLevel<double>& d = M->lev<double>(l);
  const LevelHost& h = M->H[l];
  const size_t E = h.cells.size();
  gather_blocks(M, l, V, dboff, B, s);
  {
    int* bad = nullptr;
    HIPCHK(hipMalloc(&bad, E * sizeof(int)));
    launch_check_blocks(V, dboff, B, d.dinv, bad, s);
    std::vector<int> hb(E);
    HIPCHK(hipMemcpyAsync(hb.data(), bad, E * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    (void)hipFree(bad);
    for (size_t e = 0; e < E; ++e)
      if (hb[e])
        throw Error(HPDG_ERR_HIP, "element block " + std::to_string(e) + " on level " + std::to_string(l) +
                                      ": gathered column " + std::to_string(hb[e] - 1) +
                                      " is inconsistent with the operator diagonal / symmetry");
  }
  if (!M->blas) {
    if (rocblas_create_handle(&M->blas) != rocblas_status_success) throw Error(HPDG_ERR_HIP, "rocblas handle");
  }
  rocblas_set_stream(M->blas, s);
  // batched Cholesky + inverse, one call per block size
  std::vector<int> sizes;
  for (size_t e = 0; e < E; ++e) sizes.push_back(h.einfo[e].n);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  for (int n : sizes) {
    const int N = n * n * n;
    std::vector<double*> ptrs;
    std::vector<long long> eids;
    for (size_t e = 0; e < E; ++e)
      if (h.einfo[e].n == n) {
        ptrs.push_back(B + boff[e]);
        eids.push_back((long long)e);
      }
    const int cnt = int(ptrs.size());
    double** dptrs = nullptr;
    rocblas_int* info = nullptr;
    HIPCHK(hipMalloc(&dptrs, cnt * sizeof(double*)));
    HIPCHK(hipMalloc(&info, cnt * sizeof(rocblas_int)));
    HIPCHK(hipMemcpyAsync(dptrs, ptrs.data(), cnt * sizeof(double*), hipMemcpyHostToDevice, s));
    std::vector<rocblas_int> hinfo(cnt);
    // status of a batched call and its per-block info: the first failing block is reported
    auto check = [&](rocblas_status st, const char* what) {
      HIPCHK(hipMemcpyAsync(hinfo.data(), info, cnt * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (st != rocblas_status_success) {
        (void)hipFree(dptrs);
        (void)hipFree(info);
        throw Error(HPDG_ERR_HIP, std::string(what) + " failed with rocblas status " + std::to_string(int(st)) +
                                      " (level " + std::to_string(l) + ", block size " + std::to_string(N) +
                                      ", " + std::to_string(cnt) + " blocks)");
      }
      for (int b = 0; b < cnt; ++b)
        if (hinfo[b] != 0) {
          (void)hipFree(dptrs);
          (void)hipFree(info);
          throw BlockFailure(std::string(what) + ": the block of element " + std::to_string(eids[b]) +
                                 " (size " + std::to_string(N) + ", level " + std::to_string(l) +
                                 ") is not positive definite (info " + std::to_string(hinfo[b]) + ")",
                             eids[b]);
        }
    };
    check(rocsolver_dpotrf_batched(M->blas, rocblas_fill_lower, N, dptrs, N, info, cnt), "Cholesky");
    check(rocsolver_dpotri_batched(M->blas, rocblas_fill_lower, N, dptrs, N, info, cnt), "inverse");
    (void)hipFree(dptrs);
    (void)hipFree(info);
  }
  HIPCHK(hipStreamSynchronize(s));
}

// additive Schwarz smoother of level l (Alg. schwarz_smoother, Eq. schwarz_weight): the
// subdomains (schwarz_layout), the operator blocks A_ab of every element b and its face
// neighbours a (SIPG couples no other pairs), gathered column by column from applies to unit
// vectors on the elements of one colour of a distance-2 colouring of the face graph (no two
// elements of a colour share a neighbour, so each neighbour's rows come from one of them), each
// subdomain's A_ss assembled from the blocks (all on the device; the host builds the layout and
// the slot tables), inverted (batched Cholesky + inverse, rocSOLVER, per subdomain size), and
// the weighted rows kept (FP64, and FP32 for meshes with FP32 levels)
void build_schwarz(hpdg_mesh* M, int l, hipStream_t s) {
  hpdg_mesh::SchwarzDev& W = M->sw[size_t(l)];
  if (W.minv && W.overlap == M->sp.schwarz_overlap) return;
  const LevelHost& h = M->H[l];
  SchwarzLayout lay;
  schwarz_layout(M->mm, h, M->sp.schwarz_overlap, lay);
  const int E = int(h.cells.size());
  const int n3max = lay.n * lay.n * lay.n;
  std::vector<int> en3(static_cast<size_t>(E));
  for (int e = 0; e < E; ++e) en3[e] = lay.en[e] * lay.en[e] * lay.en[e];
  int max_m = 0, max_nw = 0;
  long long minv_scalars = 0, minv32_scalars = 0, alg_scalars = 0, nrows = 0;
  for (int c = 0; c < E; ++c) {
    const int m = int(lay.off[c + 1] - lay.off[c]);
    max_m = std::max(max_m, m);
    max_nw = std::max(max_nw, lay.nw[c]);
    minv_scalars += (long long)lay.nw[c] * schwarz_stride(m, 8);  // rows padded to the vector width
    minv32_scalars += (long long)lay.nw[c] * schwarz_stride(m, 4);
    alg_scalars += (long long)lay.nw[c] * m;
    nrows += lay.nw[c];
  }
  if (size_t(schwarz_stride(max_m, 8)) * sizeof(double) > 64 * 1024)
    throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz subdomains of more than 8190 points");
  const std::vector<long long>& AS = lay.adj_start;
  const std::vector<int>& AJ = lay.adj;
  // operator blocks: element b, slot k (0: b itself, 1 + t: its t-th coupled element a), n3_a x
  // n3_b column-major at boff[sstart[b] + k]
  std::vector<long long> sstart(size_t(E) + 1, 0), boff;
  int max_slots = 1;
  size_t blk_size = 0;
  for (int b = 0; b < E; ++b) {
    const int deg = int(AS[b + 1] - AS[b]);
    max_slots = std::max(max_slots, 1 + deg);
    sstart[b + 1] = sstart[b] + 1 + deg;
    for (int k = 0; k <= deg; ++k) {
      const int a = k == 0 ? b : AJ[size_t(AS[b] + k - 1)];
      if (a < 0 || a >= E) throw Error(HPDG_ERR_HIP, "Schwarz setup: coupled element out of range");
      boff.push_back((long long)blk_size);
      blk_size += size_t(en3[a]) * en3[b];
    }
  }
  if (double(blk_size) * sizeof(double) > 16.0 * (1ull << 30))
    throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz setup: operator blocks above 16 GiB");
  // distance-2 colouring of the coupling graph (greedy, element order)
  std::vector<int> color(E, -1);
  int ncol = 0;
  {
    std::vector<int> seen;
    for (int e = 0; e < E; ++e) {
      seen.clear();
      for (long long t = AS[e]; t < AS[e + 1]; ++t) {
        const int a = AJ[size_t(t)];
        seen.push_back(color[a]);
        for (long long u = AS[a]; u < AS[a + 1]; ++u)
          if (AJ[size_t(u)] != e) seen.push_back(color[AJ[size_t(u)]]);
      }
      int c = 0;
      while (std::find(seen.begin(), seen.end(), c) != seen.end()) ++c;
      color[e] = c;
      ncol = std::max(ncol, c + 1);
    }
  }
  // the blocks, gathered on the device one colour and column at a time; kept there for the assembly
  double* dblk = nullptr;
  int* den3 = nullptr;
  long long* dboff = nullptr;
  long long* dsstart = nullptr;
  {
    DevLevel<double>& d = M->lev<double>(l);
    const LevelView<double> V = M->view<double>(l);
    std::vector<int> members;
    std::vector<int> cstart(size_t(ncol) + 1, 0);
    for (int c = 0; c < ncol; ++c) {
      for (int e = 0; e < E; ++e)
        if (color[e] == c) members.push_back(e);
      cstart[c + 1] = int(members.size());
    }
    std::vector<long long> eoff(static_cast<size_t>(E));
    for (int e = 0; e < E; ++e) eoff[e] = h.einfo[e].off;
    int* dmem = M->upload_raw(members, s);
    long long* das = M->upload_raw(AS, s);
    int* daj = M->upload_raw(AJ, s);
    long long* deoff = M->upload_raw(eoff, s);
    den3 = M->upload_raw(en3, s);
    dboff = M->upload_raw(boff, s);
    dsstart = M->upload_raw(sstart, s);
    dblk = M->alloc<double>(blk_size);
    launch_fill<double>((long long)blk_size, 0.0, dblk, s);
    launch_fill<double>(h.ndof, 0.0, d.f, s);
    for (int c = 0; c < ncol; ++c) {
      const int cnt = cstart[c + 1] - cstart[c];
      const int* mc = dmem + cstart[c];
      for (int j = 0; j < n3max; ++j) {
        launch_schwarz_units(cnt, mc, deoff, den3, j, 1.0, d.f, s);
        level_apply<double>(M, l, V, d.f, d.t, s);
        launch_schwarz_gather(cnt, max_slots, mc, das, daj, deoff, den3, dsstart, dboff, j, d.t, dblk, s);
        launch_schwarz_units(cnt, mc, deoff, den3, j, 0.0, d.f, s);
      }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    for (void* q : {(void*)dmem, (void*)das, (void*)daj, (void*)deoff}) M->release(q);
  }
  // device layout of the subdomains
  std::vector<int> gidx(lay.elem.size());
  for (size_t k = 0; k < gidx.size(); ++k) gidx[k] = int(h.einfo[lay.elem[k]].off + lay.loc[k]);
  std::vector<long long> woff(size_t(E) + 1, 0), moff(size_t(E) + 1, 0), moff32(size_t(E) + 1, 0);
  std::vector<double> wrow(static_cast<size_t>(nrows));
  for (int c = 0; c < E; ++c) {
    const int m = int(lay.off[c + 1] - lay.off[c]);
    woff[c + 1] = woff[c] + lay.nw[c];
    moff[c + 1] = moff[c] + (long long)lay.nw[c] * schwarz_stride(m, 8);
    moff32[c + 1] = moff32[c] + (long long)lay.nw[c] * schwarz_stride(m, 4);
    for (int r = 0; r < lay.nw[c]; ++r) wrow[size_t(woff[c] + r)] = lay.w[size_t(lay.off[c] + r)];
  }
  std::vector<long long> ptr(size_t(h.ndof) + 1, 0);
  for (int c = 0; c < E; ++c)
    for (int r = 0; r < lay.nw[c]; ++r) ptr[size_t(gidx[size_t(lay.off[c] + r)]) + 1] += 1;
  for (long long i = 0; i < h.ndof; ++i) ptr[size_t(i) + 1] += ptr[size_t(i)];
  std::vector<int> list(static_cast<size_t>(nrows));
  {
    std::vector<long long> fill(ptr.begin(), ptr.end() - 1);
    for (int c = 0; c < E; ++c)
      for (int r = 0; r < lay.nw[c]; ++r) list[size_t(fill[size_t(gidx[size_t(lay.off[c] + r)])]++)] = int(woff[c] + r);
  }
  for (void* q : {(void*)W.gidx, (void*)W.goff, (void*)W.woff, (void*)W.moff, (void*)W.ptr, (void*)W.list,
                  (void*)W.d, (void*)W.minv, (void*)W.minv32, (void*)W.d32, (void*)W.moff32})
    if (q) M->release(q);  // a previous overlap's
  W = hpdg_mesh::SchwarzDev{};
  W.n_sub = E;
  W.max_m = max_m;
  W.max_nw = max_nw;
  W.overlap = M->sp.schwarz_overlap;
  W.minv_scalars = minv_scalars;
  W.entries = (long long)gidx.size();
  W.alg_bytes = 8.0 * double(alg_scalars) + 12.0 * double(W.entries) + 8.0 * double(nrows) + 24.0 * double(E);
  W.alg_bytes32 = 4.0 * double(alg_scalars) + 8.0 * double(W.entries) + 4.0 * double(nrows) + 24.0 * double(E);
  W.gidx = M->upload_raw(gidx, s);
  W.goff = M->upload_raw(lay.off, s);
  W.woff = M->upload_raw(woff, s);
  W.moff = M->upload_raw(moff, s);
  W.ptr = M->upload_raw(ptr, s);
  W.list = M->upload_raw(list, s);
  W.d = M->alloc<double>(size_t(nrows));
  W.minv = M->alloc<double>(size_t(minv_scalars));
  if (M->has_f32) {  // rounded copies for the FP32 V-cycle, packed from the same inverses
    W.moff32 = M->upload_raw(moff32, s);
    W.minv32 = M->alloc<float>(size_t(minv32_scalars));
    W.d32 = M->alloc<float>(size_t(nrows));
  }
  double* dw = M->upload_raw(wrow, s);
  if (!M->blas) {
    if (rocblas_create_handle(&M->blas) != rocblas_status_success) throw Error(HPDG_ERR_HIP, "rocblas handle");
  }
  rocblas_set_stream(M->blas, s);
  // per subdomain size: assemble A_ss (column-major) on the host, invert on the device, pack
  // (chunks of at most 1 GiB of subdomain matrices)
  std::map<int, std::vector<std::vector<int>>> groups;
  for (int c = 0; c < E; ++c) {
    const int m = int(lay.off[c + 1] - lay.off[c]);
    const size_t cap = std::max<size_t>(1, (size_t(1) << 30) / (size_t(m) * m * sizeof(double)));
    std::vector<std::vector<int>>& chunks = groups[m];
    if (chunks.empty() || chunks.back().size() >= cap) chunks.emplace_back();
    chunks.back().push_back(c);
  }
  // one device buffer for the largest chunk, reused; A_ss assembled on the device from the blocks
  size_t stage = 0;
  for (const auto& g : groups)
    for (const std::vector<int>& subs : g.second) stage = std::max(stage, subs.size() * size_t(g.first) * g.first);
  double* dA = M->alloc<double>(stage);
  std::vector<unsigned char> lel;
  std::vector<int> els;
  std::vector<signed char> slot;
  schwarz_tables(lay, lel, els, slot);
  for (int c = 0; c < E; ++c)  // every coupled pair's slot exists among the column element's blocks
    for (int jb = 0; jb < kSchwarzMaxElems && els[size_t(c) * kSchwarzMaxElems + jb] >= 0; ++jb) {
      const int eb = els[size_t(c) * kSchwarzMaxElems + jb];
      for (int ia = 0; ia < kSchwarzMaxElems; ++ia) {
        const int k = slot[(size_t(c) * kSchwarzMaxElems + jb) * kSchwarzMaxElems + ia];
        if (k >= 0 && k > AS[eb + 1] - AS[eb]) throw Error(HPDG_ERR_HIP, "Schwarz setup: block slot out of range");
      }
    }
  std::vector<short> loc16(lay.loc.begin(), lay.loc.end());  // local indices < n^3 <= 4096
  unsigned char* dlel = M->upload_raw(lel, s);
  short* dloc = M->upload_raw(loc16, s);
  int* dels = M->upload_raw(els, s);
  signed char* dslot = M->upload_raw(slot, s);
  for (const auto& g : groups)
    for (const std::vector<int>& subs : g.second) {
    const int m = g.first;
    const int cnt = int(subs.size());
    int* dsubs = M->upload_raw(subs, s);
    launch_schwarz_assemble(m, cnt, dsubs, W.goff, dlel, dloc, dels, dslot, den3, dsstart, dboff, dblk, dA, s);
    HIPCHK(hipGetLastError());
    std::vector<double*> ptrs(cnt);
    std::vector<long long> pofs(cnt), gm(cnt), gm32(cnt), gw(cnt);
    std::vector<int> gnw(cnt);
    for (int b = 0; b < cnt; ++b) {
      ptrs[b] = dA + size_t(b) * m * m;
      pofs[b] = (long long)b * m * m;
      gm[b] = moff[subs[b]];
      gm32[b] = moff32[subs[b]];
      gw[b] = woff[subs[b]];
      gnw[b] = lay.nw[subs[b]];
    }
    double** dptrs = M->upload_raw(ptrs, s);
    rocblas_int* info = M->alloc<rocblas_int>(size_t(cnt));
    std::vector<rocblas_int> hinfo(cnt);
    auto check = [&](rocblas_status st, const char* what) {
      HIPCHK(hipMemcpyAsync(hinfo.data(), info, cnt * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (st != rocblas_status_success)
        throw Error(HPDG_ERR_HIP, std::string("Schwarz ") + what + " failed with rocblas status " + std::to_string(int(st)));
      for (int b = 0; b < cnt; ++b)
        if (hinfo[b] != 0)
          throw Error(HPDG_ERR_BREAKDOWN, std::string("Schwarz ") + what + ": the subdomain of element " +
                                              std::to_string(subs[b]) + " (level " + std::to_string(l) +
                                              ") is not positive definite");
    };
    check(rocsolver_dpotrf_batched(M->blas, rocblas_fill_lower, m, dptrs, m, info, cnt), "Cholesky");
    check(rocsolver_dpotri_batched(M->blas, rocblas_fill_lower, m, dptrs, m, info, cnt), "inverse");
    long long* dpofs = M->upload_raw(pofs, s);
    long long* dgm = M->upload_raw(gm, s);
    long long* dgw = M->upload_raw(gw, s);
    int* dgnw = M->upload_raw(gnw, s);
    launch_schwarz_pack<double>(m, cnt, dA, dpofs, dgm, dgnw, dgw, dw, W.minv, s);
    long long* dgm32 = nullptr;
    if (W.minv32) {
      dgm32 = M->upload_raw(gm32, s);
      launch_schwarz_pack<float>(m, cnt, dA, dpofs, dgm32, dgnw, dgw, dw, W.minv32, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    for (void* q : {(void*)dptrs, (void*)info, (void*)dpofs, (void*)dgm, (void*)dgw, (void*)dgnw, (void*)dgm32,
                    (void*)dsubs})
      if (q) M->release(q);
    }
  for (void* q : {(void*)dA, (void*)dblk, (void*)dlel, (void*)dloc, (void*)dels, (void*)dslot, (void*)den3,
                  (void*)dboff, (void*)dsstart})
    M->release(q);
  M->release(dw);

}

// exact coarse solve: the coarsest operator assembled column by column on the device (one
// apply per unit vector), symmetrised, factorised (Cholesky) and inverted with rocSOLVER;
// the explicit inverse is applied as a dense mat-vec in the V-cycle
void build_coarse_once(hpdg_mesh* M, hipStream_t s);
void build_coarse(hpdg_mesh* M, hipStream_t s) {
  // the operator is SPD: a failed factorisation that does not repeat on a fresh assembly is not
  // a property of the operator (as for the element blocks); a repeated one is an error
  for (int attempt = 0;; ++attempt) {
    try {
      build_coarse_once(M, s);
      return;
    } catch (const Error& err) {
      if (err.code != HPDG_ERR_BREAKDOWN) throw;
      std::fprintf(stderr, "hpdg: %s\n", err.what());
      if (attempt >= 1) throw;
      M->coarse_retries += 1;
    }
  }
}
void build_coarse_once(hpdg_mesh* M, hipStream_t s) {
  const int L = M->nlevels() - 1;
  if (M->H[L].ndof * M->H[L].ndof > (long long)std::numeric_limits<rocblas_int>::max())
    throw Error(HPDG_ERR_UNSUPPORTED, "the coarsest level has " + std::to_string(M->H[L].ndof) +
                                          " DOF: its dense matrix exceeds the 32-bit indexing of the dense "
                                          "Cholesky; allow more multigrid levels");
  const int n = int(M->H[L].ndof);
  M->ncoarse = n;
  DevLevel<double>& d = M->lev<double>(L);
  if (!M->Ainv64) M->Ainv64 = M->alloc<double>(size_t(n) * n);
  double* A = M->Ainv64;
  launch_fill<double>(n, 0.0, d.f, s);
  for (int j = 0; j < n; ++j) {
    launch_fill<double>(1, 1.0, d.f + j, s);
    apply_level<double>(M, L, d.f, d.t, s);
    HIPCHK(hipMemcpyAsync(A + size_t(j) * n, d.t, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_fill<double>(1, 0.0, d.f + j, s);
  }
  launch_symmetrize_dense<double>(n, A, 0, s);
  if (!M->blas) {
    if (rocblas_create_handle(&M->blas) != rocblas_status_success) throw Error(HPDG_ERR_HIP, "rocblas handle");
  }
  rocblas_set_stream(M->blas, s);
  rocblas_int* info = nullptr;
  HIPCHK(hipMalloc(&info, sizeof(rocblas_int)));
  rocblas_int hinfo = 0;
  auto check = [&](rocblas_status st, const char* what) {
    HIPCHK(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st != rocblas_status_success || hinfo != 0) {
      (void)hipFree(info);
      if (st != rocblas_status_success)
        throw Error(HPDG_ERR_HIP, std::string(what) + " of the coarsest operator failed with rocblas status " +
                                      std::to_string(int(st)));
      throw Error(HPDG_ERR_BREAKDOWN, std::string(what) + ": the coarsest operator is not positive definite (info " +
                                          std::to_string(hinfo) + ")");
    }
  };
  check(rocsolver_dpotrf(M->blas, rocblas_fill_lower, n, A, n, info), "Cholesky");
  check(rocsolver_dpotri(M->blas, rocblas_fill_lower, n, A, n, info), "inverse");
  (void)hipFree(info);
  launch_symmetrize_dense<double>(n, A, 1, s);
  HIPCHK(hipStreamSynchronize(s));
}

void check_mesh(const hpdg_mesh_desc* D) {
  if (!D || D->n_macro <= 0 || D->n_elem <= 0 || !D->macro_kind || !D->macro_params || !D->macro_nbr ||
      !D->macro_nbr_face || !D->macro_nbr_orient || !D->macro_bc || !D->elem_macro || !D->elem_level ||
      !D->elem_anchor || !D->elem_p)
    throw Error(HPDG_ERR_INVALID_ARG, "incomplete mesh description");
}

void build_levels(hpdg_mesh* M);
void macro_mesh_from(const hpdg_mesh_desc* desc, MacroMesh& mm);
std::vector<Cell> cells_from(const hpdg_mesh_desc* desc);

// host side of an upload: macro mesh, level hierarchy, geometry / mortar / transfer tables
std::unique_ptr<hpdg_mesh> build_mesh_host(hpdg_ctx* ctx, const hpdg_mesh_desc* desc, const hpdg_disc_params* disc) {
  check_mesh(desc);
  auto M = std::make_unique<hpdg_mesh>();
  M->ctx = ctx;
  macro_mesh_from(desc, M->mm);
  if (disc) {
    M->dp.C = disc->penalty_C > 0 ? disc->penalty_C : 10.0;
    M->dp.quad_extra = disc->quad_extra >= 0 ? disc->quad_extra : 1;
    M->dp.coef_kind = disc->coef_kind;
    for (int i = 0; i < 4; ++i) M->dp.coef[i] = disc->coef_params[i];
    M->has_f32 = disc->build_f32 != 0;
    M->dp.mass_term = disc->mass_term != 0 ? 1 : 0;
    M->dp.robin_gamma = disc->robin_gamma;
    if (disc->ec_mode < HPDG_EC_AUTO || disc->ec_mode > HPDG_EC_NEVER)
      throw Error(HPDG_ERR_INVALID_ARG, "unknown element-centric mode");
    M->dp.ec_mode = disc->ec_mode;
    if (!std::isfinite(M->dp.robin_gamma)) throw Error(HPDG_ERR_INVALID_ARG, "non-finite Robin coefficient");
  }
  M->max_levels = (disc && disc->max_levels > 0) ? std::min(disc->max_levels, 32) : 32;
  M->tab.build();
  // hierarchy
  LevelHost L0;
  L0.cells = cells_from(desc);
  M->H.push_back(std::move(L0));
  build_levels(M.get());
  return M;
}

void macro_mesh_from(const hpdg_mesh_desc* desc, MacroMesh& mm) {
  const int nm = desc->n_macro;
  mm.macros.resize(nm);
  for (int m = 0; m < nm; ++m) {
    mm.macros[m].kind = desc->macro_kind[m];
    if (desc->macro_kind[m] < 0 || desc->macro_kind[m] > 2) throw Error(HPDG_ERR_INVALID_MESH, "unknown map kind");
    for (int f = 0; f < 6; ++f)
      if (desc->macro_bc[6 * m + f] < 0 || desc->macro_bc[6 * m + f] > 3)
        throw Error(HPDG_ERR_INVALID_MESH, "unknown boundary kind");
    std::memcpy(mm.macros[m].par, desc->macro_params + 16 * m, 16 * sizeof(double));
  }
  mm.nbr.assign(desc->macro_nbr, desc->macro_nbr + 6 * nm);
  mm.nbr_face.assign(desc->macro_nbr_face, desc->macro_nbr_face + 6 * nm);
  mm.nbr_orient.assign(desc->macro_nbr_orient, desc->macro_nbr_orient + 6 * nm);
  mm.bc.assign(desc->macro_bc, desc->macro_bc + 6 * nm);
}

std::vector<Cell> cells_from(const hpdg_mesh_desc* desc) {
  std::vector<Cell> cells(size_t(desc->n_elem));
  for (long long e = 0; e < desc->n_elem; ++e) {
    Cell& c = cells[e];
    c.macro = desc->elem_macro[e];
    c.level = desc->elem_level[e];
    c.a[0] = desc->elem_anchor[3 * e];
    c.a[1] = desc->elem_anchor[3 * e + 1];
    c.a[2] = desc->elem_anchor[3 * e + 2];
    c.p = desc->elem_p[e];
  }
  return cells;
}

// the level hierarchy below H[0] (surrogate coarsening, Sec. II.D.3) and every level's tables;
// tabulated coefficients of H[0] are carried down level by level
void build_levels(hpdg_mesh* M) {
  M->H.resize(1);
  while (int(M->H.size()) < M->max_levels) {
    LevelHost next;
    if (!coarsen_cells(M->mm, M->H.back().cells, next.cells)) break;
    M->H.push_back(std::move(next));
  }
  for (int l = 0; l < M->nlevels(); ++l) {
    LevelHost& h = M->H[l];
    if (l > 0) coarsen_fields(M->dp, M->H[l - 1], h);  // needs the finer level's records
    build_level(M->mm, M->dp, M->tab, h);
    build_diagonal(M->tab, h);
    for (double dgv : h.diag)
      if (!(dgv > 0)) throw Error(HPDG_ERR_INVALID_MESH, "non-positive operator diagonal");
  }
  for (int l = 0; l + 1 < M->nlevels(); ++l) build_transfer(M->H[l], M->H[l + 1]);
}

// a tabulated mass coefficient c (hpdg_set_coefficient): w det J c at every level's GL points,
// and the point-Jacobi scaling of the operators with that mass term
void set_mass_tables(hpdg_mesh* M, hipStream_t s) {
  if (M->H[0].nmq == 0) throw Error(HPDG_ERR_UNSUPPORTED, "a mass coefficient needs a mesh uploaded with mass_term");
  std::vector<double> wc;
  for (int l = 0; l < M->nlevels(); ++l) {
    const LevelHost& h = M->H[l];
    mass_table(M->mm, M->dp, h, wc);
    DevLevel<double>& d = M->lev<double>(l);
    HIPCHK(hipMemcpyAsync(d.mcoef, wc.data(), wc.size() * sizeof(double), hipMemcpyHostToDevice, s));
    launch_diag_mass<double>(M->view<double>(l), d.diag, d.dinv, s);
    if (M->has_f32) {
      DevLevel<float>& f = M->lev<float>(l);
      launch_convert_d2f(h.nmq, d.mcoef, f.mcoef, s);
      launch_convert_d2f(h.ndof, d.dinv, f.dinv, s);
    }
    HIPCHK(hipStreamSynchronize(s));
  }
}

// device side of an upload: tables, level data, Krylov work vectors, coarsest inverse
void upload_mesh_device(hpdg_mesh* M, hipStream_t s) {
  // device tables
  M->tab_off = M->upload_raw(M->tab.off, s);
  M->dg_off = M->upload_raw(M->tab.dg_off, s);
  M->w_off = M->upload_raw(M->tab.w_off, s);
  M->dface_off = M->upload_raw(M->tab.dface_off, s);
  M->gl_off = M->upload_raw(M->tab.gl_off, s);
  M->tab64 = M->upload_raw(M->tab.data, s);
  if (M->has_f32) M->tab32 = M->upload<float>(M->tab.data, s);
  M->L64.resize(M->nlevels());
  if (M->has_f32) M->L32.resize(M->nlevels());
  for (int l = 0; l < M->nlevels(); ++l) {
    build_device_level<double>(M, l, s);
    if (M->has_f32) build_device_level<float>(M, l, s);
  }
  if (M->dp.cfield) set_mass_tables(M, s);
  const long long n0 = M->H[0].ndof;
  M->r = M->alloc<double>(n0);
  M->vv = M->alloc<double>(n0);
  M->w = M->alloc<double>(n0);
  M->d = M->alloc<double>(n0);
  M->q = M->alloc<double>(n0);
  M->partials = M->alloc<double>(3 * kRedBlocks);
  M->sc = M->alloc<double>(16);
  HIPCHK(hipHostMalloc((void**)&M->host_sc, 16 * sizeof(double), hipHostMallocDefault));
  launch_fill<double>(16, 0.0, M->sc, s);
  M->lam.assign(M->nlevels(), 0.0);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
}

// device bytes an upload (and a smoother setup with ``scaling``) will allocate
size_t estimate_device_bytes(const hpdg_mesh* M, int scaling) {
  const size_t prec = M->has_f32 ? 12 : 8;  // bytes per scalar over the FP64 (+ FP32) copies
  size_t b = M->tab.data.size() * prec + M->tab.off.size() * 4 + 4096;
  size_t full_max = 0;  // the full FP64 blocks of one level, alive while that level is set up
  for (int l = 0; l < M->nlevels(); ++l) {
    const LevelHost& h = M->H[l];
    b += h.einfo.size() * sizeof(ElemInfo) * (M->has_f32 ? 2 : 1);
    b += h.minfo.size() * sizeof(MortarInfo) * (M->has_f32 ? 2 : 1);
    b += (h.fmlist.size() + h.bucket_elems.size()) * 4 * (M->has_f32 ? 2 : 1);
    b += h.mtask.size() * sizeof(MortarTask) * (M->has_f32 ? 2 : 1);
    b += (h.vgeo.size() + h.mgeo.size()) * prec;
    b += size_t(h.ndof) * prec * 5;  // dinv, f, v, t, p
    b += size_t(h.ntrace + h.nslot) * prec;  // face traces and slots
    b += size_t(h.nmq) * prec + (h.nmq ? size_t(h.ndof) * prec : 0);
    b += (h.tinfo.size() * sizeof(TransferInfo) + (h.cstart.size() + h.clist.size()) * 4) * (M->has_f32 ? 2 : 1);
    if (scaling != HPDG_SMOOTH_NONE && l + 1 < M->nlevels())
      b += size_t(h.ntrace) * prec;  // the second face-trace buffer of the fused steps
    if (scaling == HPDG_SMOOTH_BLOCK && l + 1 < M->nlevels()) {
      size_t packed = 0, full = 0;
      for (const ElemInfo& I : h.einfo) {
        const size_t N = size_t(I.n) * I.n * I.n;
        packed += N * (N + 1) / 2;
        full += N * N;
      }
      b += packed * (M->has_f32 ? 12 : 8) + (M->has_f32 ? full * 2 : 0) + h.einfo.size() * 8;  // FP64 (+ FP32, bf16)
      full_max = std::max(full_max, full * 8 + h.einfo.size() * 8);
    }
  }
  const size_t n0 = size_t(M->H[0].ndof), nc = size_t(M->H.back().ndof);
  b += full_max + n0 * 8 * 5 + 3 * kRedBlocks * 8 + 128 + nc * nc * 8;
  return b;
}

void setup_smoother_impl(hpdg_mesh* mesh, const hpdg_smoother_params* params, double* lambda_max, hipStream_t s);

// rebuild every level's tables and device data after the discretisation changed (a new
// coefficient): a fresh mesh object is built and uploaded, its device state is exchanged with
// M's (so the caller's handle stays valid), and the old state is freed with the fresh object;
// a smoother that was set up is set up again with its parameters (bounds recomputed)
void rebuild_mesh(hpdg_mesh* M, hipStream_t s) {
  HIPCHK(hipStreamSynchronize(s));
  collect_timing(M);
  auto F = std::make_unique<hpdg_mesh>();
  F->ctx = M->ctx;
  F->mm = M->mm;
  F->dp = M->dp;
  F->tab = M->tab;
  F->has_f32 = M->has_f32;
  F->max_levels = M->max_levels;
  F->H.resize(1);
  F->H[0].cells = M->H[0].cells;
  F->H[0].kvals = M->H[0].kvals;
  F->H[0].cvals = M->H[0].cvals;
  build_levels(F.get());
  upload_mesh_device(F.get(), s);
  using std::swap;
  swap(M->H, F->H);
  swap(M->allocs, F->allocs);
  swap(M->alloc_bytes, F->alloc_bytes);
  swap(M->bytes, F->bytes);
  swap(M->tab_off, F->tab_off);
  swap(M->dg_off, F->dg_off);
  swap(M->w_off, F->w_off);
  swap(M->dface_off, F->dface_off);
  swap(M->gl_off, F->gl_off);
  swap(M->tab64, F->tab64);
  swap(M->tab32, F->tab32);
  swap(M->L64, F->L64);
  swap(M->L32, F->L32);
  swap(M->Ainv64, F->Ainv64);
  swap(M->ncoarse, F->ncoarse);
  swap(M->lam, F->lam);
  swap(M->est, F->est);
  swap(M->dmacros, F->dmacros);
  swap(M->dcells, F->dcells);
  swap(M->bad, F->bad);
  swap(M->host_bad, F->host_bad);
  swap(M->nl_b, F->nl_b);
  swap(M->nl_rhs, F->nl_rhs);
  swap(M->nl_delta, F->nl_delta);
  swap(M->nl_key, F->nl_key);
  swap(M->nl_kind, F->nl_kind);
  swap(M->r, F->r);
  swap(M->vv, F->vv);
  swap(M->w, F->w);
  swap(M->d, F->d);
  swap(M->q, F->q);
  swap(M->partials, F->partials);
  swap(M->sc, F->sc);
  swap(M->host_sc, F->host_sc);
  swap(M->gm_V, F->gm_V);
  swap(M->gm_Z, F->gm_Z);
  swap(M->gm_m, F->gm_m);
  swap(M->block_scalars, F->block_scalars);
  swap(M->block_full_scalars, F->block_full_scalars);
  swap(M->sw, F->sw);
  F.reset();  // frees M's previous device state
  if (M->smoother_ready) setup_smoother_impl(M, nullptr, nullptr, s);
}

void assemble_rhs_impl(hpdg_mesh* mesh, const hpdg_rhs_desc* rhs, double* F_dev, hipStream_t s) {
  if (rhs->kind < 0 || rhs->kind > 6) throw Error(HPDG_ERR_INVALID_ARG, "unknown rhs kind");
  if (rhs->n_params > 0 && !rhs->params) throw Error(HPDG_ERR_INVALID_ARG, "rhs parameters missing");
  if (rhs->kind == 3 && rhs->n_params > 16 * 16 * 16) throw Error(HPDG_ERR_INVALID_ARG, "polynomial degree above 15");
  std::vector<double> P(rhs->params, rhs->params + std::max(rhs->n_params, 0));
  std::vector<double> F;
  assemble_rhs(mesh->mm, mesh->dp, mesh->tab, mesh->H[0], rhs->kind, P, F);  // boundary faces
  if (!mesh->dmacros) {
    mesh->dmacros = mesh->upload_raw(mesh->mm.macros, s);
    mesh->dcells = mesh->upload_raw(mesh->H[0].cells, s);
  }
  double* Pd = mesh->upload_raw(P, s);
  hipError_t err = hipMemcpyAsync(F_dev, F.data(), F.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (err == hipSuccess) {
    launch_rhs_volume(mesh->view<double>(0), mesh->dmacros, mesh->dcells, rhs->kind, Pd, int(P.size()), F_dev, s);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (err == hipSuccess) mesh->release(Pd);
  HIPCHK(err);
}

// eta2(e) of u on level 0 (Eqs. Eta2_Ingredients .. Eta2_Local)
void estimate_impl(hpdg_mesh* M, const hpdg_rhs_desc* rhs, const double* u, double* eta2, double* eta2_vol,
                   hipStream_t s) {
  if (rhs->kind < 0 || rhs->kind > 6) throw Error(HPDG_ERR_INVALID_ARG, "unknown rhs kind");
  if (rhs->n_params > 0 && !rhs->params) throw Error(HPDG_ERR_INVALID_ARG, "rhs parameters missing");
  const LevelHost& h = M->H[0];
  if (est_lds_bytes(h.nmax, h.qmax) > 64 * 1024)
    throw Error(HPDG_ERR_UNSUPPORTED, "estimator: degree too high for one element's workspace");
  std::vector<double> P(rhs->params, rhs->params + std::max(rhs->n_params, 0));
  std::vector<double> key{double(rhs->kind)};
  key.insert(key.end(), P.begin(), P.end());
  auto& E = M->est;
  if (E.key != key) {
    HIPCHK(hipStreamSynchronize(s));
    for (void* ptr : E.ptrs) M->release(ptr);
    E = hpdg_mesh::EstCache{};
    EstTables t;
    estimator_tables(M->mm, M->est_grid.get(), M->dp, h, rhs->kind, P, t);
    auto keep = [&](auto* ptr) {
      E.ptrs.push_back(ptr);
      return ptr;
    };
    E.ev.vol = keep(M->upload_raw(t.vol, s));
    E.ev.voff = keep(M->upload_raw(t.voff, s));
    E.ev.he2p2 = keep(M->upload_raw(t.he2p2, s));
    E.tasks = keep(M->upload_raw(t.tasks, s));
    E.n_tasks = (long long)t.tasks.size();
    E.ef.face = keep(M->upload_raw(t.face, s));
    E.ef.foff = keep(M->upload_raw(t.foff, s));
    E.ef.tmortar = keep(M->upload_raw(t.task_mortar, s));
    E.ef.out = keep(M->alloc<double>(h.minfo.size()));
    E.vpart = keep(M->alloc<double>(h.cells.size()));
    E.key = key;
    long long mg = 0;
    for (const MortarTask& t : t.tasks) mg += 8LL * (t.gmode ? (long long)t.q * t.q : 1);
    E.vpoints = (long long)t.vol.size() / 3;
    E.mpoints = (long long)t.face.size() / 4;
    E.alg_bytes = 8 * (h.ndof + (long long)t.vol.size() + (long long)h.vgeo.size() + (long long)t.face.size() + mg +
                       2 * (long long)h.cells.size()) +
                  (long long)(h.einfo.size() * sizeof(ElemInfo) + t.tasks.size() * sizeof(MortarTask) +
                              h.fmlist.size() * sizeof(int) + (t.voff.size() + t.foff.size()) * sizeof(long long));
  }
  LevelView<double> V = M->view<double>(0);
  V.mtask = E.tasks;
  V.n_mtask = E.n_tasks;
  launch_fill<double>((long long)h.minfo.size(), 0.0, E.ef.out, s);
  launch_estimator(V, u, E.ev, E.ef, E.n_tasks, eta2_vol ? eta2_vol : E.vpart, eta2, s);
  HIPCHK(hipGetLastError());
}

// u_to = u_from carried from mesh ``from`` onto mesh ``to`` (the same macro-mesh; every cell of
// ``to`` is a cell of ``from`` or one of its children, of equal or higher degree): the child-half
// and degree interpolation of the multigrid prolongation, exact for these pairs
void transfer_impl(const hpdg_mesh* A, hpdg_mesh* B, const double* u_from, double* u_to, hipStream_t s) {
  const MacroMesh &ma = A->mm, &mb = B->mm;
  bool same = ma.macros.size() == mb.macros.size() && ma.nbr == mb.nbr && ma.nbr_face == mb.nbr_face &&
              ma.nbr_orient == mb.nbr_orient && ma.bc == mb.bc;
  for (size_t m = 0; same && m < ma.macros.size(); ++m)
    same = ma.macros[m].kind == mb.macros[m].kind &&
           std::memcmp(ma.macros[m].par, mb.macros[m].par, sizeof(ma.macros[m].par)) == 0;
  if (!same) throw Error(HPDG_ERR_INVALID_ARG, "transfer: the meshes have different macro-meshes");
  LevelHost fine;
  fine.cells = B->H[0].cells;
  fine.einfo = B->H[0].einfo;
  try {
    build_transfer(fine, A->H[0]);
  } catch (const Error& e) {
    throw Error(HPDG_ERR_INVALID_ARG, std::string("transfer: ") + e.what());
  }
  TransferInfo* ti = B->upload_raw(fine.tinfo, s);  // synchronises s
  hipError_t err;
  {
    TransferView<double> V;
    V.tinfo = ti;
    V.cstart = nullptr;
    V.clist = nullptr;
    V.tab = B->table<double>();
    V.tv = B->tabview();
    V.n_fine = (long long)fine.cells.size();
    V.n_coarse = (long long)A->H[0].cells.size();
    V.nmax = std::max(A->H[0].nmax, B->H[0].nmax);
    launch_fill<double>(B->H[0].ndof, 0.0, u_to, s);
    launch_prolong_add<double>(V, u_from, u_to, s);
    err = hipGetLastError();
    if (err == hipSuccess) err = hipStreamSynchronize(s);
  }
  if (err == hipSuccess) B->release(ti);
  HIPCHK(err);
}

void setup_smoother_impl(hpdg_mesh* mesh, const hpdg_smoother_params* params, double* lambda_max, hipStream_t s) {
  if (params) {
    mesh->sp = *params;
    if (mesh->sp.n_cheb <= 0) mesh->sp.n_cheb = 4;
    if (mesh->sp.n_cheb_coarse < 0) mesh->sp.n_cheb_coarse = 0;
    mesh->sp.unfused = mesh->sp.unfused ? 1 : 0;
    if (mesh->sp.n_eigs <= 0) mesh->sp.n_eigs = 15;
    if (!(mesh->sp.Lambda > 1.0)) mesh->sp.Lambda = 20.0;
    if (mesh->sp.scaling < HPDG_SMOOTH_NONE || mesh->sp.scaling > HPDG_SMOOTH_SCHWARZ)
      throw Error(HPDG_ERR_INVALID_ARG, "unknown smoother scaling");
    if (mesh->sp.scaling == HPDG_SMOOTH_SCHWARZ && mesh->sp.schwarz_overlap < 1)
      throw Error(HPDG_ERR_INVALID_ARG, "Schwarz overlap must be at least 1");
  }
  if (mesh->sp.scaling == HPDG_SMOOTH_SCHWARZ) {
    if (!mesh->Ainv64) build_coarse(mesh, s);
    if (mesh->sw.size() < size_t(mesh->nlevels())) mesh->sw.resize(size_t(mesh->nlevels()));
    for (int l = 0; l + 1 < mesh->nlevels(); ++l) build_schwarz(mesh, l, s);
    for (int l = 0; l + 1 < mesh->nlevels(); ++l) {
      mesh->lam[l] = 0.0;  // no spectral bound
      if (lambda_max) lambda_max[l] = 0.0;
    }
    HIPCHK(hipStreamSynchronize(s));
    mesh->smoother_ready = true;
    return;
  }
  // the exact coarse solve is part of the solver's setup: a mesh used only for applies never
  // forms the dense inverse (whose size limits the coarsest level)
  if (!mesh->Ainv64) build_coarse(mesh, s);
  if (mesh->sp.scaling == HPDG_SMOOTH_BLOCK)
    for (int l = 0; l + 1 < mesh->nlevels(); ++l) build_blocks(mesh, l, s);
  if (mesh->sp.scaling != HPDG_SMOOTH_NONE)  // the fused Jacobi-scaled steps' second trace buffer
    for (int l = 0; l + 1 < mesh->nlevels(); ++l) {
      if (!mesh->H[l].fast_n.empty()) continue;  // levels with element-centric elements do not chain traces
      const size_t nt = size_t(mesh->H[l].ntrace);
      if (!mesh->lev<double>(l).trace2) mesh->lev<double>(l).trace2 = mesh->alloc<double>(nt);
      if (mesh->has_f32 && !mesh->lev<float>(l).trace2) mesh->lev<float>(l).trace2 = mesh->alloc<float>(nt);
    }
  for (int l = 0; l + 1 < mesh->nlevels(); ++l) {
    if (lambda_max && lambda_max[l] > 0)
      mesh->lam[l] = lambda_max[l];
    else
      mesh->lam[l] = cg_bound(mesh, l, mesh->sp.n_eigs, mesh->sp.seed, s);
    if (lambda_max) lambda_max[l] = mesh->lam[l];
  }
  HIPCHK(hipStreamSynchronize(s));
  mesh->smoother_ready = true;
}

// FCG (Alg. 2, device-resident scalars, one host read per iteration) or PCG, from the initial
// guess in u; returns false when the iteration cap is reached
bool krylov_solve(hpdg_mesh* mesh, const hpdg_solve_params& params, const double* b_dev, double* u_dev, int& iters,
                  double& rel, hipStream_t s) {
  const bool mixed = params.precision == HPDG_PREC_MIXED || params.precision == HPDG_PREC_MIXED_BF16;
  mesh->bf16_blocks = params.precision == HPDG_PREC_MIXED_BF16;
  iters = 0;
  rel = 0;
  const long long n = mesh->H[0].ndof;
  const double nb = std::sqrt(dot_sync(mesh, n, b_dev, b_dev, s));
  if (!std::isfinite(nb)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite right-hand side");
  double* r = mesh->r;
  apply_level<double>(mesh, 0, u_dev, mesh->w, s);
  launch_copy<double>(n, b_dev, r, s);
  launch_axpby<double>(n, -1.0, mesh->w, 1.0, r, s);  // r0 = b - A u0
  if (nb == 0.0) {
    launch_fill<double>(n, 0.0, u_dev, s);
    HIPCHK(hipStreamSynchronize(s));
    return true;
  }
  double rr = dot_sync(mesh, n, r, r, s);
  rel = std::sqrt(rr) / nb;
  auto precond = [&](const double* in, double* out) {
    if (mixed) {
      DevLevel<float>& d32 = mesh->L32[0];
      // level-0 FP32 f / v buffers are free (the V-cycle takes f_0, v_0 as arguments)
      launch_convert_d2f(n, in, d32.f, s);
      vcycle<float>(mesh, d32.f, d32.v, s);
      launch_convert_f2d(n, d32.v, out, s);
    } else {
      vcycle<double>(mesh, in, out, s);
    }
  };
  if (params.solver == HPDG_SOLVER_PCG) {
    // textbook PCG: z = M r, p = z + beta p, alpha = r.z / p.Ap
    double* z = mesh->vv;
    double* p = mesh->d;
    double* Ap = mesh->w;
    precond(r, z);
    launch_copy<double>(n, z, p, s);
    double rz = dot_sync(mesh, n, r, z, s);
    while (rel > params.tol_rel && iters < params.max_iter) {
      apply_level<double>(mesh, 0, p, Ap, s);
      const double pAp = dot_sync(mesh, n, p, Ap, s);
      if (!(pAp > 0) || !std::isfinite(pAp)) throw Error(HPDG_ERR_BREAKDOWN, "PCG breakdown");
      const double alpha = rz / pAp;
      launch_axpby<double>(n, alpha, p, 1.0, u_dev, s);
      launch_axpby<double>(n, -alpha, Ap, 1.0, r, s);
      precond(r, z);
      const double rz2 = dot_sync(mesh, n, r, z, s);
      launch_axpby<double>(n, 1.0, z, rz2 / rz, p, s);
      rz = rz2;
      rr = dot_sync(mesh, n, r, r, s);
      rel = std::sqrt(rr) / nb;
      ++iters;
    }
  } else if (params.solver == HPDG_SOLVER_FGMRES) {
    // restarted flexible GMRES: V[0..m] an orthonormal basis, Z[j] = M V[j] (kept, since
    // the preconditioner may vary), H the (m+1) x m Hessenberg matrix reduced by Givens
    // rotations on the host; u += Z y at the end of a cycle
    const int m = params.restart > 0 ? params.restart : 30;
    if (mesh->gm_m < m) {
      if (mesh->gm_V) mesh->release(mesh->gm_V);
      if (mesh->gm_Z) mesh->release(mesh->gm_Z);
      mesh->gm_V = mesh->alloc<double>(size_t(m + 1) * size_t(n));
      mesh->gm_Z = mesh->alloc<double>(size_t(m) * size_t(n));
      mesh->gm_m = m;
    }
    auto V = [&](int j) { return mesh->gm_V + size_t(j) * size_t(n); };
    auto Z = [&](int j) { return mesh->gm_Z + size_t(j) * size_t(n); };
    std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto h = [&](int i, int j) -> double& { return H[size_t(j) * (m + 1) + i]; };
    while (rel > params.tol_rel && iters < params.max_iter) {
      const double beta = std::sqrt(rr);
      launch_fill<double>(n, 0.0, V(0), s);
      launch_axpby<double>(n, 1.0 / beta, r, 0.0, V(0), s);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;  // columns of this cycle
      while (k < m && iters < params.max_iter) {
        const int j = k;
        precond(V(j), Z(j));
        apply_level<double>(mesh, 0, Z(j), V(j + 1), s);
        for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
          h(i, j) = dot_sync(mesh, n, V(j + 1), V(i), s);
          launch_axpby<double>(n, -h(i, j), V(i), 1.0, V(j + 1), s);
        }
        const double hn = std::sqrt(dot_sync(mesh, n, V(j + 1), V(j + 1), s));
        if (!std::isfinite(hn)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite FGMRES basis vector");
        h(j + 1, j) = hn;
        if (hn > 0) launch_axpby<double>(n, 0.0, V(j + 1), 1.0 / hn, V(j + 1), s);
        for (int i = 0; i < j; ++i) {  // earlier rotations on column j
          const double a = h(i, j), b2 = h(i + 1, j);
          h(i, j) = cs[i] * a + sn[i] * b2;
          h(i + 1, j) = -sn[i] * a + cs[i] * b2;
        }
        const double den = std::hypot(h(j, j), h(j + 1, j));
        if (!(den > 0)) throw Error(HPDG_ERR_BREAKDOWN, "FGMRES breakdown (zero column)");
        cs[j] = h(j, j) / den;
        sn[j] = h(j + 1, j) / den;
        h(j, j) = den;
        h(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++k;
        ++iters;
        if (std::fabs(g[j + 1]) / nb <= params.tol_rel || hn == 0.0) break;
      }
      for (int i = k - 1; i >= 0; --i) {  // y = R^-1 g (back substitution)
        double t = g[i];
        for (int l = i + 1; l < k; ++l) t -= h(i, l) * y[l];
        y[i] = t / h(i, i);
      }
      for (int i = 0; i < k; ++i) launch_axpby<double>(n, y[i], Z(i), 1.0, u_dev, s);
      apply_level<double>(mesh, 0, u_dev, mesh->w, s);  // true residual
      launch_copy<double>(n, b_dev, r, s);
      launch_axpby<double>(n, -1.0, mesh->w, 1.0, r, s);
      rr = dot_sync(mesh, n, r, r, s);
      if (!std::isfinite(rr)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite residual");
      rel = std::sqrt(rr) / nb;
    }
  } else {
    // Alg. 2 with device-resident scalars; one host read of |r|^2 per iteration
    launch_fill<double>(16, 0.0, mesh->sc, s);
    while (rel > params.tol_rel && iters < params.max_iter) {
      const int first = iters == 0 ? 1 : 0;
      precond(r, mesh->vv);
      apply_level<double>(mesh, 0, mesh->vv, mesh->w, s);
      launch_dot3(n, mesh->vv, r, mesh->w, first ? nullptr : mesh->q, mesh->partials, mesh->sc, s);
      launch_fcg_scalars(mesh->sc, first, s);
      launch_fcg_update(n, mesh->vv, mesh->w, mesh->d, mesh->q, u_dev, r, mesh->sc, mesh->partials, first, s);
      HIPCHK(hipMemcpyAsync(mesh->host_sc, mesh->sc, 9 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      ++iters;
      if (mesh->host_sc[8] != 0.0) throw Error(HPDG_ERR_BREAKDOWN, "FCG breakdown (rho <= 0 or non-finite)");
      rr = mesh->host_sc[7];
      if (!std::isfinite(rr)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite residual");
      rel = std::sqrt(rr) / nb;
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  return rel <= params.tol_rel;
}

// alpha and w det J beta at the GL points of every level for the source ``nl`` (host, FP64)
void set_nonlinear(hpdg_mesh* M, const hpdg_nonlinear_desc* nl, hipStream_t s) {
  if (M->H[0].nmq == 0) throw Error(HPDG_ERR_UNSUPPORTED, "mesh uploaded without mass_term");
  if (nl->kind != HPDG_NL_PUNCTURE && nl->kind != HPDG_NL_QUADRATIC && nl->kind != HPDG_NL_STAR)
    throw Error(HPDG_ERR_INVALID_ARG, "unknown nonlinear source kind");
  if (nl->n_params < 0 || (nl->n_params > 0 && !nl->params)) throw Error(HPDG_ERR_INVALID_ARG, "bad parameters");
  const std::vector<double> P(nl->params, nl->params + nl->n_params);
  if (nl->kind == HPDG_NL_PUNCTURE && (P.empty() || (P.size() - 1) % 5 != 0 || !(P[0] > 0)))
    throw Error(HPDG_ERR_INVALID_ARG, "puncture parameters are [s > 0, rows of 5]");
  if (nl->kind == HPDG_NL_QUADRATIC && P.size() != 28)
    throw Error(HPDG_ERR_INVALID_ARG, "quadratic parameters are [alpha, 27 coefficients]");
  if (nl->kind == HPDG_NL_STAR && (P.size() != 2 || !(P[0] > 0) || !(P[1] > 0)))
    throw Error(HPDG_ERR_INVALID_ARG, "star parameters are [rho0 > 0, r0 > 0]");
  std::vector<double> key(1, double(nl->kind));
  key.insert(key.end(), P.begin(), P.end());
  if (key == M->nl_key) return;
  if (!M->bad) {
    M->bad = M->alloc<int>(1);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&M->host_bad), sizeof(int)));
  }
  std::vector<double> x, wdet, al, wb;
  for (int l = 0; l < M->nlevels(); ++l) {
    const LevelHost& h = M->H[l];
    mass_points(M->mm, h, x, wdet);
    al.resize(wdet.size());
    wb.resize(wdet.size());
    for (size_t k = 0; k < wdet.size(); ++k) {
      double a, b;
      nl_coefficients(nl->kind, P, &x[3 * k], a, b);
      al[k] = a;
      wb[k] = wdet[k] * b;
    }
    DevLevel<double>& d = M->lev<double>(l);
    if (!d.nl_alpha) {
      d.nl_alpha = M->alloc<double>(al.size());
      d.nl_wbeta = M->alloc<double>(wb.size());
    }
    HIPCHK(hipMemcpyAsync(d.nl_alpha, al.data(), al.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.nl_wbeta, wb.data(), wb.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  M->nl_key = key;
  M->nl_kind = nl->kind;
}

void clear_bad(hpdg_mesh* M, hipStream_t s) {
  *M->host_bad = 0;
  HIPCHK(hipMemcpyAsync(M->bad, M->host_bad, sizeof(int), hipMemcpyHostToDevice, s));
}

void check_bad(hpdg_mesh* M, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(M->host_bad, M->bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (*M->host_bad) throw Error(HPDG_ERR_BREAKDOWN, "1 + alpha u <= 0 at a quadrature point");
}

// R = A u - N(u) - F on level 0 (F may be null)
void nl_residual(hpdg_mesh* M, const double* F, const double* u, double* R, hipStream_t s) {
  const long long n = M->H[0].ndof;
  DevLevel<double>& d = M->lev<double>(0);
  M->mass_on = false;
  apply_level<double>(M, 0, u, R, s);
  M->mass_on = true;
  clear_bad(M, s);
  launch_nl_eval(M->view<double>(0), M->nl_kind, u, d.nl_alpha, d.nl_wbeta, d.t, nullptr, M->bad, s);
  launch_axpby<double>(n, -1.0, d.t, 1.0, R, s);
  if (F) launch_axpby<double>(n, -1.0, F, 1.0, R, s);
  check_bad(M, s);
}

// Jacobian mass terms on every level from the state u (injected downwards), then the
// point-Jacobi scaling, the spectral bounds and the coarsest inverse of the new operators
void linearize(hpdg_mesh* M, const double* u, hipStream_t s) {
  if (!M->smoother_ready) throw Error(HPDG_ERR_INVALID_ARG, "call hpdg_setup_smoother first");
  if (M->sp.scaling == HPDG_SMOOTH_BLOCK)
    throw Error(HPDG_ERR_UNSUPPORTED, "block-Jacobi smoothing is not rebuilt for Newton linearisations");
  if (M->sp.scaling == HPDG_SMOOTH_SCHWARZ)
    throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing is not rebuilt for Newton linearisations");
  const int L = M->nlevels();
  clear_bad(M, s);
  const double* ul = u;
  for (int l = 0; l < L; ++l) {
    DevLevel<double>& d = M->lev<double>(l);
    if (l > 0) {
      launch_inject<double>(M->tview<double>(l - 1), ul, d.p, s);
      ul = d.p;
    }
    launch_nl_eval(M->view<double>(l), M->nl_kind, ul, d.nl_alpha, d.nl_wbeta, nullptr, d.mcoef, M->bad, s);
  }
  check_bad(M, s);
  for (int l = 0; l < L; ++l) {
    DevLevel<double>& d = M->lev<double>(l);
    launch_diag_mass<double>(M->view<double>(l), d.diag, d.dinv, s);
    if (M->has_f32) {
      DevLevel<float>& f = M->lev<float>(l);
      launch_convert_d2f(M->H[l].nmq, d.mcoef, f.mcoef, s);
      launch_convert_d2f(M->H[l].ndof, d.dinv, f.dinv, s);
    }
  }
  for (int l = 0; l + 1 < L; ++l) M->lam[l] = cg_bound(M, l, M->sp.n_eigs, M->sp.seed, s);
  build_coarse(M, s);
}


}  // namespace

// ---- solve server ------------------------------------------------------------------
namespace {

// a mesh uploaded with its smoother set up, and its right-hand side and solution vectors
struct Prepared {
  std::unique_ptr<hpdg_mesh> M;
  double* F = nullptr;
  double* u = nullptr;
  size_t bytes = 0;      // the footprint estimate of the requests on it
  uint64_t last_use = 0;
};

struct ServerRequest {
  uint64_t ticket = 0;
  Prepared pre;          // an idle prepared mesh of the same key, claimed when the request is picked
  std::string key;       // bytes of the mesh description and discretisation (host-table cache key)
  std::vector<int32_t> mkind, mnbr, mnface, mnor, mbc, emacro, elevel, eanchor, ep;
  std::vector<double> mparams, rhs_params;
  hpdg_mesh_desc desc{};
  hpdg_disc_params disc{};
  hpdg_rhs_desc rhs{};
  double* u_out = nullptr;
  size_t estimate = 0;   // footprint used for admission (upper estimate from the description)
  int bypassed = 0;      // times passed over while at the head of the queue
  hpdg_request_status st{};
};

// device footprint from the description alone (before any table is built): vectors and
// tables of every level, metric at GL points, smoother data, FP32 copies; an upper estimate
size_t estimate_from_desc(const hpdg_mesh_desc& d, const hpdg_disc_params& disc, int scaling) {
  double dof = 0, geo = 0, blocks = 0;
  int pmin = 16;
  for (int64_t e = 0; e < d.n_elem; ++e) {
    const double n = d.elem_p[e] + 1.0, q = n + 1.0;
    pmin = std::min(pmin, d.elem_p[e]);
    const bool affine = d.macro_kind[d.elem_macro[e]] == HPDG_MAP_AFFINE && disc.coef_kind == HPDG_COEF_CONSTANT;
    dof += n * n * n;
    geo += (affine ? 6.0 : 6.0 * q * q * q) + 3.0 * 8.0 * q * q + (disc.mass_term ? q * q * q : 0.0) + 12.0 * n * n;
    if (scaling == HPDG_SMOOTH_BLOCK) blocks += n * n * n * (n * n * n + 1.0) / 2.0;
  }
  const double prec = disc.build_f32 ? 12.0 : 8.0;
  // packed inverse blocks: FP64, plus FP32 and full bf16 copies (as many bytes as packed FP32);
  // the full FP64 blocks of the finest level exist while it is set up (twice the packed count)
  const double bprec = disc.build_f32 ? 16.0 : 8.0;
  const double levels = 8.0 / 7.0;  // coarser levels: a geometric series in the element count
  const double coarse = double(d.n_macro) * std::pow(pmin + 1.0, 3);
  const double b = levels * (prec * (6.0 * dof + geo) + bprec * blocks + 250.0 * d.n_elem) + 8.0 * 5.0 * dof +
                   16.0 * blocks + prec * coarse * coarse + (1 << 20);
  return size_t(1.25 * b);
}

}  // namespace

struct hpdg_server {
  hpdg_ctx* ctx = nullptr;
  hpdg_server_params p{};
  std::mutex mu;
  // host tables (hierarchy, geometry, mortars, transfers) of recently served meshes: a request
  // on a mesh seen before copies them instead of rebuilding; least recently used evicted
  // beyond kHostCacheBytes
  static constexpr size_t kHostCacheBytes = size_t(16) << 30;
  struct Cached {
    std::shared_ptr<const hpdg_mesh> host;
    size_t bytes = 0;
    uint64_t last_use = 0;
  };
  std::mutex cache_mu;
  std::map<std::string, Cached> cache;
  size_t cache_bytes = 0;
  uint64_t cache_clock = 0;
  // meshes a finished request leaves uploaded with their smoother set up and their right-hand
  // side and solution vectors: a later request on the same mesh (same key) takes one instead of
  // uploading and setting up again.  Their device bytes (the requests' footprint estimates)
  // count against the budget; the least recently used are freed when a request needs the room
  // or when they pass kIdleBytes.  Guarded by mu.
  static constexpr size_t kIdleBytes = size_t(64) << 30;
  std::map<std::string, std::vector<Prepared>> idle;
  size_t idle_bytes = 0;
  uint64_t idle_clock = 0;
  // frees the least recently used idle mesh (not one of key ``keep``); false when there is none
  // (caller holds mu)
  bool evict_idle(const std::string* keep = nullptr) {
    std::string key;
    size_t at = 0;
    uint64_t best = UINT64_MAX;
    for (auto& kv : idle)
      for (size_t i = 0; i < kv.second.size(); ++i)
        if ((!keep || kv.first != *keep) && kv.second[i].last_use < best) {
          best = kv.second[i].last_use;
          key = kv.first;
          at = i;
        }
    if (best == UINT64_MAX) return false;
    auto& v = idle[key];
    idle_bytes -= v[at].bytes;
    v.erase(v.begin() + at);
    if (v.empty()) idle.erase(key);
    return true;
  }
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<ServerRequest>> reqs;
  size_t in_flight_bytes = 0;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  // the first queued request that fits (the head is not passed over more than 2 max_active
  // times); caller holds mu
  ServerRequest* pick() {
    const size_t budget = p.hbm_budget_bytes;
    for (size_t k = 0; k < queue.size(); ++k) {
      ServerRequest* r = reqs[queue[k]].get();
      // a request on a mesh that waits idle reuses it: those bytes are already counted
      const bool reuse = idle.count(r->key) != 0;
      const size_t others = idle_bytes - (reuse ? r->estimate : 0);
      if (budget && k == 0) {  // other idle meshes give way to the head of the queue
        while (in_flight_bytes + others + r->estimate > budget && idle_bytes > (reuse ? r->estimate : 0)) {
          if (!evict_idle(reuse ? &r->key : nullptr)) break;
        }
      }
      const size_t used = in_flight_bytes + idle_bytes - (idle.count(r->key) ? r->estimate : 0);
      const bool fits = !budget || used + r->estimate <= budget || (in_flight_bytes == 0 && k == 0);
      if (fits) {
        if (k > 0) reqs[queue[0]]->bypassed += 1;
        queue.erase(queue.begin() + k);
        auto it = idle.find(r->key);
        if (it != idle.end()) {  // its bytes move from the idle to the in-flight count
          r->pre = std::move(it->second.back());
          it->second.pop_back();
          if (it->second.empty()) idle.erase(it);
          idle_bytes -= r->pre.bytes;
        }
        return r;
      }
      if (k == 0 && reqs[queue[0]]->bypassed >= 2 * p.max_active) return nullptr;
    }
    return nullptr;
  }
  void run(ServerRequest* r, hipStream_t s) {
    int iters = 0;
    double rel = 0;
    int rc = HPDG_OK;
    std::string msg;
    try {
      Prepared P = std::move(r->pre);
      if (!P.M) {
        P.M = host_tables(r);
        upload_mesh_device(P.M.get(), s);
        setup_smoother_impl(P.M.get(), &p.smoother, nullptr, s);
        P.F = P.M->alloc<double>(size_t(P.M->H[0].ndof));
        P.u = P.M->alloc<double>(size_t(P.M->H[0].ndof));
      }
      hpdg_mesh* M = P.M.get();
      const long long n = M->H[0].ndof;
      double* F = P.F;
      double* u = P.u;
      assemble_rhs_impl(M, &r->rhs, F, s);
      launch_fill<double>(n, 0.0, u, s);
      hpdg_solve_params sp{HPDG_SOLVER_FCG, p.precision, p.tol_rel, p.max_iter, 0};
      const bool ok = krylov_solve(M, sp, F, u, iters, rel, s);
      if (!ok) rc = HPDG_ERR_NOT_CONVERGED;
      HIPCHK(hipMemcpyAsync(r->u_out, u, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::lock_guard<std::mutex> lock(mu);
      r->st.n_dof = n;
      // keep the prepared mesh for a later request on it
      P.bytes = r->estimate;
      P.last_use = ++idle_clock;
      if (P.bytes <= kIdleBytes) {
        idle_bytes += P.bytes;
        idle[r->key].push_back(std::move(P));
        while (idle_bytes > kIdleBytes && evict_idle()) {
        }
      }
    } catch (const Error& e) {
      rc = e.code;
      msg = e.what();
    } catch (const std::exception& e) {
      rc = HPDG_ERR_INVALID_ARG;
      msg = e.what();
    } catch (...) {
      rc = HPDG_ERR_INVALID_ARG;
      msg = "unknown error";
    }
    std::lock_guard<std::mutex> lock(mu);
    if (rc != HPDG_OK) {
      if (msg.empty()) msg = "error " + std::to_string(rc);
      std::snprintf(r->st.message, sizeof(r->st.message), "%s", msg.c_str());
    }
    r->st.iterations = iters;
    r->st.rel_residual = rel;
    r->st.status = rc;
    r->st.state = rc == HPDG_OK ? HPDG_REQ_DONE : HPDG_REQ_FAILED;
    r->st.end_ms = now_ms();
  }
  std::unique_ptr<hpdg_mesh> host_tables(const ServerRequest* r) {
    std::shared_ptr<const hpdg_mesh> C;
    {
      std::lock_guard<std::mutex> lock(cache_mu);
      auto it = cache.find(r->key);
      if (it != cache.end()) {
        it->second.last_use = ++cache_clock;
        C = it->second.host;
      }
    }
    if (!C) {
      std::shared_ptr<hpdg_mesh> built(build_mesh_host(ctx, &r->desc, &r->disc).release());
      const size_t bytes = host_bytes(*built);
      std::lock_guard<std::mutex> lock(cache_mu);
      if (bytes <= kHostCacheBytes && !cache.count(r->key)) {
        while (cache_bytes + bytes > kHostCacheBytes && !cache.empty()) {
          auto lru = cache.begin();
          for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->second.last_use < lru->second.last_use) lru = it;
          cache_bytes -= lru->second.bytes;
          cache.erase(lru);
        }
        cache[r->key] = Cached{built, bytes, ++cache_clock};
        cache_bytes += bytes;
      }
      C = built;
    }
    auto M = std::make_unique<hpdg_mesh>();
    M->ctx = ctx;
    M->mm = C->mm;
    M->dp = C->dp;
    M->tab = C->tab;
    M->H = C->H;
    M->has_f32 = C->has_f32;
    return M;
  }
  static size_t host_bytes(const hpdg_mesh& M) {
    size_t b = M.tab.data.size() * 8;
    for (const LevelHost& h : M.H)
      b += (h.vgeo.size() + h.mgeo.size() + h.diag.size()) * 8 + h.einfo.size() * sizeof(ElemInfo) +
           h.minfo.size() * sizeof(MortarInfo) + h.mortars.size() * sizeof(Mortar) + h.cells.size() * sizeof(Cell) +
           (h.fmlist.size() + h.bucket_elems.size() + h.cstart.size() + h.clist.size()) * 4 +
           h.tinfo.size() * sizeof(TransferInfo);
    return b;
  }
  void worker() {
    (void)hipSetDevice(ctx->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (;;) {
      ServerRequest* r = nullptr;
      {
        std::unique_lock<std::mutex> lock(mu);
        cv_work.wait(lock, [&] { return stop || (!queue.empty() && (r = pick()) != nullptr); });
        if (!r) break;  // stop with nothing admissible
        in_flight_bytes += r->estimate;
        r->st.state = HPDG_REQ_RUNNING;
        r->st.start_ms = now_ms();
        r->st.device_bytes = r->estimate;
      }
      run(r, s);
      {
        std::lock_guard<std::mutex> lock(mu);
        in_flight_bytes -= r->estimate;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

int hpdg_create(hpdg_ctx** out, int hip_device, size_t hbm_budget_bytes) {
  if (!out) return HPDG_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return HPDG_ERR_HIP;
  if (hip_device < 0 || hip_device >= count) return HPDG_ERR_INVALID_ARG;
  if (hipSetDevice(hip_device) != hipSuccess) return HPDG_ERR_HIP;
  try {
    init_noalloc_scratch(hip_device);
  } catch (const Error& e) {
    return fail(nullptr, HPDG_ERR_HIP, e.what());
  }
  auto* c = new hpdg_ctx;
  c->device = hip_device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return HPDG_OK;
}

int hpdg_destroy(hpdg_ctx* ctx) {
  if (!ctx) return HPDG_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  for (hpdg_mesh* m : ctx->meshes) delete m;
  delete ctx;
  return HPDG_OK;
}

const char* hpdg_last_error(const hpdg_ctx* ctx) {
  (void)ctx;
  return t_last_error.c_str();
}

int hpdg_mesh_upload(hpdg_ctx* ctx, const hpdg_mesh_desc* desc, const hpdg_disc_params* disc,
                     hpdg_mesh** out, void* stream) {
  if (!ctx || !out) return fail(ctx, HPDG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  return guarded(ctx, [&] {
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_ptr<hpdg_mesh> M = build_mesh_host(ctx, desc, disc);
    upload_mesh_device(M.get(), S(stream));
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->meshes.push_back(M.get());
    *out = M.release();
  });
}

int hpdg_mesh_info_get(const hpdg_mesh* mesh, hpdg_mesh_info* out) {
  if (!mesh || !out) return HPDG_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->n_levels = mesh->nlevels();
  for (int l = 0; l < mesh->nlevels() && l < 32; ++l) {
    out->n_elem[l] = (int64_t)mesh->H[l].cells.size();
    out->n_dof[l] = mesh->H[l].ndof;
    out->n_mortar[l] = (int64_t)mesh->H[l].mortars.size();
    out->vgeo_scalars[l] = (int64_t)mesh->H[l].vgeo.size();
    out->mgeo_scalars[l] = (int64_t)mesh->H[l].mgeo.size();
    out->table_bytes[l] = (int64_t)(mesh->H[l].einfo.size() * sizeof(ElemInfo) +
                                    mesh->H[l].minfo.size() * sizeof(MortarInfo) +
                                    mesh->H[l].fmlist.size() * sizeof(int));
    out->n_elem_centric[l] = (int64_t)mesh->H[l].fast_elems.size();
    out->n_mortar_tasks[l] = (int64_t)mesh->H[l].mtask.size();
    double fma = 0;
    const LevelHost& h = mesh->H[l];
    for (size_t e = 0; e < h.einfo.size(); ++e) {
      const double n = h.einfo[e].n, q = h.einfo[e].q;
      if (h.fast[e])
        fma += 8 * n * n * n * n + 6 * n * n * (3 * n + 6);
      else
        fma += 2 * (n * n * n * q + n * n * q * q + n * q * q * q) + 6 * q * q * q * q + 9 * q * q * q +
               6 * (9 * n * n * q + 12 * n * q * q + 20 * q * q);
    }
    out->apply_flops[l] = 2 * fma;
  }
  out->device_bytes = mesh->bytes;
  out->est_alg_bytes = mesh->est.alg_bytes;
  out->est_volume_points = mesh->est.vpoints;
  out->est_mortar_points = mesh->est.mpoints;
  out->block_retries = mesh->block_retries;
  out->coarse_retries = mesh->coarse_retries;
  return HPDG_OK;
}

int hpdg_level_cells(const hpdg_mesh* mesh, int level, int32_t* macro, int32_t* lvl, int32_t* anchor,
                     int32_t* p) {
  if (!mesh || level < 0 || level >= mesh->nlevels()) return HPDG_ERR_INVALID_ARG;
  const auto& cells = mesh->H[level].cells;
  for (size_t e = 0; e < cells.size(); ++e) {
    if (macro) macro[e] = cells[e].macro;
    if (lvl) lvl[e] = cells[e].level;
    if (anchor)
      for (int d = 0; d < 3; ++d) anchor[3 * e + d] = cells[e].a[d];
    if (p) p[e] = cells[e].p;
  }
  return HPDG_OK;
}

int hpdg_mesh_free(hpdg_mesh* mesh) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  hpdg_ctx* ctx = mesh->ctx;
  (void)hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->meshes.erase(std::remove(ctx->meshes.begin(), ctx->meshes.end(), mesh), ctx->meshes.end());
  }
  delete mesh;
  return HPDG_OK;
}

int hpdg_assemble_rhs(hpdg_mesh* mesh, const hpdg_rhs_desc* rhs, double* F_dev, void* stream) {
  if (!mesh || !rhs || !F_dev) return HPDG_ERR_INVALID_ARG;
  return guarded(mesh->ctx, [&] { assemble_rhs_impl(mesh, rhs, F_dev, S(stream)); });
}

int hpdg_apply(hpdg_mesh* mesh, int level, int prec, const void* x_dev, void* y_dev, void* stream) {
  if (!mesh || !x_dev || !y_dev || x_dev == y_dev || level < 0 || level >= mesh->nlevels())
    return mesh ? fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid apply arguments") : HPDG_ERR_INVALID_ARG;
  if (prec == HPDG_F32 && !mesh->has_f32) return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  return guarded(mesh->ctx, [&] {
    hipStream_t s = S(stream);
    if (prec == HPDG_F32)
      apply_level<float>(mesh, level, static_cast<const float*>(x_dev), static_cast<float*>(y_dev), s);
    else
      apply_level<double>(mesh, level, static_cast<const double*>(x_dev), static_cast<double*>(y_dev), s);
    HIPCHK(hipGetLastError());
  });
}

int hpdg_estimate(hpdg_mesh* mesh, const hpdg_rhs_desc* rhs, const double* u_dev, double* eta2_dev,
                  double* eta2_vol_dev, void* stream) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  if (!rhs || !u_dev || !eta2_dev || eta2_dev == eta2_vol_dev)
    return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid estimator arguments");
  return guarded(mesh->ctx, [&] {
    HIPCHK(hipSetDevice(mesh->ctx->device));
    estimate_impl(mesh, rhs, u_dev, eta2_dev, eta2_vol_dev, S(stream));
  });
}

int hpdg_set_estimator_grid(hpdg_mesh* mesh, const hpdg_mesh_desc* grid) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  return guarded(mesh->ctx, [&] {
    if (!grid) {
      mesh->est_grid.reset();
    } else {
      if (!grid->macro_kind || !grid->macro_params || !grid->macro_nbr || !grid->macro_nbr_face ||
          !grid->macro_nbr_orient || !grid->macro_bc)
        throw Error(HPDG_ERR_INVALID_ARG, "incomplete estimator grid");
      auto g = std::make_unique<MacroMesh>();
      macro_mesh_from(grid, *g);
      const MacroMesh& mm = mesh->mm;
      if (g->macros.size() != mm.macros.size() || g->nbr != mm.nbr || g->nbr_face != mm.nbr_face ||
          g->nbr_orient != mm.nbr_orient)
        throw Error(HPDG_ERR_INVALID_MESH, "the estimator grid must have the mesh's macro connectivity");
      mesh->est_grid = std::move(g);
    }
    mesh->est.key.clear();  // the point data are rebuilt on the next estimate
  });
}

int hpdg_transfer(const hpdg_mesh* from, hpdg_mesh* to, const double* u_from_dev, double* u_to_dev,
                  void* stream) {
  if (!from || !to) return HPDG_ERR_INVALID_ARG;
  if (!u_from_dev || !u_to_dev || u_from_dev == u_to_dev || from->ctx != to->ctx)
    return fail(to->ctx, HPDG_ERR_INVALID_ARG, "invalid transfer arguments");
  return guarded(to->ctx, [&] {
    HIPCHK(hipSetDevice(to->ctx->device));
    transfer_impl(from, to, u_from_dev, u_to_dev, S(stream));
  });
}

int hpdg_amr_mark(const double* eta2, int64_t n, int mode, double param, uint8_t* marked) {
  if (!eta2 || !marked || n <= 0 || !std::isfinite(param) || (mode != HPDG_MARK_FRACTION && mode != HPDG_MARK_MEAN) ||
      (mode == HPDG_MARK_FRACTION && !(param >= 0 && param <= 1)))
    return fail(nullptr, HPDG_ERR_INVALID_ARG, "invalid marking arguments");
  for (int64_t e = 0; e < n; ++e)
    if (!std::isfinite(eta2[e])) return fail(nullptr, HPDG_ERR_INVALID_ARG, "non-finite estimate");
  std::fill(marked, marked + n, uint8_t(0));
  if (mode == HPDG_MARK_MEAN) {
    double sum = 0;
    for (int64_t e = 0; e < n; ++e) sum += eta2[e];
    const double thr = param * (sum / double(n));
    for (int64_t e = 0; e < n; ++e) marked[e] = eta2[e] > thr ? 1 : 0;
    return HPDG_OK;
  }
  return guarded(nullptr, [&] {
    const int64_t k = std::min<int64_t>(n, (int64_t)std::ceil(param * double(n) - 1e-9));
    std::vector<int64_t> order(static_cast<size_t>(n));
    for (int64_t e = 0; e < n; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return eta2[a] > eta2[b]; });
    for (int64_t i = 0; i < k; ++i) marked[order[i]] = 1;
  });
}

int hpdg_amr_smooth_pred(const double* eta2, const double* eta2_pred, const int32_t* p, const uint8_t* marked,
                         int64_t n, double gamma_h, double gamma_p, int8_t* action, double* pred_out) {
  if (!eta2 || !eta2_pred || !p || !marked || !action || !pred_out || n <= 0 || !(gamma_h > 0) || !(gamma_p > 0))
    return fail(nullptr, HPDG_ERR_INVALID_ARG, "invalid smooth-pred arguments");
  for (int64_t e = 0; e < n; ++e) {
    action[e] = 0;
    pred_out[e] = eta2_pred[e];
    if (!marked[e]) continue;
    if (eta2[e] > eta2_pred[e]) {  // worse than predicted: not smooth, h-refine
      action[e] = 1;
      pred_out[e] = gamma_h * std::pow(0.5, 3 + 2 * p[e]) * eta2[e];
    } else {  // as predicted (or no prediction yet): p-refine
      action[e] = 2;
      pred_out[e] = gamma_p * eta2[e];
    }
  }
  return HPDG_OK;
}

int hpdg_amr_adapt(const hpdg_mesh_desc* mesh, const int8_t* action, int32_t max_degree, int64_t capacity,
                   int32_t* macro, int32_t* level, int32_t* anchor, int32_t* p, int64_t* origin, int64_t* n_out) {
  if (!mesh || !action || !n_out || !macro || !level || !anchor || !p || !origin || max_degree < 1 ||
      max_degree > kMaxN - 1)
    return fail(nullptr, HPDG_ERR_INVALID_ARG, "invalid adaptation arguments");
  return guarded(nullptr, [&] {
    check_mesh(mesh);
    MacroMesh mm;
    macro_mesh_from(mesh, mm);
    const std::vector<Cell> cells = cells_from(mesh);
    std::vector<Cell> out;
    std::vector<int> org;
    adapt_cells(mm, cells, reinterpret_cast<const signed char*>(action), max_degree, out, org);
    *n_out = (int64_t)out.size();
    if (*n_out > capacity) throw Error(HPDG_ERR_INVALID_ARG, "adaptation: output capacity too small");
    for (size_t e = 0; e < out.size(); ++e) {
      macro[e] = out[e].macro;
      level[e] = out[e].level;
      for (int d = 0; d < 3; ++d) anchor[3 * e + d] = out[e].a[d];
      p[e] = out[e].p;
      origin[e] = org[e];
    }
  });
}

int hpdg_set_coefficient(hpdg_mesh* mesh, int kind, int where, const double* host_vals, const double* params,
                         void* stream) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  if ((kind != HPDG_COEF_DIFFUSION && kind != HPDG_COEF_MASS) ||
      (where != HPDG_WHERE_ELEMENT && where != HPDG_WHERE_NODE && where != HPDG_WHERE_ANALYTIC))
    return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "unknown coefficient kind or placement");
  if (where == HPDG_WHERE_ANALYTIC ? !params : !host_vals)
    return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "coefficient values missing");
  return guarded(mesh->ctx, [&] {
    HIPCHK(hipSetDevice(mesh->ctx->device));
    LevelHost& h0 = mesh->H[0];
    std::vector<double> vals;
    if (where == HPDG_WHERE_ELEMENT) vals.assign(host_vals, host_vals + h0.cells.size());
    if (where == HPDG_WHERE_NODE) vals.assign(host_vals, host_vals + h0.ndof);
    for (double v : vals) {
      if (!std::isfinite(v)) throw Error(HPDG_ERR_INVALID_ARG, "non-finite coefficient value");
      if (kind == HPDG_COEF_DIFFUSION && !(v > 0)) throw Error(HPDG_ERR_INVALID_ARG, "the diffusion coefficient must be positive");
    }
    if (kind == HPDG_COEF_MASS && !mesh->dp.mass_term)
      throw Error(HPDG_ERR_UNSUPPORTED, "a mass coefficient needs a mesh uploaded with mass_term = 1");
    if (kind == HPDG_COEF_DIFFUSION) {
      if (where == HPDG_WHERE_ANALYTIC) {
        const int ck = int(params[0]);
        if (ck != HPDG_COEF_CONSTANT && ck != HPDG_COEF_RADIAL_STEP)
          throw Error(HPDG_ERR_INVALID_ARG, "unknown analytic diffusion coefficient");
        if (ck == HPDG_COEF_RADIAL_STEP && !(params[2] > 0 && params[3] > 0))
          throw Error(HPDG_ERR_INVALID_ARG, "the diffusion coefficient must be positive");
        mesh->dp.coef_kind = ck;
        for (int i = 0; i < 4; ++i) mesh->dp.coef[i] = params[1 + i];
        mesh->dp.kfield = 0;
        h0.kvals.clear();
      } else {
        mesh->dp.kfield = where == HPDG_WHERE_ELEMENT ? 1 : 2;
        h0.kvals = vals;
      }
    } else {
      if (where == HPDG_WHERE_ANALYTIC) {
        if (!std::isfinite(params[0])) throw Error(HPDG_ERR_INVALID_ARG, "non-finite coefficient value");
        vals.assign(h0.cells.size(), params[0]);
        mesh->dp.cfield = 1;
      } else {
        mesh->dp.cfield = where == HPDG_WHERE_ELEMENT ? 1 : 2;
      }
      h0.cvals = vals;
    }
    rebuild_mesh(mesh, S(stream));
  });
}

int hpdg_apply_noalloc(hpdg_mesh* mesh, int level, int prec, const void* x_dev, void* y_dev, void* stream) {
  if (!mesh || !x_dev || !y_dev || x_dev == y_dev || level < 0 || level >= mesh->nlevels())
    return mesh ? fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid apply arguments") : HPDG_ERR_INVALID_ARG;
  if (prec == HPDG_F32 && !mesh->has_f32) return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  return guarded(mesh->ctx, [&] {
    void* scr = noalloc_scratch(mesh->ctx->device);
    if (!scr) throw Error(HPDG_ERR_HIP, "the no-allocation scratch is not set up on this device");
    const LevelHost& h = mesh->H[level];
    const size_t need = size_t(h.ntrace + h.nslot) * (prec == HPDG_F32 ? sizeof(float) : sizeof(double));
    if (need > noalloc_scratch_bytes())
      throw Error(HPDG_ERR_INVALID_ARG, "level " + std::to_string(level) + " needs " + std::to_string(need) +
                                            " bytes of face traces and face slots; the no-allocation apply holds "
                                            "at most " + std::to_string(noalloc_scratch_bytes()) + " bytes");
    hipStream_t s = S(stream);
    if (prec == HPDG_F32) {
      float* tr = static_cast<float*>(scr);
      apply_level_scratch<float>(mesh, level, static_cast<const float*>(x_dev), static_cast<float*>(y_dev), tr,
                                 tr + h.ntrace, s);
    } else {
      double* tr = static_cast<double*>(scr);
      apply_level_scratch<double>(mesh, level, static_cast<const double*>(x_dev), static_cast<double*>(y_dev), tr,
                                  tr + h.ntrace, s);
    }
    HIPCHK(hipGetLastError());
  });
}

int hpdg_timing_enable(hpdg_mesh* mesh, int every) {
  if (!mesh || every < 0) return HPDG_ERR_INVALID_ARG;
  mesh->timing = every > 0;
  mesh->timing_every = std::max(every, 1);
  std::memset(mesh->timing_count, 0, sizeof(mesh->timing_count));
  return HPDG_OK;
}

int hpdg_kernel_timing(hpdg_mesh* mesh, int kind, int level, int prec, double* total_ms, int64_t* launches,
                       double* alg_bytes) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  if (kind < 0 || kind >= HPDG_TIMING_KINDS || level < 0 || level >= mesh->nlevels() || level >= 32 ||
      (prec != HPDG_F64 && prec != HPDG_F32))
    return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid timing entry");
  return guarded(mesh->ctx, [&] {
    collect_timing(mesh);
    hpdg_mesh::Acc& a = mesh->acc[kind][level][prec];
    if (total_ms) *total_ms = a.ms;
    if (launches) *launches = a.calls;
    if (alg_bytes) *alg_bytes = a.bytes;
    a = hpdg_mesh::Acc();
  });
}

int hpdg_setup_smoother(hpdg_mesh* mesh, const hpdg_smoother_params* params, double* lambda_max,
                        void* stream) {
  if (!mesh) return HPDG_ERR_INVALID_ARG;
  return guarded(mesh->ctx, [&] { setup_smoother_impl(mesh, params, lambda_max, S(stream)); });
}

int hpdg_smooth(hpdg_mesh* mesh, int level, int prec, const void* b_dev, void* x_dev, int n_iter,
                void* stream) {
  if (!mesh || !b_dev || !x_dev || level < 0 || level >= mesh->nlevels() - 1 || n_iter < 0)
    return mesh ? fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid smooth arguments") : HPDG_ERR_INVALID_ARG;
  if (!mesh->smoother_ready) return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "call hpdg_setup_smoother first");
  if (prec == HPDG_F32 && !mesh->has_f32) return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  return guarded(mesh->ctx, [&] {
    if (prec == HPDG_F32)
      smooth_level<float>(mesh, level, static_cast<const float*>(b_dev), static_cast<float*>(x_dev), n_iter,
                          false, S(stream));
    else
      smooth_level<double>(mesh, level, static_cast<const double*>(b_dev), static_cast<double*>(x_dev),
                           n_iter, false, S(stream));
    HIPCHK(hipGetLastError());
  });
}

int hpdg_vcycle(hpdg_mesh* mesh, int prec, const void* r_dev, void* z_dev, void* stream) {
  if (!mesh || !r_dev || !z_dev || r_dev == z_dev)
    return mesh ? fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "invalid vcycle arguments") : HPDG_ERR_INVALID_ARG;
  if (!mesh->smoother_ready) return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "call hpdg_setup_smoother first");
  if (prec == HPDG_F32 && !mesh->has_f32) return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  return guarded(mesh->ctx, [&] {
    if (prec == HPDG_F32)
      vcycle<float>(mesh, static_cast<const float*>(r_dev), static_cast<float*>(z_dev), S(stream));
    else
      vcycle<double>(mesh, static_cast<const double*>(r_dev), static_cast<double*>(z_dev), S(stream));
    HIPCHK(hipGetLastError());
  });
}

int hpdg_solve(hpdg_mesh* mesh, const hpdg_solve_params* params, const double* b_dev, double* u_dev,
               hpdg_solve_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!mesh || !params || !b_dev || !u_dev) return HPDG_ERR_INVALID_ARG;
  if (!mesh->smoother_ready) return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "call hpdg_setup_smoother first");
  if (params->precision != HPDG_PREC_F64 && !mesh->has_f32)
    return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  if (params->solver < HPDG_SOLVER_FCG || params->solver > HPDG_SOLVER_FGMRES || params->restart < 0 ||
      params->restart > 1000)
    return fail(mesh->ctx, HPDG_ERR_INVALID_ARG, "unknown solver or restart length out of [0, 1000]");
  int iters = 0;
  double rel = 0;
  bool converged = true;
  auto t0 = std::chrono::steady_clock::now();
  int rc = guarded(mesh->ctx, [&] {
    converged = krylov_solve(mesh, *params, b_dev, u_dev, iters, rel, S(stream));
  });
  auto t1 = std::chrono::steady_clock::now();
  if (rc == HPDG_OK && !converged) rc = fail(mesh->ctx, HPDG_ERR_NOT_CONVERGED, "iteration cap reached");
  if (stats) {
    stats->iterations = iters;
    stats->rel_residual = rel;
    stats->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->status = rc;
  }
  return rc;
}

int hpdg_nonlinear_residual(hpdg_mesh* mesh, const hpdg_nonlinear_desc* nl, const double* F_dev,
                            const double* u_dev, double* R_dev, void* stream) {
  if (!mesh || !nl || !u_dev || !R_dev || R_dev == u_dev || R_dev == F_dev) return HPDG_ERR_INVALID_ARG;
  return guarded(mesh->ctx, [&] {
    hipStream_t s = S(stream);
    set_nonlinear(mesh, nl, s);
    nl_residual(mesh, F_dev, u_dev, R_dev, s);
    HIPCHK(hipStreamSynchronize(s));
  });
}

int hpdg_nonlinear_linearize(hpdg_mesh* mesh, const hpdg_nonlinear_desc* nl, const double* u_dev,
                             void* stream) {
  if (!mesh || !nl || !u_dev) return HPDG_ERR_INVALID_ARG;
  return guarded(mesh->ctx, [&] {
    hipStream_t s = S(stream);
    set_nonlinear(mesh, nl, s);
    linearize(mesh, u_dev, s);
  });
}

int hpdg_newton_solve(hpdg_mesh* mesh, const hpdg_newton_params* params, const hpdg_nonlinear_desc* nl,
                      const double* F_dev, double* u_dev, hpdg_newton_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!mesh || !params || !nl || !u_dev || F_dev == u_dev) return HPDG_ERR_INVALID_ARG;
  if (params->precision != HPDG_PREC_F64 && !mesh->has_f32)
    return fail(mesh->ctx, HPDG_ERR_UNSUPPORTED, "mesh built without FP32 levels");
  int steps = 0, lin = 0;
  double rel = 1.0;
  auto t0 = std::chrono::steady_clock::now();
  int rc = guarded(mesh->ctx, [&] {
    hipStream_t s = S(stream);
    set_nonlinear(mesh, nl, s);
    const long long n = mesh->H[0].ndof;
    if (!mesh->nl_b) {
      mesh->nl_b = mesh->alloc<double>(size_t(n));
      mesh->nl_rhs = mesh->alloc<double>(size_t(n));
      mesh->nl_delta = mesh->alloc<double>(size_t(n));
    }
    double* R = mesh->nl_b;
    nl_residual(mesh, F_dev, u_dev, R, s);
    const double r0 = std::sqrt(dot_sync(mesh, n, R, R, s));
    if (!std::isfinite(r0)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite initial residual");
    rel = r0 > 0 ? 1.0 : 0.0;
    hpdg_solve_params lp{HPDG_SOLVER_FCG, params->precision, params->lin_tol_rel, params->max_lin_iter};
    while (rel > params->tol_rel && steps < params->max_newton) {
      linearize(mesh, u_dev, s);
      launch_fill<double>(n, 0.0, mesh->nl_rhs, s);
      launch_axpby<double>(n, -1.0, R, 1.0, mesh->nl_rhs, s);  // b = -R
      launch_fill<double>(n, 0.0, mesh->nl_delta, s);
      int its = 0;
      double lrel = 0;
      krylov_solve(mesh, lp, mesh->nl_rhs, mesh->nl_delta, its, lrel, s);  // an inexact correction is still taken
      lin += its;
      launch_axpby<double>(n, 1.0, mesh->nl_delta, 1.0, u_dev, s);
      nl_residual(mesh, F_dev, u_dev, R, s);
      const double rn = std::sqrt(dot_sync(mesh, n, R, R, s));
      if (!std::isfinite(rn)) throw Error(HPDG_ERR_BREAKDOWN, "non-finite Newton residual");
      rel = rn / r0;
      ++steps;
    }
    HIPCHK(hipStreamSynchronize(s));
  });
  auto t1 = std::chrono::steady_clock::now();
  if (rc == HPDG_OK && rel > params->tol_rel) rc = fail(mesh->ctx, HPDG_ERR_NOT_CONVERGED, "Newton step cap reached");
  if (stats) {
    stats->newton_steps = steps;
    stats->linear_iterations = lin;
    stats->rel_residual = rel;
    stats->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->status = rc;
  }
  return rc;
}

int hpdg_server_create(hpdg_ctx* ctx, const hpdg_server_params* params, hpdg_server** out) {
  if (!ctx || !params || !out || params->max_active < 1 || params->max_active > 64)
    return fail(ctx, HPDG_ERR_INVALID_ARG, "invalid server parameters");
  auto* sv = new hpdg_server;
  sv->ctx = ctx;
  sv->p = *params;
  if (sv->p.max_iter <= 0) sv->p.max_iter = 1000;
  if (!(sv->p.tol_rel > 0)) sv->p.tol_rel = 1e-10;
  sv->t0 = std::chrono::steady_clock::now();
  for (int w = 0; w < sv->p.max_active; ++w) sv->workers.emplace_back([sv] { sv->worker(); });
  *out = sv;
  return HPDG_OK;
}

int hpdg_server_submit(hpdg_server* sv, const hpdg_request* rq, uint64_t* ticket) {
  if (!sv || !rq || !ticket || !rq->u_out) return HPDG_ERR_INVALID_ARG;
  return guarded(sv->ctx, [&] {
    check_mesh(&rq->mesh);
    auto r = std::make_unique<ServerRequest>();
    const hpdg_mesh_desc& d = rq->mesh;
    const int nm = d.n_macro;
    const int64_t E = d.n_elem;
    r->mkind.assign(d.macro_kind, d.macro_kind + nm);
    r->mparams.assign(d.macro_params, d.macro_params + 16 * nm);
    r->mnbr.assign(d.macro_nbr, d.macro_nbr + 6 * nm);
    r->mnface.assign(d.macro_nbr_face, d.macro_nbr_face + 6 * nm);
    r->mnor.assign(d.macro_nbr_orient, d.macro_nbr_orient + 6 * nm);
    r->mbc.assign(d.macro_bc, d.macro_bc + 6 * nm);
    r->emacro.assign(d.elem_macro, d.elem_macro + E);
    r->elevel.assign(d.elem_level, d.elem_level + E);
    r->eanchor.assign(d.elem_anchor, d.elem_anchor + 3 * E);
    r->ep.assign(d.elem_p, d.elem_p + E);
    for (int m = 0; m < nm; ++m)
      if (r->mkind[m] < 0 || r->mkind[m] > 2) throw Error(HPDG_ERR_INVALID_MESH, "unknown map kind");
    for (int64_t e = 0; e < E; ++e)
      if (r->emacro[e] < 0 || r->emacro[e] >= nm) throw Error(HPDG_ERR_INVALID_MESH, "element macro out of range");
    r->desc = hpdg_mesh_desc{nm, r->mkind.data(), r->mparams.data(), r->mnbr.data(), r->mnface.data(),
                             r->mnor.data(), r->mbc.data(), E, r->emacro.data(), r->elevel.data(),
                             r->eanchor.data(), r->ep.data()};
    r->disc = rq->disc;
    r->disc.build_f32 = sv->p.precision != HPDG_PREC_F64 ? 1 : r->disc.build_f32;
    if (rq->rhs.n_params > 0) {
      if (!rq->rhs.params) throw Error(HPDG_ERR_INVALID_ARG, "rhs parameters missing");
      r->rhs_params.assign(rq->rhs.params, rq->rhs.params + rq->rhs.n_params);
    }
    r->rhs = hpdg_rhs_desc{rq->rhs.kind, int32_t(r->rhs_params.size()), r->rhs_params.data()};
    r->u_out = rq->u_out;
    r->estimate = estimate_from_desc(r->desc, r->disc, sv->p.smoother.scaling);
    auto put = [&](const void* ptr, size_t bytes) { r->key.append(static_cast<const char*>(ptr), bytes); };
    const hpdg_disc_params& dc = r->disc;  // field by field (the struct has padding)
    put(&dc.penalty_C, 8);
    put(&dc.quad_extra, 4);
    put(&dc.coef_kind, 4);
    put(dc.coef_params, 32);
    put(&dc.max_levels, 4);
    put(&dc.build_f32, 4);
    put(&dc.mass_term, 4);
    put(&dc.robin_gamma, 8);
    put(&dc.ec_mode, 4);
    put(r->mkind.data(), 4 * r->mkind.size());
    put(r->mparams.data(), 8 * r->mparams.size());
    put(r->mnbr.data(), 4 * r->mnbr.size());
    put(r->mnface.data(), 4 * r->mnface.size());
    put(r->mnor.data(), 4 * r->mnor.size());
    put(r->mbc.data(), 4 * r->mbc.size());
    put(r->emacro.data(), 4 * r->emacro.size());
    put(r->elevel.data(), 4 * r->elevel.size());
    put(r->eanchor.data(), 4 * r->eanchor.size());
    put(r->ep.data(), 4 * r->ep.size());
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->stop) throw Error(HPDG_ERR_INVALID_ARG, "server is shutting down");
    r->ticket = sv->next_ticket++;
    r->st.state = HPDG_REQ_QUEUED;
    r->st.submit_ms = sv->now_ms();
    *ticket = r->ticket;
    sv->queue.push_back(r->ticket);
    sv->reqs[r->ticket] = std::move(r);
    sv->cv_work.notify_one();
  });
}

int hpdg_server_poll(hpdg_server* sv, uint64_t ticket, hpdg_request_status* status) {
  if (!sv || !status) return HPDG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HPDG_ERR_INVALID_ARG;
  *status = it->second->st;
  return HPDG_OK;
}

int hpdg_server_wait(hpdg_server* sv, uint64_t ticket, int64_t timeout_ms, hpdg_request_status* status) {
  if (!sv || !status) return HPDG_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lock(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HPDG_ERR_INVALID_ARG;
  ServerRequest* r = it->second.get();
  auto done = [&] { return r->st.state == HPDG_REQ_DONE || r->st.state == HPDG_REQ_FAILED; };
  if (timeout_ms < 0)
    sv->cv_done.wait(lock, done);
  else
    sv->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), done);
  *status = r->st;
  return HPDG_OK;
}

int hpdg_server_destroy(hpdg_server* sv) {
  if (!sv) return HPDG_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->stop = true;
    for (uint64_t t : sv->queue) {
      ServerRequest* r = sv->reqs[t].get();
      r->st.state = HPDG_REQ_FAILED;
      r->st.status = HPDG_ERR_INVALID_ARG;
      std::snprintf(r->st.message, sizeof(r->st.message), "%s", "server destroyed before the request ran");
    }
    sv->queue.clear();
  }
  sv->cv_work.notify_all();
  for (auto& w : sv->workers) w.join();
  sv->cv_done.notify_all();
  (void)hipSetDevice(sv->ctx->device);
  sv->idle.clear();
  delete sv;
  return HPDG_OK;
}

}  // extern "C"
