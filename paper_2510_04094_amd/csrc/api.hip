// Host side of the C ABI: plan creation and validation, workspace layout, and the work
// functions, which only enqueue kernels on the caller's stream.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "nyls_internal.h"

struct nyls_plan {
  int32_t batch = 0, mode = 0, maxm = 0, maxp = 0, maxn = 0;
  int32_t maxm_narrow = 0;  // largest m <= NYLS_NARROW_MAX_M
  int64_t total = 0;        // sum of n
  int64_t ws_doubles = 0;   // per-instance blocks
  int64_t scratch_off = 0;  // explicit-mode scratch (doubles)
  int64_t scratch_doubles = 0;
  bool linear_ok = true;    // every instance has f and r
  bool all_first_order = true;
  unsigned nt_mask = 0;
  unsigned p_mask = 0;
  unsigned rec_mask = 0;
  unsigned nb_mask = 0;
  unsigned gnb_mask = 0;
  unsigned gcls_mask = 0;
  unsigned tl_mask = 0;
  unsigned ntl_mask = 0;
  int32_t n_big = 0;        // instances with m > 64
  int32_t n_split = 0, max_chunks = 0;
  int32_t n_vgram = 0;      // unsplit instances on the LDS-tile FP64 Gram
  int32_t n_vks = 0;        // ... of them whose kernel-space Gram it forms too
  int64_t split_off = 0;       // partial sums of split instances (doubles from ws)
  int64_t split_doubles = 0;
  // work of the one-wave refinement/output passes per (slot class 2, 4, 8 blocks; order p),
  // sum of n (m + 2) over the unsplit instances: the solve shares these launches out over
  // its streams
  double pcost[3][NYLS_MAX_P + 1] = {};
  nyls_tuning tune = {0, 64, 0, 1, 1, -1};
  nyls_desc* d_desc = nullptr;
  int32_t* d_lidx = nullptr;
  int32_t* d_order = nullptr;
  std::vector<nyls_desc> h_desc;
  rocblas_handle blas = nullptr;
  // FP64 solves run the kernel-space Gram on `side` while the eigensolver runs on the
  // caller's stream (fork and join through the events); with bases on both sides of 64
  // landmarks the eigensolver of the m <= 64 ones runs on `side2` (joined by ev_join2).
  // (NYLS_FP64 and NYLS_MIXED plans.)
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  // the refinement/output passes of different slot classes run on the three streams as well
  hipEvent_t ev_fork_p = nullptr, ev_join_p = nullptr, ev_join_p2 = nullptr;
};

namespace {

bool finite(double x) { return std::isfinite(x); }

int validate(const nyls_problem& q, std::vector<int32_t>& lidx) {
  if (q.p < 1 || q.p > NYLS_MAX_P) return NYLS_E_ORDER;
  if (q.n < 2 || q.n > NYLS_MAX_N || q.m < 2 || q.m > q.n || q.m > NYLS_MAX_M) return NYLS_E_SIZE;
  if (!(finite(q.sigma) && q.sigma > 0) || !(finite(q.gamma) && q.gamma > 0) ||
      !(finite(q.tau) && q.tau >= 0 && q.tau < 1))
    return NYLS_E_PARAM;
  if (q.uniform) {
    if (!(finite(q.dt) && q.dt > 0 && finite(q.t0))) return NYLS_E_GRID;
  } else if (!q.t) {
    return NYLS_E_GRID;
  }
  if (!q.v) return NYLS_E_NULL;
  lidx.resize(q.m);
  if (q.lidx) {
    for (int s = 0; s < q.m; ++s) {
      lidx[s] = q.lidx[s];
      if (lidx[s] < 0 || lidx[s] >= q.n || (s > 0 && lidx[s] <= lidx[s - 1])) return NYLS_E_LANDMARK;
    }
  } else {
    // equidistant rule i_s = floor(s (n-1)/(m-1) + 1/2), in integers
    for (int s = 0; s < q.m; ++s)
      lidx[s] = (int32_t)((2LL * s * (q.n - 1) + (q.m - 1)) / (2LL * (q.m - 1)));
  }
  for (int j = 0; j < q.p; ++j) {
    if (q.cond_d[j] < 0 || q.cond_d[j] >= q.p || q.cond_i[j] < 0 || q.cond_i[j] >= q.n)
      return NYLS_E_COND;
    for (int k = 0; k < j; ++k)
      if (q.cond_d[k] == q.cond_d[j] && q.cond_i[k] == q.cond_i[j]) return NYLS_E_COND;
  }
  return NYLS_OK;
}

nyls_plan_view view(const nyls_plan* pl) {
  nyls_plan_view v;
  v.batch = pl->batch;
  v.mode = pl->mode;
  v.maxm = pl->maxm;
  v.maxp = pl->maxp;
  v.maxn = pl->maxn;
  v.maxm_narrow = pl->maxm_narrow;
  v.d_desc = pl->d_desc;
  v.d_order = pl->d_order;
  v.total = pl->total;
  v.nt_mask = pl->nt_mask;
  v.p_mask = pl->p_mask;
  v.rec_mask = pl->rec_mask;
  v.nb_mask = pl->nb_mask;
  v.gnb_mask = pl->gnb_mask;
  v.gcls_mask = pl->gcls_mask;
  v.tl_mask = pl->tl_mask;
  v.ntl_mask = pl->ntl_mask;
  v.n_big = pl->n_big;
  v.n_split = pl->n_split;
  v.n_vgram = pl->n_vgram;
  v.n_vks = pl->n_vks;
  v.max_chunks = pl->max_chunks;
  v.eig_ql = pl->tune.eig_ql;
  v.ql_lanes = pl->tune.ql_lanes;
  v.overlap = pl->tune.overlap;
  v.only = 0;
  return v;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? NYLS_OK : NYLS_E_HIP; }

// --- optional kernel timing -------------------------------------------------------------
struct ProfState {
  int enabled = 0;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  hipEvent_t open[NYLS_K_COUNT] = {};
  double total_ms[NYLS_K_COUNT] = {};
  int64_t count[NYLS_K_COUNT] = {};
};
ProfState g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

}  // namespace

void nyls_prof_begin(int k, hipStream_t st) {
  if (!g_prof.enabled) return;
  hipEvent_t e = prof_event();
  (void)hipEventRecord(e, st);
  g_prof.open[k] = e;
}

void nyls_prof_end(int k, hipStream_t st) {
  if (!g_prof.enabled || !g_prof.open[k]) return;
  hipEvent_t e = prof_event();
  (void)hipEventRecord(e, st);
  g_prof.pending.push_back({k, {g_prof.open[k], e}});
  g_prof.open[k] = nullptr;
}

// Workspace of nyls_solve_static: a file-scope device array, one copy per GPU for the life
// of the process.  Host code never uses the array's name as an address (on the host it is a
// stand-in symbol); the device address of each GPU's copy is looked up once, with that GPU
// current, and kept in g_scratch_ptr.
constexpr size_t NYLS_SCRATCH_DOUBLES = NYLS_STATIC_WS_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[NYLS_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array, or nullptr on failure.
double* scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

// NYLS_MIXED: the FP32 Gram of the bases with m + 2 <= 64; wider ones take the FP64 Gram
// from the start (their FP32 refinement failed on every such instance of the uneven batch,
// and rotating their rows into the eigenbasis costs m^2 multiply-adds per point).
hipError_t launch_gram_mixed(const nyls_plan_view& pv, double* w, hipStream_t stream) {
  hipError_t e = nyls_launch_gram32(pv, w, stream);
  if (e == hipSuccess && (pv.nt_mask >> 5)) e = nyls_launch_gram64_over64(pv, w, stream);
  return e;
}

// Clears n doubles at p (a kernel rather than hipMemsetAsync, so a captured graph replays it
// faithfully).
__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}
}  // namespace

namespace {
// Per-instance kernel choices (nyls_desc::flags) and the launch masks that follow from the
// plan's tuning.
// Grid points per workgroup of split instances for the plan's `split` setting (0: none;
// bases wider than NYLS_NARROW_MAX_M are split whatever it says).
int split_chunk(const nyls_plan* pl) {
  if (pl->mode != NYLS_FP64) return 0;
  if (pl->tune.split > 0) return pl->tune.split;
  if (pl->tune.split == 0 || pl->batch > 64) return 0;
  return 1024;
}

void apply_tuning(nyls_plan* pl) {
  pl->gcls_mask = pl->tl_mask = pl->ntl_mask = 0;
  pl->n_split = pl->max_chunks = pl->n_vgram = pl->n_vks = 0;
  pl->split_off = pl->ws_doubles + pl->scratch_doubles;
  pl->split_doubles = 0;
  for (auto& row : pl->pcost)
    for (double& c : row) c = 0.0;
  const int ch = split_chunk(pl);
  const int min_n = pl->tune.split > 0 ? 0 : 4096;
  const int wide_ch = pl->tune.split > 0 ? pl->tune.split : 1024;
  for (nyls_desc& d : pl->h_desc) {
    int f = 0;
    d.chunk = d.nchunks = 0;
    d.part = 0;
    const bool wide = d.m > NYLS_NARROW_MAX_M;
    if (wide || (ch > 0 && d.n >= min_n)) {
      f |= NYLS_DF_SPLIT;
      d.chunk = wide ? wide_ch : ch;
      d.nchunks = (d.n + d.chunk - 1) / d.chunk;
      d.part = pl->split_off + pl->split_doubles;
      pl->split_doubles += nyls_split_doubles(d.m, d.nchunks);
      ++pl->n_split;
      pl->max_chunks = std::max(pl->max_chunks, d.nchunks);
    }
    if (pl->tune.tail_layout && d.rec == 1 && nyls_walk_tail(d.m) != 0 && !(f & NYLS_DF_SPLIT))
      f |= NYLS_DF_TAIL;
    if (pl->tune.tail_layout && (nyls_gram_class(d.m) & 1)) f |= NYLS_DF_GRAM_TAIL;
    if (pl->tune.gram_valu && d.m + 2 <= 64 && pl->mode == NYLS_FP64) f |= NYLS_DF_GRAM_VALU;
    d.flags = f;
    if (!(f & NYLS_DF_SPLIT) && (d.m + 2 > 64 || (f & NYLS_DF_GRAM_VALU))) ++pl->n_vgram;
    if (!(f & NYLS_DF_SPLIT) && (d.m + 2 > NYLS_GRAM4_MAX_G || (f & NYLS_DF_GRAM_VALU))) ++pl->n_vks;
    if (d.m + 2 <= 64 && !(f & NYLS_DF_GRAM_VALU)) pl->gcls_mask |= 1u << nyls_gram_class_of(d);
    if (f & NYLS_DF_TAIL) pl->tl_mask |= 1u << nyls_slot_blocks(d.m);
    else pl->ntl_mask |= 1u << nyls_slot_blocks(d.m);
    if (!(f & NYLS_DF_SPLIT) && d.m <= NYLS_NARROW_MAX_M) {
      const int nb = nyls_slot_blocks(d.m);
      pl->pcost[nb == 2 ? 0 : (nb == 4 ? 1 : 2)][d.p] += (double)d.n * (d.m + 2);
    }
  }
}
}  // namespace

// accessors used by the other translation units
int64_t nyls_plan_newton_stride(const nyls_plan* pl) {
  return pl ? (int64_t)pl->maxm + 1 + pl->maxp + pl->maxn : 0;
}
bool nyls_plan_first_order(const nyls_plan* pl) { return pl && pl->all_first_order; }
// The ODE order shared by every instance of the plan, or 0 when the orders differ.
int nyls_plan_common_order(const nyls_plan* pl) {
  if (!pl) return 0;
  const unsigned pm = pl->p_mask;
  return (pm & (pm - 1)) ? 0 : __builtin_ctz(pm);
}
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl) { return view(pl); }

extern "C" {

int nyls_plan_create(const nyls_problem* probs, int32_t batch, int32_t mode, nyls_plan** out) {
  if (!out) return NYLS_E_NULL;
  *out = nullptr;
  if (!probs) return NYLS_E_NULL;
  if (batch < 1) return NYLS_E_BATCH;
  if (mode != NYLS_FP64 && mode != NYLS_MIXED && mode != NYLS_FP64_EXPLICIT) return NYLS_E_MODE;
  nyls_plan* pl = new (std::nothrow) nyls_plan;
  if (!pl) return NYLS_E_HIP;
  pl->batch = batch;
  pl->mode = mode;
  pl->h_desc.resize(batch);
  std::vector<int32_t> all_lidx, lid;
  std::vector<int64_t> lidx_off(batch);
  int64_t wsd = 0, goff = 0;
  for (int i = 0; i < batch; ++i) {
    const nyls_problem& q = probs[i];
    int rc = validate(q, lid);
    if (rc == NYLS_OK && mode == NYLS_MIXED && q.m > 126) rc = NYLS_E_SIZE;
    if (rc == NYLS_OK && mode != NYLS_FP64 && q.m > NYLS_NARROW_MAX_M) rc = NYLS_E_SIZE;
    if (rc != NYLS_OK) { delete pl; return rc; }
    if (!q.f || !q.r) pl->linear_ok = false;
    if (q.p != 1) pl->all_first_order = false;
    nyls_desc& d = pl->h_desc[i];
    d.p = q.p; d.n = q.n; d.m = q.m; d.uniform = q.uniform ? 1 : 0;
    d.t0 = q.t0; d.dt = q.dt; d.t = q.t; d.f = q.f; d.r = q.r; d.v = q.v;
    for (int j = 0; j < NYLS_MAX_P; ++j) {
      d.cond_d[j] = j < q.p ? q.cond_d[j] : 0;
      d.cond_i[j] = j < q.p ? q.cond_i[j] : -1;
    }
    d.sigma = q.sigma; d.gamma = q.gamma; d.tau = q.tau;
    {
      const double a = q.uniform ? q.dt / q.sigma : 0.0;
      d.rec = (q.uniform && a <= 0.25) ? 1 : 0;
      d.flags = 0;  // apply_tuning
    }
    d.ws = wsd;
    d.goff = goff;
    wsd += nyls_layout(q.m, q.p, q.p == 1 ? q.n : 0).end;
    goff += q.n;
    lidx_off[i] = (int64_t)all_lidx.size();
    all_lidx.insert(all_lidx.end(), lid.begin(), lid.end());
    pl->nt_mask |= 1u << ((q.m + 2 + 15) / 16);
    pl->p_mask |= 1u << q.p;
    pl->rec_mask |= 1u << d.rec;
    pl->nb_mask |= 1u << nyls_slot_blocks(q.m);
    pl->gnb_mask |= 1u << nyls_slot_blocks(q.m + 2);
    if (q.m > 64) ++pl->n_big;
    pl->maxm = std::max(pl->maxm, q.m);
    if (q.m <= NYLS_NARROW_MAX_M) pl->maxm_narrow = std::max(pl->maxm_narrow, q.m);
    pl->maxp = std::max(pl->maxp, q.p);
    pl->maxn = std::max(pl->maxn, q.n);
  }
  pl->total = goff;
  pl->ws_doubles = wsd;
  pl->scratch_off = wsd;
  pl->scratch_doubles = 0;
  if (mode == NYLS_FP64_EXPLICIT) {
    const int64_t nn = pl->maxn, mm = pl->maxm;
    pl->scratch_doubles = nn * (NYLS_MAX_P + 1) * mm + nn * (mm + 2) + (mm + 2) * (mm + 2) + 64;
  }
  apply_tuning(pl);
  // explicit grids must be strictly ascending (checked on a host copy)
  for (int i = 0; i < batch; ++i) {
    if (probs[i].uniform) continue;
    std::vector<double> t(probs[i].n);
    if (hipMemcpy(t.data(), probs[i].t, sizeof(double) * t.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      delete pl;
      return NYLS_E_HIP;
    }
    for (size_t k = 1; k < t.size(); ++k)
      if (!(t[k] > t[k - 1])) { delete pl; return NYLS_E_GRID; }
  }
  // instance order: most expensive first (n m^2), ties by index
  std::vector<int32_t> order(batch);
  for (int i = 0; i < batch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = (double)probs[a].n * probs[a].m * probs[a].m;
    const double cb = (double)probs[b].n * probs[b].m * probs[b].m;
    return ca > cb;
  });
  bool ok = hipMalloc(&pl->d_lidx, sizeof(int32_t) * all_lidx.size()) == hipSuccess &&
            hipMalloc(&pl->d_desc, sizeof(nyls_desc) * batch) == hipSuccess &&
            hipMalloc(&pl->d_order, sizeof(int32_t) * batch) == hipSuccess;
  if (ok) {
    for (int i = 0; i < batch; ++i) pl->h_desc[i].lidx = pl->d_lidx + lidx_off[i];
    ok = hipMemcpy(pl->d_lidx, all_lidx.data(), sizeof(int32_t) * all_lidx.size(),
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(pl->d_desc, pl->h_desc.data(), sizeof(nyls_desc) * batch,
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(pl->d_order, order.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) ==
             hipSuccess;
  }
  if (ok && mode == NYLS_FP64_EXPLICIT) ok = rocblas_create_handle(&pl->blas) == rocblas_status_success;
  if (ok && mode != NYLS_FP64_EXPLICIT)
    ok = hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&pl->side2, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_join2, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_fork_p, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_join_p, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->ev_join_p2, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    nyls_plan_destroy(pl);
    return NYLS_E_HIP;
  }
  *out = pl;
  return NYLS_OK;
}

void nyls_plan_destroy(nyls_plan* pl) {
  if (!pl) return;
  if (pl->blas) rocblas_destroy_handle(pl->blas);
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  if (pl->ev_join2) (void)hipEventDestroy(pl->ev_join2);
  if (pl->ev_fork_p) (void)hipEventDestroy(pl->ev_fork_p);
  if (pl->ev_join_p) (void)hipEventDestroy(pl->ev_join_p);
  if (pl->ev_join_p2) (void)hipEventDestroy(pl->ev_join_p2);
  if (pl->side) (void)hipStreamDestroy(pl->side);
  if (pl->side2) (void)hipStreamDestroy(pl->side2);
  if (pl->d_desc) (void)hipFree(pl->d_desc);
  if (pl->d_lidx) (void)hipFree(pl->d_lidx);
  if (pl->d_order) (void)hipFree(pl->d_order);
  delete pl;
}

}  // extern "C"

namespace {
__global__ void k_set_params(nyls_desc* __restrict__ desc, const double* __restrict__ sigma,
                             const double* __restrict__ gamma, int32_t* __restrict__ status, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  nyls_desc& d = desc[i];
  const double s = sigma ? sigma[i] : d.sigma, g = gamma ? gamma[i] : d.gamma;
  const bool ok = isfinite(s) && s > 0.0 && isfinite(g) && g > 0.0 && (d.rec != 1 || d.dt <= 0.25 * s);
  if (ok) {
    d.sigma = s;
    d.gamma = g;
  }
  if (status) status[i] = ok ? 0 : NYLS_S_PARAM_KEPT;
}
}  // namespace

extern "C" {

int nyls_plan_set_params(nyls_plan* pl, const double* sigma, const double* gamma, int32_t* status,
                         hipStream_t stream) {
  if (!pl) return NYLS_E_NULL;
  hipLaunchKernelGGL(k_set_params, dim3((pl->batch + 255) / 256), dim3(256), 0, stream, pl->d_desc, sigma,
                     gamma, status, pl->batch);
  return hip_rc(hipGetLastError());
}

int nyls_plan_set_tuning(nyls_plan* pl, const nyls_tuning* t) {
  if (!pl || !t) return NYLS_E_NULL;
  if ((t->eig_ql != 0 && t->eig_ql != 1) || t->ql_lanes < 1 || t->ql_lanes > 64 ||
      (t->gram_valu != 0 && t->gram_valu != 1) || (t->tail_layout != 0 && t->tail_layout != 1) ||
      (t->overlap != 0 && t->overlap != 1) ||
      (t->split != -1 && t->split != 0 && (t->split < 512 || t->split % 64 != 0 || t->split > (1 << 24))))
    return NYLS_E_ARG;
  // sigma and gamma may have been changed on the device (nyls_plan_set_params): keep them
  std::vector<nyls_desc> cur(pl->batch);
  if (hipMemcpy(cur.data(), pl->d_desc, sizeof(nyls_desc) * pl->batch, hipMemcpyDeviceToHost) != hipSuccess)
    return NYLS_E_HIP;
  for (int i = 0; i < pl->batch; ++i) {
    pl->h_desc[i].sigma = cur[i].sigma;
    pl->h_desc[i].gamma = cur[i].gamma;
  }
  pl->tune = *t;
  apply_tuning(pl);
  return hipMemcpy(pl->d_desc, pl->h_desc.data(), sizeof(nyls_desc) * pl->batch,
                   hipMemcpyHostToDevice) == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}

int nyls_plan_get_tuning(const nyls_plan* pl, nyls_tuning* t) {
  if (!pl || !t) return NYLS_E_NULL;
  *t = pl->tune;
  return NYLS_OK;
}

size_t nyls_workspace_size(const nyls_plan* pl) {
  if (!pl) return 0;
  return (size_t)(pl->ws_doubles + pl->scratch_doubles + pl->split_doubles) * sizeof(double);
}

int64_t nyls_total_points(const nyls_plan* pl) { return pl ? pl->total : 0; }

int32_t nyls_max_m(const nyls_plan* pl) { return pl ? pl->maxm : 0; }

namespace {
__global__ void k_instance_info(const nyls_desc* __restrict__ desc, const double* __restrict__ ws,
                                double* __restrict__ info, int batch) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= batch * 8) return;
  const int i = e >> 3, k = e & 7;
  const nyls_desc& d = desc[i];
  info[e] = ws[d.ws + nyls_layout(d.m, d.p, 0).info + k];
}

// Grid (instance, tiles of 256 entries of the MAXM x MAXM output).
__global__ void k_basis(const nyls_desc* __restrict__ desc, const double* __restrict__ ws,
                        double* __restrict__ lam, double* __restrict__ U, int maxm) {
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  const double* w = ws + d.ws;
  const int e = (int)blockIdx.y * blockDim.x + (int)threadIdx.x;
  if (lam && blockIdx.y == 0 && (int)threadIdx.x < maxm) {
    const int k = threadIdx.x;
    lam[(size_t)blockIdx.x * maxm + k] = k < m ? w[L.lam + k] : 0.0;
  }
  if (!U || e >= maxm * maxm) return;
  const int s = e / maxm, k = e - s * maxm;
  U[(size_t)blockIdx.x * maxm * maxm + e] = (s < m && k < m) ? w[L.U + s * m + k] : 0.0;
}
}  // namespace

int nyls_basis(const nyls_plan* pl, const void* ws, double* lam, double* U, hipStream_t stream) {
  if (!pl || !ws) return NYLS_E_NULL;
  if (!lam && !U) return NYLS_OK;
  const int threads = 256, maxm = pl->maxm;
  const dim3 grid(pl->batch, (maxm * maxm + threads - 1) / threads);
  hipLaunchKernelGGL(k_basis, grid, dim3(threads), 0, stream, pl->d_desc,
                     static_cast<const double*>(ws), lam, U, maxm);
  return hip_rc(hipGetLastError());
}

int nyls_instance_info(const nyls_plan* pl, const void* ws, double* info, hipStream_t stream) {
  if (!pl || !ws || !info) return NYLS_E_NULL;
  const int threads = 256, blocks = (pl->batch * 8 + threads - 1) / threads;
  hipLaunchKernelGGL(k_instance_info, dim3(blocks), dim3(threads), 0, stream, pl->d_desc,
                     static_cast<const double*>(ws), info, pl->batch);
  return hip_rc(hipGetLastError());
}

int nyls_features(const nyls_plan* pl, const double* t_eval, const int64_t* eval_off, int32_t dmax,
                  double* phi, double* eigval, int32_t* rank, void* ws, hipStream_t stream) {
  if (!pl || !t_eval || !eval_off || !phi || !ws) return NYLS_E_NULL;
  if (dmax < 0 || dmax > NYLS_MAX_P) return NYLS_E_ARG;
  const nyls_plan_view pv = view(pl);
  double* w = static_cast<double*>(ws);
  nyls_prof_begin(NYLS_K_EIG, stream);
  hipError_t e = nyls_launch_eig(pv, w, -1, stream);
  nyls_prof_end(NYLS_K_EIG, stream);
  nyls_prof_begin(NYLS_K_FEATURES, stream);
  if (e == hipSuccess)
    e = nyls_launch_features(pv, w, t_eval, eval_off, dmax, phi, eigval, rank, 1 << 20, -1, stream);
  nyls_prof_end(NYLS_K_FEATURES, stream);
  return hip_rc(e);
}

int nyls_assemble(const nyls_plan* pl, double* kkt, double* rhs, void* ws, hipStream_t stream) {
  if (!pl || !kkt || !rhs || !ws) return NYLS_E_NULL;
  if (!pl->linear_ok) return NYLS_E_NULL;
  const nyls_plan_view pv = view(pl);
  double* w = static_cast<double*>(ws);
  hipError_t e = nyls_launch_eig(pv, w, -1, stream);
  if (e == hipSuccess)
    e = (pl->mode == NYLS_MIXED) ? launch_gram_mixed(pv, w, stream) : nyls_launch_gram64(pv, w, stream);
  if (e == hipSuccess) e = nyls_launch_kkt(pv, w, kkt, rhs, 0, stream);
  return hip_rc(e);
}

}  // extern "C"

namespace {
// The solve of nyls_solve / nyls_solve_static with the workspace at w.
int solve_impl(const nyls_plan* pl, int32_t refine_steps, double* omega, double* bias,
               double* lambda, double* yhat, int32_t* status, double* w, hipStream_t stream) {
  const nyls_plan_view pv = view(pl);
  hipError_t e = hipSuccess;
  if (pl->mode == NYLS_FP64_EXPLICIT) {
    double* scratch = w + pl->scratch_off;
    rocblas_set_stream(pl->blas, stream);
    for (int i = 0; i < pl->batch && e == hipSuccess; ++i) {
      const nyls_desc& d = pl->h_desc[i];
      const int g = d.m + 2;
      double* phi = scratch;
      double* rows = phi + (int64_t)pl->maxn * (NYLS_MAX_P + 1) * pl->maxm;
      double* C = rows + (int64_t)pl->maxn * (pl->maxm + 2);
      e = nyls_launch_eig(pv, w, i, stream);
      if (e == hipSuccess)
        e = nyls_launch_features(pv, w, nullptr, nullptr, d.p, phi, nullptr, nullptr, d.n, i, stream);
      if (e == hipSuccess) e = nyls_launch_explicit_rows(pv, i, w, phi, rows, d.n, d.m, stream);
      if (e == hipSuccess) {
        // C (g x g, row-major == column-major symmetric) = rows^T rows; rows is n x g row-major,
        // i.e. a column-major g x n matrix A with lda = g:  C = A A^T.
        const double one = 1.0, zero = 0.0;
        if (rocblas_dgemm(pl->blas, rocblas_operation_none, rocblas_operation_transpose, g, g, d.n,
                          &one, rows, g, rows, g, &zero, C, g) != rocblas_status_success)
          e = hipErrorUnknown;
      }
      if (e == hipSuccess) e = nyls_launch_explicit_kkt(pv, i, w, phi, C, stream);
      if (e == hipSuccess)
        e = nyls_launch_points(pv, w, refine_steps, yhat, omega, bias, lambda, status, i, stream);
    }
    return hip_rc(e);
  }
  if (pl->mode == NYLS_FP64 && !pl->tune.overlap) {
    nyls_prof_begin(NYLS_K_EIG, stream);
    e = nyls_launch_eig(pv, w, -1, stream);
    nyls_prof_end(NYLS_K_EIG, stream);
    nyls_prof_begin(NYLS_K_GRAM64, stream);
    if (e == hipSuccess) e = nyls_launch_gram64(pv, w, stream);
    nyls_prof_end(NYLS_K_GRAM64, stream);
  } else if (pl->mode == NYLS_FP64) {
    // The kernel-space Grams need nothing from the eigensolver, and the eigensolver is
    // latency-bound (part of it runs one lane per instance on a few CUs): the Grams run on
    // the side stream meanwhile, and the eigenbasis Grams that replace them where K_mm is
    // ill-conditioned follow the join.
    // With bases on both sides of 64 landmarks the two eigensolver paths (disjoint
    // instances, each latency-bound on few CUs) run side by side as well.
    const bool split_eig = (pv.nb_mask & (4 | 16)) && (pv.nb_mask & (256 | (1u << 16)));
    e = hipEventRecord(pl->ev_fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->side, pl->ev_fork, 0);
    if (e == hipSuccess && split_eig) e = hipStreamWaitEvent(pl->side2, pl->ev_fork, 0);
    // (the eigensolver of the larger bases, the longest chain, is enqueued first)
    nyls_prof_begin(NYLS_K_EIG, stream);
    if (e == hipSuccess && split_eig) e = nyls_launch_eig(pv, w, -1, stream, NYLS_EIG_BIG);
    nyls_prof_begin(NYLS_K_GRAM64, pl->side);
    if (e == hipSuccess) e = nyls_launch_gram64_kspace(pv, w, pl->side);
    nyls_prof_end(NYLS_K_GRAM64, pl->side);
    hipError_t ej = hipEventRecord(pl->ev_join, pl->side);
    hipError_t ej2 = hipSuccess;
    if (split_eig) {
      if (e == hipSuccess) e = nyls_launch_eig(pv, w, -1, pl->side2, NYLS_EIG_NARROW);
      ej2 = hipEventRecord(pl->ev_join2, pl->side2);
    }
    if (e == hipSuccess && !split_eig) e = nyls_launch_eig(pv, w, -1, stream);
    nyls_prof_end(NYLS_K_EIG, stream);
    // joined whatever happened above, so no work is left running on the side streams
    if (ej == hipSuccess) ej = hipStreamWaitEvent(stream, pl->ev_join, 0);
    if (split_eig && ej2 == hipSuccess) ej2 = hipStreamWaitEvent(stream, pl->ev_join2, 0);
    if (e == hipSuccess) e = ej;
    if (e == hipSuccess) e = ej2;
    if (e == hipSuccess) e = nyls_launch_gram64_rest(pv, w, stream, true);
  } else {
    nyls_prof_begin(NYLS_K_EIG, stream);
    e = nyls_launch_eig(pv, w, -1, stream);
    nyls_prof_end(NYLS_K_EIG, stream);
    nyls_prof_begin(NYLS_K_GRAM32, stream);
    if (e == hipSuccess) e = launch_gram_mixed(pv, w, stream);
    nyls_prof_end(NYLS_K_GRAM32, stream);
  }
  nyls_prof_begin(NYLS_K_KKT, stream);
  if (e == hipSuccess) e = nyls_launch_kkt(pv, w, nullptr, nullptr, 1, stream);
  nyls_prof_end(NYLS_K_KKT, stream);
  nyls_prof_begin(NYLS_K_POINTS, stream);
  // the one-wave pass launches, one per (slot class, order p) present, largest work first
  struct pitem { double cost; unsigned cls; int p; };
  pitem items[3 * NYLS_MAX_P];
  int nitems = 0;
  for (int c = 0; c < 3; ++c)
    for (int p = 1; p <= NYLS_MAX_P; ++p)
      if (pl->pcost[c][p] > 0.0) items[nitems++] = {pl->pcost[c][p], 1u << (2 << c), p};
  std::sort(items, items + nitems, [](const pitem& a, const pitem& b) { return a.cost > b.cost; });
  if (e == hipSuccess && pl->side && pl->tune.overlap && nitems >= 2) {
    // several such launches (disjoint instances; each holds only its own instances'
    // wavefronts): shared out over the three streams, each to the least loaded so far, the
    // split instances here; joined before anything else reads the solution
    e = hipEventRecord(pl->ev_fork_p, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->side, pl->ev_fork_p, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->side2, pl->ev_fork_p, 0);
    hipStream_t sts[3] = {stream, pl->side, pl->side2};
    double load[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nitems && e == hipSuccess; ++k) {
      const int t = load[0] <= load[1] ? (load[0] <= load[2] ? 0 : 2) : (load[1] <= load[2] ? 1 : 2);
      load[t] += items[k].cost;
      nyls_plan_view pq = pv;
      pq.p_mask = pv.p_mask & (1u << items[k].p);
      e = nyls_launch_points(pq, w, refine_steps, yhat, omega, bias, lambda, status, -1, sts[t], items[k].cls);
    }
    if (e == hipSuccess)
      e = nyls_launch_points(pv, w, refine_steps, yhat, omega, bias, lambda, status, -1, stream, 1);
    hipError_t ej = hipEventRecord(pl->ev_join_p, pl->side);
    hipError_t ej2 = hipEventRecord(pl->ev_join_p2, pl->side2);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(stream, pl->ev_join_p, 0);
    if (ej2 == hipSuccess) ej2 = hipStreamWaitEvent(stream, pl->ev_join_p2, 0);
    if (e == hipSuccess) e = ej;
    if (e == hipSuccess) e = ej2;
  } else if (e == hipSuccess) {
    e = nyls_launch_points(pv, w, refine_steps, yhat, omega, bias, lambda, status, -1, stream);
  }
  nyls_prof_end(NYLS_K_POINTS, stream);
  if (pl->mode == NYLS_MIXED && refine_steps > 0 && e == hipSuccess) {
    // Instances whose refinement on the FP32 Gram did not converge (K_mm too ill-conditioned
    // for FP32 features) are solved again with the FP64 Gram in the eigenbasis; the kernels
    // of this second round leave every other instance untouched.
    nyls_plan_view rv = pv;
    rv.only = NYLS_S_REFINE_NOCONV;
    nyls_prof_begin(NYLS_K_GRAM64, stream);
    e = nyls_launch_gram64(rv, w, stream);
    nyls_prof_end(NYLS_K_GRAM64, stream);
    nyls_prof_begin(NYLS_K_KKT, stream);
    if (e == hipSuccess) e = nyls_launch_kkt(rv, w, nullptr, nullptr, 1, stream);
    nyls_prof_end(NYLS_K_KKT, stream);
    nyls_prof_begin(NYLS_K_POINTS, stream);
    if (e == hipSuccess)
      e = nyls_launch_points(rv, w, refine_steps, yhat, omega, bias, lambda, status, -1, stream);
    nyls_prof_end(NYLS_K_POINTS, stream);
  }
  return hip_rc(e);
}
}  // namespace

extern "C" {

int nyls_solve(const nyls_plan* pl, int32_t refine_steps, double* omega, double* bias,
               double* lambda, double* yhat, int32_t* status, void* ws, hipStream_t stream) {
  if (!pl || !yhat || !ws) return NYLS_E_NULL;
  if (!pl->linear_ok) return NYLS_E_NULL;
  if (refine_steps < 0 || refine_steps > 8) return NYLS_E_ARG;
  return solve_impl(pl, refine_steps, omega, bias, lambda, yhat, status, static_cast<double*>(ws),
                    stream);
}

int nyls_solve_static(const nyls_plan* pl, int32_t refine_steps, double* omega, double* bias,
                      double* lambda, double* yhat, int32_t* status, hipStream_t stream) {
  if (!pl || !yhat) return NYLS_E_NULL;
  if (!pl->linear_ok) return NYLS_E_NULL;
  if (pl->mode == NYLS_FP64_EXPLICIT) return NYLS_E_MODE;  // its GEMM library may allocate
  if (refine_steps < 0 || refine_steps > 8) return NYLS_E_ARG;
  const size_t bytes = nyls_workspace_size(pl);
  if (bytes > NYLS_STATIC_WS_BYTES) return NYLS_E_SIZE;
  double* w = scratch_for_current_device();
  if (!w) return NYLS_E_HIP;
  // the array keeps the previous call's contents: start from zeros, as a fresh workspace
  const int64_t nd = (int64_t)(bytes / sizeof(double));
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nd + 255) / 256));
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, stream, w, nd);
  if (hipGetLastError() != hipSuccess) return NYLS_E_HIP;
  return solve_impl(pl, refine_steps, omega, bias, lambda, yhat, status, w, stream);
}

int nyls_predict(const nyls_plan* pl, const double* t_eval, const int64_t* eval_off, int32_t d,
                 double* out, const void* ws, hipStream_t stream) {
  if (!pl || !t_eval || !eval_off || !out || !ws) return NYLS_E_NULL;
  if (d < 0 || d > NYLS_MAX_P) return NYLS_E_ARG;
  nyls_prof_begin(NYLS_K_PREDICT, stream);
  const hipError_t e = nyls_launch_predict(view(pl), static_cast<const double*>(ws), t_eval, eval_off,
                                           d, out, 1 << 20, stream);
  nyls_prof_end(NYLS_K_PREDICT, stream);
  return hip_rc(e);
}

void nyls_profile_enable(int32_t on) { g_prof.enabled = on ? 1 : 0; }

int nyls_profile_read(int32_t kernel, double* total_ms, int64_t* count) {
  if (kernel < 0 || kernel >= NYLS_K_COUNT || !total_ms || !count) return NYLS_E_ARG;
  for (auto& pr : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second.second) != hipSuccess) return NYLS_E_HIP;
    if (hipEventElapsedTime(&ms, pr.second.first, pr.second.second) != hipSuccess) return NYLS_E_HIP;
    g_prof.total_ms[pr.first] += ms;
    g_prof.count[pr.first] += 1;
    g_prof.pool.push_back(pr.second.first);
    g_prof.pool.push_back(pr.second.second);
  }
  g_prof.pending.clear();
  *total_ms = g_prof.total_ms[kernel];
  *count = g_prof.count[kernel];
  return NYLS_OK;
}

void nyls_profile_reset(void) {
  int64_t c;
  double t;
  nyls_profile_read(0, &t, &c);
  for (int k = 0; k < NYLS_K_COUNT; ++k) { g_prof.total_ms[k] = 0.0; g_prof.count[k] = 0; }
}

const char* nyls_error_string(int32_t code) {
  switch (code) {
    case NYLS_OK: return "ok";
    case NYLS_E_NULL: return "a required pointer is NULL";
    case NYLS_E_BATCH: return "batch must be >= 1";
    case NYLS_E_MODE: return "unknown or unsupported mode";
    case NYLS_E_ORDER: return "ODE order p outside 1..4";
    case NYLS_E_SIZE:
      return "need 2 <= m <= n and m <= 256 (m <= 126 in NYLS_MIXED; m <= 128 in NYLS_FP64_EXPLICIT and "
             "for the Newton and leverage calls)";
    case NYLS_E_PARAM: return "need sigma > 0, gamma > 0, 0 <= tau < 1 (finite)";
    case NYLS_E_GRID: return "grid: dt <= 0 or explicit times missing / not ascending";
    case NYLS_E_LANDMARK: return "landmark indices not strictly ascending inside [0, n)";
    case NYLS_E_COND: return "condition order or index out of range, or duplicated";
    case NYLS_E_NONLINEAR: return "Newton calls need instances all of order 1 or all of order 2";
    case NYLS_E_HIP: return "HIP runtime error";
    case NYLS_E_ARG: return "argument out of range";
    case NYLS_S_TRUNCATED: return "basis truncated (r < m)";
    case NYLS_S_SINGULAR: return "zero pivot in the factorisation";
    case NYLS_S_NONFINITE: return "non-finite value in the solution";
    case NYLS_S_EIG_NOCONV: return "eigensolver hit its iteration limit";
    case NYLS_S_SMALL_PIVOT: return "Newton diagonal block entry below 1e-10 gamma (kept in the dense system)";
    case NYLS_S_PIVOT_OVERFLOW: return "more than 32 small Newton pivots, or a non-finite one";
    case NYLS_S_REFINE_NOCONV: return "iterative refinement did not reach rounding level";
    case NYLS_S_FP64_RESOLVED: return "solved again with the FP64 Gram";
    case NYLS_S_PARAM_KEPT: return "new sigma or gamma not taken";
    default: return "unknown code";
  }
}

}  // extern "C"
