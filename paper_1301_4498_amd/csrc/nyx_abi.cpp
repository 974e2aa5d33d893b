// nyx_abi.cpp -- the C ABI of include/nyx_hydro.h: argument validation,
// workspace layout, batched plans and dispatch to the stage kernels.
// Validation runs on the host before anything is enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "nyx_internal.h"

using namespace nyx;

// Scratch of the allocation-free single-box step (nyx_hydro_step_noalloc): a
// file-scope device array that every call on a GPU shares.  In host code
// `scratch` only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (scratch_address below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// Single-box workspace header: [0, 256) running maximum of the CFL reduction,
// then kStatSlots x kStatFields partial counters, the one-entry box table, its
// block prefixes and the box's step constants; stage arrays follow.
constexpr size_t kSlotBytes = sizeof(unsigned long long) * kStatSlots * kStatFields;
constexpr size_t kOffSlots = 256;
constexpr size_t kOffTable = kOffSlots + (kSlotBytes + 255) / 256 * 256;
constexpr size_t kOffPrefix = kOffTable + 512;
constexpr size_t kOffConsts = kOffPrefix + 256;
constexpr size_t kHeaderBytes = kOffConsts + 256;
static_assert(sizeof(BoxDev) <= 512 && sizeof(StepC) <= 256, "header slots");

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_params(const nyx_params* p) {
  if (!p) return NYX_E_NULL;
  if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) return NYX_E_PARAM;
  if (!(std::isfinite(p->eta_dual) && p->eta_dual >= 0.0)) return NYX_E_PARAM;
  if (!finite_pos(p->small_dens) || !finite_pos(p->small_pres)) return NYX_E_PARAM;
  if (!finite_pos(p->riemann_tol)) return NYX_E_PARAM;
  if (!finite_pos(p->cfl)) return NYX_E_PARAM;
  if (!(std::isfinite(p->mixed_riemann_stop) && p->mixed_riemann_stop >= 0.0)) return NYX_E_PARAM;
  if (p->riemann_maxiter < 1 || p->riemann_maxiter > 64) return NYX_E_PARAM;
  if (p->precision != NYX_FP64 && p->precision != NYX_MIXED) return NYX_E_PARAM;
  if (p->riemann != NYX_RIEMANN_TWOSHOCK && p->riemann != NYX_RIEMANN_LEARNED &&
      p->riemann != NYX_RIEMANN_LINEARIZED)
    return NYX_E_PARAM;
  if (p->recon != NYX_RECON_PPM && p->recon != NYX_RECON_PLM) return NYX_E_PARAM;
  if (p->grav_energy_form != 1 && p->grav_energy_form != 2) return NYX_E_PARAM;
  if (p->riemann == NYX_RIEMANN_LEARNED) {
    if (p->precision != NYX_MIXED) return NYX_E_UNSUPPORTED;
    if (!p->mlp_weights) return NYX_E_NULL;
    if ((uintptr_t)p->mlp_weights & 15) return NYX_E_PARAM;
    if (p->learned_stages_mask < 1 || p->learned_stages_mask > 7) return NYX_E_PARAM;
    if (!(std::isfinite(p->mlp_resid_tol) && p->mlp_resid_tol >= 0.0)) return NYX_E_PARAM;
  }
  return NYX_OK;
}

int check_box(const nyx_box* b) {
  if (!b) return NYX_E_NULL;
  for (int d = 0; d < 3; ++d)
    if (b->n[d] < 2 || (b->n[d] & 1) || b->n[d] > (1 << 20)) return NYX_E_SHAPE;
  if (b->ng < 4 || b->ng > 64) return NYX_E_SHAPE;
  long long P = 1;
  for (int d = 0; d < 3; ++d) P *= (long long)(b->n[d] + 2 * b->ng);
  if (P >= (1ll << 29)) return NYX_E_SHAPE;  // per-box byte offsets of FP64 arrays are 32-bit
  if (b->comp_stride < P || b->grav_stride < P) return NYX_E_SHAPE;
  if (b->state_off < 0 || b->grav_off < 0) return NYX_E_SHAPE;
  if (!finite_pos(b->dx)) return NYX_E_PARAM;
  return NYX_OK;
}

size_t real_bytes(const nyx_params* p) { return p->precision == NYX_MIXED ? 4 : 8; }

long long blocks_for(long long n) { return (n + kBlock - 1) / kBlock; }

void set_blocks(const BoxDev& b, int* nb) {
  nb[kSpaceP] = (int)blocks_for(b.P);
  nb[kSpaceE] = (int)blocks_for(b.E);
  nb[kSpaceV] = (int)blocks_for(b.V);
  nb[kSpaceT] = b.ntiles;
  nb[kSpaceF] = b.fbx;
}

// [a0, a0 + alen) and [b0, b0 + blen) in bytes
bool overlaps(const void* a, size_t alen, const void* b, size_t blen) {
  uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + blen && y < x + alen;
}

size_t state_span_bytes(const nyx_box& b) {
  long long P = (long long)(b.n[0] + 2 * b.ng) * (b.n[1] + 2 * b.ng) * (b.n[2] + 2 * b.ng);
  return (size_t)(b.state_off + 5 * b.comp_stride + P) * sizeof(double);
}

void fill_physics(StepArgs& a, const nyx_params* p) {
  a.gamma = p->gamma;
  a.igm1 = 1.0 / (p->gamma - 1.0);
  a.igm1f = 1.0f / (float)(p->gamma - 1.0);
  a.eta = p->eta_dual;
  a.small_dens = p->small_dens;
  a.small_pres = p->small_pres;
  a.riemann_tol = p->riemann_tol;
  // FP32-mixed stopping step: the star state is stored in FP32, so the
  // iteration stops once the next Newton correction would be far below FP32
  // resolution (see two_shock in the mixed build).
  a.mixed_stop = p->mixed_riemann_stop > 0.0 ? p->mixed_riemann_stop
                                               : std::max(std::sqrt(p->riemann_tol), 0x1p-12);
  a.cfl = p->cfl;
  a.maxiter = p->riemann_maxiter;
  const bool learned = p->riemann == NYX_RIEMANN_LEARNED;
  a.mlp = learned ? p->mlp_weights : nullptr;
  a.learned_mask = learned ? p->learned_stages_mask : 0;
  a.mlp_tol = p->mlp_resid_tol;
  a.recon = p->recon;
  a.grav_form = p->grav_energy_form;
  a.linear_riemann = p->riemann == NYX_RIEMANN_LINEARIZED ? 1 : 0;
  // the expansion term's coefficient 2 - 3(gamma-1) is exactly 0.0 in FP64
  // for gamma = 5/3; the term is then skipped
  a.expansion = (2.0 - 3.0 * (p->gamma - 1.0)) != 0.0 ? 1 : 0;
}

// ---- stage timing ----
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t*> pending, free_;
  double ms[kStages] = {0};
  long long seq = 0;
};
Profiler& prof() {
  static Profiler p;
  return p;
}

hipEvent_t* take_events() {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on) return nullptr;
  hipEvent_t* ev;
  if (!P.free_.empty()) {
    ev = P.free_.back();
    P.free_.pop_back();
  } else {
    ev = new (std::nothrow) hipEvent_t[kStages + 1];
    if (!ev) return nullptr;
    for (int i = 0; i <= kStages; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) return nullptr;
  }
  P.pending.push_back(ev);
  return ev;
}

hipError_t run_stages(const nyx_params* p, StepArgs a, hipStream_t s, bool timed = true) {
  a.ev = timed ? take_events() : nullptr;
  return p->precision == NYX_MIXED ? mixed::launch_step(a, s) : fp64::launch_step(a, s);
}

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {nullptr};

// Device address of the current GPU's scratch array, looked up once per
// device (with that device current); nullptr on a HIP error.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

// The single-box step on a validated box and workspace (shared by
// nyx_hydro_step and nyx_hydro_step_noalloc).
int step_one_box(const nyx_params* p, const nyx_box* box, const double* state_in,
                 const void* grav, double dt, double a_old, double a_new, double* state_out,
                 double* dt_next, nyx_stats* stats, void* workspace, hipStream_t s,
                 bool timed) {
  StepArgs A{};
  box_layout(*box, 0, 0, &A.single);
  set_blocks(A.single, A.nblocks);
  fill_physics(A, p);
  A.Uin = state_in;
  A.Uout = state_out;
  A.grav = grav;
  A.work = (char*)workspace + kHeaderBytes;
  A.smax = (unsigned long long*)workspace;
  A.dt_host = dt;
  A.a_old = a_old;
  A.a_new = a_new;
  A.stats = stats;
  A.slots = (unsigned long long*)((char*)workspace + kOffSlots);
  A.dt_next = dt_next;
  BoxDev* tab = (BoxDev*)((char*)workspace + kOffTable);
  int* pre = (int*)((char*)workspace + kOffPrefix);
  StepC* cst = (StepC*)((char*)workspace + kOffConsts);
  if (launch_prologue(A, 1, cst, tab, pre, s) != hipSuccess) return NYX_E_HIP;
  A.table = tab;
  A.nb = 1;
  for (int k = 0; k < kSpaces; ++k) A.prefix[k] = pre + 2 * k;
  A.consts = cst;
  // the running CFL maximum and the partial counters start from zero (fill
  // kernels, so that a captured graph holds no memset node)
  if (dt_next && launch_zero_u64(A.smax, 1, s) != hipSuccess) return NYX_E_HIP;
  if (stats && launch_zero_u64(A.slots, kStatSlots * kStatFields, s) != hipSuccess) return NYX_E_HIP;
  if (run_stages(p, A, s, timed) != hipSuccess) return NYX_E_HIP;
  if (stats && launch_stats_reduce(A.slots, stats, s) != hipSuccess) return NYX_E_HIP;
  if (dt_next && launch_dt_finalize(A, a_new, p->cfl, dt_next, s) != hipSuccess) return NYX_E_HIP;
  return NYX_OK;
}

}  // namespace

// shape check of one box, shared with the level-fill planner (nyx_fill.hip)
int nyx::validate_box(const nyx_box* b) { return check_box(b); }

extern "C" {

void nyx_default_params(nyx_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->gamma = 5.0 / 3.0;
  p->eta_dual = 1e-4;
  p->small_dens = 1e-20;
  p->small_pres = 1e-20;
  p->riemann_tol = 1e-14;
  p->mlp_resid_tol = 1e-3;
  p->cfl = 0.5;
  p->riemann_maxiter = 20;
  p->precision = NYX_FP64;
  p->riemann = NYX_RIEMANN_TWOSHOCK;
  p->learned_stages_mask = 0;
  p->recon = NYX_RECON_PPM;
  p->grav_energy_form = 1;
  p->mlp_weights = nullptr;
  p->mixed_riemann_stop = 0.0;
}

const char* nyx_status_string(int s) {
  switch (s) {
    case NYX_OK: return "ok";
    case NYX_E_NULL: return "a required pointer is NULL";
    case NYX_E_SHAPE: return "invalid box extents, ghost width or strides";
    case NYX_E_PARAM: return "parameter out of range";
    case NYX_E_ALIAS: return "input and output state overlap";
    case NYX_E_HIP: return "HIP runtime or launch error";
    case NYX_E_UNSUPPORTED: return "combination not supported by this library";
    case NYX_E_WORKSPACE: return "workspace too small or misaligned";
    case NYX_E_SCRATCH:
      return "box needs more scratch than the allocation-free entry point holds";
    default: return "unknown status";
  }
}

int nyx_workspace_bytes(const nyx_params* p, const nyx_box* box, size_t* bytes) {
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_box(box))) return rc;
  if (!bytes) return NYX_E_NULL;
  long long elems = box_layout(*box, 0, 0, nullptr);
  *bytes = kHeaderBytes + (size_t)elems * real_bytes(p);
  return NYX_OK;
}

int nyx_estimate_dt(const nyx_params* p, const nyx_box* box, const double* state, double a,
                    double cfl, double* dt_out, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_box(box))) return rc;
  if (!state || !dt_out || !workspace) return NYX_E_NULL;
  if (!finite_pos(a) || !finite_pos(cfl)) return NYX_E_PARAM;
  if (ws_bytes < 16 || ((uintptr_t)workspace & 255)) return NYX_E_WORKSPACE;
  StepArgs A{};
  box_layout(*box, 0, 0, &A.single);
  set_blocks(A.single, A.nblocks);
  fill_physics(A, p);
  A.Uin = state;
  A.smax = (unsigned long long*)workspace;
  hipStream_t s = (hipStream_t)stream;
  if (launch_zero_u64(A.smax, 1, s) != hipSuccess) return NYX_E_HIP;
  if (launch_dtmax(A, a, s) != hipSuccess) return NYX_E_HIP;
  if (launch_dt_finalize(A, a, cfl, dt_out, s) != hipSuccess) return NYX_E_HIP;
  return NYX_OK;
}

int nyx_hydro_step(const nyx_params* p, const nyx_box* box, const double* state_in,
                   const void* grav, double dt, double a_old, double a_new, double* state_out,
                   double* dt_next, nyx_stats* stats, void* workspace, size_t ws_bytes,
                   void* stream) {
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_box(box))) return rc;
  if (!state_in || !grav || !state_out || !workspace) return NYX_E_NULL;
  if (!finite_pos(dt) || !finite_pos(a_old) || !finite_pos(a_new)) return NYX_E_PARAM;
  size_t span = state_span_bytes(*box);
  if (overlaps(state_in, span, state_out, span)) return NYX_E_ALIAS;
  size_t need = 0;
  nyx_workspace_bytes(p, box, &need);
  if (ws_bytes < need || ((uintptr_t)workspace & 255)) return NYX_E_WORKSPACE;
  return step_one_box(p, box, state_in, grav, dt, a_old, a_new, state_out, dt_next, stats,
                      workspace, (hipStream_t)stream, true);
}

int nyx_noalloc_max_bytes(size_t* bytes) {
  if (!bytes) return NYX_E_NULL;
  *bytes = kScratchBytes;
  return NYX_OK;
}

int nyx_hydro_step_noalloc(const nyx_params* p, const nyx_box* box, const double* state_in,
                           const void* grav, double dt, double a_old, double a_new,
                           double* state_out, double* dt_next, nyx_stats* stats, void* stream) {
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_box(box))) return rc;
  if (!state_in || !grav || !state_out) return NYX_E_NULL;
  if (!finite_pos(dt) || !finite_pos(a_old) || !finite_pos(a_new)) return NYX_E_PARAM;
  size_t span = state_span_bytes(*box);
  if (overlaps(state_in, span, state_out, span)) return NYX_E_ALIAS;
  size_t need = 0;
  nyx_workspace_bytes(p, box, &need);
  if (need > kScratchBytes) return NYX_E_SCRATCH;
  void* ws = scratch_address();
  if (!ws) return NYX_E_HIP;
  // no stage timing here: the profiler creates events on demand
  return step_one_box(p, box, state_in, grav, dt, a_old, a_new, state_out, dt_next, stats, ws,
                      (hipStream_t)stream, false);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched plans
// ---------------------------------------------------------------------------
struct nyx_batch {
  nyx_params prm;
  int nbox;
  std::vector<nyx_box> boxes;
  struct Group {
    int b0, b1;
    int nblocks[kSpaces];
    const int* prefix[kSpaces];  // device
  };
  std::vector<Group> groups;
  BoxDev* table;                 // device, nbox entries in box order
  unsigned long long* smax;      // device, nbox entries
  unsigned long long* slots;     // device, partial counters
  StepC* consts;                 // device, per-box step constants
  void* stage;                   // device stage region
  size_t state_span;             // bytes spanned by the state of all boxes
  // training-record harvest (final-stage faces)
  float* harvest = nullptr;
  unsigned long long* harvest_count = nullptr;
  long long harvest_cap = 0;
  unsigned harvest_keep = 0;
  unsigned long long harvest_seed = 0;
  int tune[kStages] = {0};        // launch-order candidate per stage
  // flux register fed after every group's update (two-level sync)
  const FluxRec* reg_recs = nullptr;  // device, sorted by box
  std::vector<long long> reg_prefix;  // per box, host
  double* reg = nullptr;
  long long reg_slots = 0;
  // persistent launch mode: control block (device) and barrier time limit
  unsigned long long* ctl = nullptr;
  unsigned long long barrier_ticks = 0;
  int mode = NYX_LAUNCH_STAGED;
  // ghost source of stage 1 (StepArgs::gsrc) and the tiling grid
  int gsrc = 0;
  int gg[3] = {1, 1, 1};
};

namespace {

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// bytes of the table region for a plan with `ngroups` groups
size_t table_bytes(int nbox, int ngroups) {
  return round256(sizeof(BoxDev) * (size_t)nbox) +
         round256(sizeof(int) * kSpaces * (size_t)(nbox + ngroups)) +
         round256(sizeof(unsigned long long) * (size_t)nbox) + round256(kSlotBytes) +
         round256(sizeof(StepC) * (size_t)nbox) + round256(sizeof(unsigned long long) * kCtlWords);
}

int check_boxes(const nyx_params* p, int nbox, const nyx_box* boxes) {
  int rc = check_params(p);
  if (rc) return rc;
  if (nbox < 1 || nbox > (1 << 24)) return NYX_E_SHAPE;
  if (!boxes) return NYX_E_NULL;
  for (int i = 0; i < nbox; ++i)
    if ((rc = check_box(&boxes[i]))) return rc;
  return NYX_OK;
}

}  // namespace

extern "C" {

int nyx_batch_workspace_bytes(const nyx_params* p, int nbox, const nyx_box* boxes,
                              size_t* min_bytes, size_t* single_group_bytes) {
  int rc = check_boxes(p, nbox, boxes);
  if (rc) return rc;
  if (!min_bytes || !single_group_bytes) return NYX_E_NULL;
  long long maxe = 0, tot = 0;
  for (int i = 0; i < nbox; ++i) {
    long long e = box_layout(boxes[i], i, 0, nullptr);
    maxe = e > maxe ? e : maxe;
    tot += e;
  }
  *min_bytes = table_bytes(nbox, nbox) + (size_t)maxe * real_bytes(p);
  *single_group_bytes = table_bytes(nbox, nbox) + (size_t)tot * real_bytes(p);
  return NYX_OK;
}

int nyx_batch_create(const nyx_params* p, int nbox, const nyx_box* boxes, void* workspace,
                     size_t ws_bytes, void* stream, nyx_batch** out) {
  int rc = check_boxes(p, nbox, boxes);
  if (rc) return rc;
  if (!workspace || !out) return NYX_E_NULL;
  if ((uintptr_t)workspace & 255) return NYX_E_WORKSPACE;
  const size_t rb = real_bytes(p);
  // Pack boxes greedily into groups.  The group count is not known before
  // packing, so the table region is sized for the worst case (one group per
  // box) -- a few bytes per box.
  const size_t tbytes = table_bytes(nbox, nbox);
  if (ws_bytes <= tbytes) return NYX_E_WORKSPACE;
  const long long cap = (long long)((ws_bytes - tbytes) / rb);
  nyx_batch* plan = new (std::nothrow) nyx_batch();
  if (!plan) return NYX_E_WORKSPACE;
  plan->prm = *p;
  plan->nbox = nbox;
  plan->boxes.assign(boxes, boxes + nbox);
  std::vector<BoxDev> host(nbox);
  std::vector<int> prefix;
  long long used = 0;
  int g0 = 0;
  size_t span = 0;
  for (int i = 0; i <= nbox; ++i) {
    long long need = 0;
    if (i < nbox) {
      need = box_layout(boxes[i], i, 0, nullptr);
      if (need > cap) { delete plan; return NYX_E_WORKSPACE; }
      size_t sp = state_span_bytes(boxes[i]);
      span = sp > span ? sp : span;
    }
    if (i == nbox || used + need > cap) {
      // close group [g0, i)
      nyx_batch::Group g{};
      g.b0 = g0;
      g.b1 = i;
      for (int s = 0; s < kSpaces; ++s) {
        g.prefix[s] = (const int*)(size_t)prefix.size();  // host offset for now
        int acc = 0;
        for (int b = g0; b < i; ++b) {
          prefix.push_back(acc);
          if (s == kSpaceT) {
            acc += host[b].ntiles;
            continue;
          }
          if (s == kSpaceF) {
            acc += host[b].fbx;
            continue;
          }
          long long cnt = s == kSpaceP ? host[b].P : (s == kSpaceE ? host[b].E : host[b].V);
          acc += (int)blocks_for(cnt);
        }
        prefix.push_back(acc);
        g.nblocks[s] = acc;
      }
      if (i > g0) plan->groups.push_back(g);
      g0 = i;
      used = 0;
      if (i == nbox) break;
    }
    used = box_layout(boxes[i], i, used, &host[i]);
  }
  char* w = (char*)workspace;
  plan->table = (BoxDev*)w;
  int* pre_dev = (int*)(w + round256(sizeof(BoxDev) * (size_t)nbox));
  plan->smax = (unsigned long long*)((char*)pre_dev +
                                     round256(sizeof(int) * kSpaces * (size_t)(nbox + nbox)));
  plan->slots = (unsigned long long*)((char*)plan->smax + round256(sizeof(unsigned long long) * (size_t)nbox));
  plan->consts = (StepC*)((char*)plan->slots + round256(kSlotBytes));
  plan->ctl = (unsigned long long*)((char*)plan->consts + round256(sizeof(StepC) * (size_t)nbox));
  plan->stage = w + tbytes;
  {
    // the persistent step's grid barrier gives up after 5 s of wall clock
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      plan->barrier_ticks = (unsigned long long)khz * 5000ull;
    else
      plan->barrier_ticks = 500000000ull;  // 5 s at 100 MHz
  }
  plan->state_span = span;
  for (auto& g : plan->groups)
    for (int s = 0; s < kSpaces; ++s) g.prefix[s] = pre_dev + (size_t)g.prefix[s];
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(plan->table, host.data(), sizeof(BoxDev) * (size_t)nbox, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(pre_dev, prefix.data(), sizeof(int) * prefix.size(), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      launch_zero_u64(plan->ctl, kCtlWords, st) != hipSuccess ||  // no abort before any launch
      hipStreamSynchronize(st) != hipSuccess) {
    delete plan;
    return NYX_E_HIP;
  }
  *out = plan;
  return NYX_OK;
}

int nyx_batch_destroy(nyx_batch* plan) {
  delete plan;
  return NYX_OK;
}

int nyx_batch_num_groups(const nyx_batch* plan) { return plan ? (int)plan->groups.size() : 0; }

}  // extern "C"

namespace {

StepArgs group_args(const nyx_batch* plan, const nyx_batch::Group& g) {
  StepArgs A{};
  A.table = plan->table + g.b0;
  for (int s = 0; s < kSpaces; ++s) {
    A.prefix[s] = g.prefix[s];
    A.nblocks[s] = g.nblocks[s];
  }
  A.nb = g.b1 - g.b0;
  A.work = plan->stage;
  A.smax = plan->smax;
  A.slots = plan->slots;
  A.consts = plan->consts;
  fill_physics(A, &plan->prm);
  A.harvest = plan->harvest;
  A.harvest_count = plan->harvest_count;
  A.harvest_cap = plan->harvest_cap;
  A.harvest_keep = plan->harvest_keep;
  A.harvest_seed = plan->harvest_seed;
  for (int i = 0; i < kStages; ++i) A.tune[i] = plan->tune[i];
  A.ctl = plan->ctl;
  A.barrier_ticks = plan->barrier_ticks;
  A.gsrc = plan->gsrc;
  for (int d = 0; d < 3; ++d) A.gg[d] = plan->gg[d];
  A.gfull = plan->table;
  return A;
}

StepArgs all_boxes_args(const nyx_batch* plan) {
  StepArgs A{};
  A.table = plan->table;
  A.nb = plan->nbox;
  A.smax = plan->smax;
  fill_physics(A, &plan->prm);
  return A;
}

}  // namespace

extern "C" {

int nyx_batch_estimate_dt(nyx_batch* plan, const double* state, double a, double cfl, double* dt,
                          void* stream) {
  if (!plan || !state || !dt) return NYX_E_NULL;
  if (!finite_pos(a) || !finite_pos(cfl)) return NYX_E_PARAM;
  hipStream_t s = (hipStream_t)stream;
  if (launch_zero_u64(plan->smax, plan->nbox, s) != hipSuccess) return NYX_E_HIP;
  for (const auto& g : plan->groups) {
    StepArgs A = group_args(plan, g);
    A.Uin = state;
    if (launch_dtmax(A, a, s) != hipSuccess) return NYX_E_HIP;
  }
  if (launch_dt_finalize(all_boxes_args(plan), a, cfl, dt, s) != hipSuccess) return NYX_E_HIP;
  return NYX_OK;
}

int nyx_batch_min_dt(nyx_batch* plan, double* dt, void* stream) {
  if (!plan || !dt) return NYX_E_NULL;
  return launch_min_dt(dt, plan->nbox, (hipStream_t)stream) == hipSuccess ? NYX_OK : NYX_E_HIP;
}

}  // extern "C"

namespace {

// Enqueue one batched step.  group_ev: per group, kStages + 1 events to
// record around its stages (autotuning), or nullptr for the profiler's.
int enqueue_batched(nyx_batch* plan, const double* state_in, const void* grav, const double* dt,
                    double a_old, double a_new, double* state_out, double* dt_next,
                    nyx_stats* stats, hipStream_t s, hipEvent_t* const* group_ev,
                    bool record = true) {
  if (dt_next && launch_zero_u64(plan->smax, plan->nbox, s) != hipSuccess) return NYX_E_HIP;
  if (stats && launch_zero_u64(plan->slots, kStatSlots * kStatFields, s) != hipSuccess)
    return NYX_E_HIP;
  {
    StepArgs P = all_boxes_args(plan);
    P.dt_dev = dt;
    P.a_old = a_old;
    P.a_new = a_new;
    if (launch_prologue(P, plan->nbox, plan->consts, nullptr, nullptr, s) != hipSuccess)
      return NYX_E_HIP;
  }
  for (const auto& g : plan->groups) {
    StepArgs A = group_args(plan, g);
    A.Uin = state_in;
    A.Uout = state_out;
    A.grav = grav;
    A.dt_dev = dt;
    A.a_old = a_old;
    A.a_new = a_new;
    A.stats = stats;
    A.dt_next = dt_next;
    // the fused kernels where the plan allows them (flux registers read the
    // final face states the fused final stage does not store; the fused
    // front stores everything the staged kernels do); the launch-order sweep
    // times the staged kernels
    A.fuse_final = plan->mode == NYX_LAUNCH_FUSED && !plan->reg && !group_ev ? 1 : 0;
    A.fuse_front = plan->mode == NYX_LAUNCH_FUSED && !group_ev ? 1 : 0;
    hipError_t e;
    if (group_ev) {
      A.ev = group_ev[&g - plan->groups.data()];
      e = plan->prm.precision == NYX_MIXED ? mixed::launch_step(A, s) : fp64::launch_step(A, s);
    } else if (plan->mode == NYX_LAUNCH_PERSISTENT && !plan->harvest) {
      e = plan->prm.precision == NYX_MIXED ? mixed::launch_step_persistent(A, s)
                                           : fp64::launch_step_persistent(A, s);
    } else {
      e = run_stages(&plan->prm, A, s);
    }
    if (e != hipSuccess) return NYX_E_HIP;
    if (record && plan->reg) {
      // the group's final-stage states are in the stage region until the
      // next group runs
      const long long r0 = plan->reg_prefix[g.b0], r1 = plan->reg_prefix[g.b1];
      e = plan->prm.precision == NYX_MIXED
              ? mixed::launch_flux_record(A, plan->table, plan->reg_recs + r0, r1 - r0, plan->reg,
                                          plan->reg_slots, s)
              : fp64::launch_flux_record(A, plan->table, plan->reg_recs + r0, r1 - r0, plan->reg,
                                         plan->reg_slots, s);
      if (e != hipSuccess) return NYX_E_HIP;
    }
  }
  if (stats && launch_stats_reduce(plan->slots, stats, s) != hipSuccess) return NYX_E_HIP;
  if (dt_next &&
      launch_dt_finalize(all_boxes_args(plan), a_new, plan->prm.cfl, dt_next, s) != hipSuccess)
    return NYX_E_HIP;
  return NYX_OK;
}

int check_step_args(nyx_batch* plan, const double* state_in, const void* grav, const double* dt,
                    double a_old, double a_new, double* state_out) {
  if (!plan || !state_in || !grav || !dt || !state_out) return NYX_E_NULL;
  if (!finite_pos(a_old) || !finite_pos(a_new)) return NYX_E_PARAM;
  if (overlaps(state_in, plan->state_span, state_out, plan->state_span)) return NYX_E_ALIAS;
  return NYX_OK;
}

}  // namespace

extern "C" {

int nyx_hydro_step_batched(nyx_batch* plan, const double* state_in, const void* grav,
                           const double* dt, double a_old, double a_new, double* state_out,
                           double* dt_next, nyx_stats* stats, void* stream) {
  int rc = check_step_args(plan, state_in, grav, dt, a_old, a_new, state_out);
  if (rc) return rc;
  return enqueue_batched(plan, state_in, grav, dt, a_old, a_new, state_out, dt_next, stats,
                         (hipStream_t)stream, nullptr);
}

int nyx_batch_set_tuning(nyx_batch* plan, const int* tune) {
  if (!plan || !tune) return NYX_E_NULL;
  for (int i = 0; i < kStages; ++i)
    if (tune[i] < 0 || tune[i] >= kTuneCandidates) return NYX_E_PARAM;
  for (int i = 0; i < kStages; ++i) plan->tune[i] = tune[i];
  return NYX_OK;
}

int nyx_batch_get_tuning(const nyx_batch* plan, int* tune) {
  if (!plan || !tune) return NYX_E_NULL;
  for (int i = 0; i < kStages; ++i) tune[i] = plan->tune[i];
  return NYX_OK;
}

int nyx_batch_set_launch_mode(nyx_batch* plan, int mode) {
  if (!plan) return NYX_E_NULL;
  if (mode != NYX_LAUNCH_STAGED && mode != NYX_LAUNCH_PERSISTENT && mode != NYX_LAUNCH_FUSED)
    return NYX_E_PARAM;
  if (mode == NYX_LAUNCH_PERSISTENT) {
    if (plan->groups.empty()) return NYX_E_UNSUPPORTED;
    StepArgs A = group_args(plan, plan->groups[0]);
    const int grid = plan->prm.precision == NYX_MIXED ? mixed::persistent_grid(A)
                                                      : fp64::persistent_grid(A);
    if (grid <= 0) return NYX_E_UNSUPPORTED;
  }
  plan->mode = mode;
  return NYX_OK;
}

int nyx_batch_get_launch_mode(const nyx_batch* plan, int* mode) {
  if (!plan || !mode) return NYX_E_NULL;
  *mode = plan->mode;
  return NYX_OK;
}

int nyx_batch_persistent_aborted(nyx_batch* plan, int* aborted, void* stream) {
  if (!plan || !aborted) return NYX_E_NULL;
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&v, plan->ctl + kCtlAbort, sizeof v, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return NYX_E_HIP;
  *aborted = v ? 1 : 0;
  return NYX_OK;
}

int nyx_batch_autotune(nyx_batch* plan, const double* state_in, const void* grav,
                       const double* dt, double a_old, double a_new, double* state_out,
                       double* dt_next, int reps, float* ms_out, int* tune_out, void* stream) {
  int rc = check_step_args(plan, state_in, grav, dt, a_old, a_new, state_out);
  if (rc) return rc;
  if (reps < 1 || reps > 1000) return NYX_E_PARAM;
  hipStream_t s = (hipStream_t)stream;
  const size_t ng = plan->groups.size();
  std::vector<hipEvent_t> evs(ng * (kStages + 1));
  std::vector<hipEvent_t*> gev(ng);
  size_t made = 0;
  rc = NYX_OK;
  for (; made < evs.size(); ++made)
    if (hipEventCreate(&evs[made]) != hipSuccess) {
      rc = NYX_E_HIP;
      break;
    }
  for (size_t g = 0; g < ng; ++g) gev[g] = evs.data() + g * (kStages + 1);
  const std::vector<int> saved(plan->tune, plan->tune + kStages);
  double best_ms[kTuneCandidates][kStages];
  for (auto& row : best_ms)
    for (double& v : row) v = 1e30;
  // every candidate is applied to all stages at once; each stage's time is
  // read from the events around its launches, so one pass per candidate
  // times all stages; a stage keeps its fastest repetition (least disturbed
  // by other work on the device)
  for (int c = 0; c < kTuneCandidates && rc == NYX_OK; ++c) {
    for (int i = 0; i < kStages; ++i) plan->tune[i] = c;
    for (int r = 0; r <= reps && rc == NYX_OK; ++r) {  // r = 0 warms up
      rc = enqueue_batched(plan, state_in, grav, dt, a_old, a_new, state_out, dt_next, nullptr, s,
                           gev.data(), false);
      if (rc == NYX_OK && hipStreamSynchronize(s) != hipSuccess) rc = NYX_E_HIP;
      double step_ms[kStages] = {};
      for (size_t g = 0; g < ng && rc == NYX_OK && r > 0; ++g)
        for (int i = 0; i < kStages; ++i) {
          float t = 0.f;
          if (hipEventElapsedTime(&t, gev[g][i], gev[g][i + 1]) != hipSuccess) {
            rc = NYX_E_HIP;
            break;
          }
          step_ms[i] += t;
        }
      if (r > 0)
        for (int i = 0; i < kStages; ++i) best_ms[c][i] = std::min(best_ms[c][i], step_ms[i]);
    }
  }
  for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(evs[i]);
  if (rc != NYX_OK) {
    for (int i = 0; i < kStages; ++i) plan->tune[i] = saved[i];
    return rc;
  }
  for (int i = 0; i < kStages; ++i) {
    int best = 0;
    for (int c = 1; c < kTuneCandidates; ++c)
      if (best_ms[c][i] < best_ms[best][i]) best = c;
    plan->tune[i] = best;
    if (tune_out) tune_out[i] = best;
    if (ms_out)
      for (int c = 0; c < kTuneCandidates; ++c) ms_out[i * kTuneCandidates + c] = (float)best_ms[c][i];
  }
  return NYX_OK;
}

int nyx_batch_autotune_mode(nyx_batch* plan, const double* state_in, const void* grav,
                            const double* dt, double a_old, double a_new, double* state_out,
                            int reps, float* ms_out, int* mode_out, void* stream) {
  int rc = check_step_args(plan, state_in, grav, dt, a_old, a_new, state_out);
  if (rc) return rc;
  if (reps < 1 || reps > 1000) return NYX_E_PARAM;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return NYX_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return NYX_E_HIP;
  }
  const int saved = plan->mode;
  float best[3] = {-1.f, -1.f, -1.f};
  for (int mode = NYX_LAUNCH_STAGED; mode <= NYX_LAUNCH_FUSED && rc == NYX_OK; ++mode) {
    if (nyx_batch_set_launch_mode(plan, mode) != NYX_OK) continue;  // not available
    for (int r = 0; r <= reps && rc == NYX_OK; ++r) {  // r = 0 warms up
      if (hipEventRecord(e0, s) != hipSuccess) rc = NYX_E_HIP;
      if (rc == NYX_OK)
        rc = enqueue_batched(plan, state_in, grav, dt, a_old, a_new, state_out, nullptr, nullptr,
                             s, nullptr, false);
      float t = 0.f;
      if (rc == NYX_OK && (hipEventRecord(e1, s) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = NYX_E_HIP;
      if (rc == NYX_OK && r > 0 && (best[mode] < 0.f || t < best[mode])) best[mode] = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NYX_OK) {
    plan->mode = saved;
    return rc;
  }
  int keep = NYX_LAUNCH_STAGED;
  for (int mode = NYX_LAUNCH_PERSISTENT; mode <= NYX_LAUNCH_FUSED; ++mode)
    if (best[mode] >= 0.f && best[mode] < best[keep]) keep = mode;
  plan->mode = keep;
  if (ms_out)
    for (int mode = 0; mode < 3; ++mode) ms_out[mode] = best[mode];
  if (mode_out) *mode_out = plan->mode;
  return NYX_OK;
}

int nyx_fill_ghosts_periodic(const nyx_box* box, double* state, int ncomp, void* stream) {
  int rc = check_box(box);
  if (rc) return rc;
  if (!state) return NYX_E_NULL;
  if (ncomp < 1 || ncomp > 16) return NYX_E_PARAM;
  StepArgs A{};
  box_layout(*box, 0, 0, &A.single);
  set_blocks(A.single, A.nblocks);
  return launch_fill_periodic(A, nullptr, state, ncomp, 0, 1, 1, 1, (hipStream_t)stream) == hipSuccess
             ? NYX_OK
             : NYX_E_HIP;
}

int nyx_batch_set_harvest(nyx_batch* plan, float* records, unsigned long long* count,
                          long long capacity, double keep_fraction, unsigned long long seed) {
  if (!plan) return NYX_E_NULL;
  if (!records) {
    plan->harvest = nullptr;
    return NYX_OK;
  }
  if (!count) return NYX_E_NULL;
  if (capacity < 1 || !(keep_fraction > 0.0 && keep_fraction <= 1.0)) return NYX_E_PARAM;
  plan->harvest = records;
  plan->harvest_count = count;
  plan->harvest_cap = capacity;
  const double k = keep_fraction * 4294967296.0;
  plan->harvest_keep = k >= 4294967295.0 ? 4294967295u : (unsigned)k;
  plan->harvest_seed = seed;
  return NYX_OK;
}

int nyx_batch_set_flux_register(nyx_batch* plan, const nyx_sync_plan* sync, int level,
                                double* reg) {
  if (!plan) return NYX_E_NULL;
  if (!reg) {
    plan->reg = nullptr;
    plan->reg_recs = nullptr;
    plan->reg_prefix.clear();
    return NYX_OK;
  }
  if (!sync) return NYX_E_NULL;
  SyncLevelView v{};
  int rc = sync_level_view(sync, level, &v);
  if (rc) return rc;
  if (v.nbox != plan->nbox) return NYX_E_SHAPE;
  for (int b = 0; b < plan->nbox; ++b)
    for (int d = 0; d < 3; ++d)
      if (v.shapes[3 * b + d] != plan->boxes[b].n[d]) return NYX_E_SHAPE;
  plan->reg_recs = v.recs;
  plan->reg_prefix.assign(v.prefix, v.prefix + plan->nbox + 1);
  plan->reg = reg;
  plan->reg_slots = v.nslots;
  return NYX_OK;
}

int nyx_mlp_init(float* params, unsigned long long seed, void* stream) {
  if (!params) return NYX_E_NULL;
  return launch_mlp_init(params, seed, (hipStream_t)stream) == hipSuccess ? NYX_OK : NYX_E_HIP;
}

int nyx_mlp_loss_grad(const float* params, const float* records, long long n, double gamma,
                      double inv_batch, float* grad, float* loss, void* stream) {
  if (!params || !records || !grad || !loss) return NYX_E_NULL;
  if (n < 0 || n > (1ll << 40) || !(gamma > 1.0) || !finite_pos(inv_batch)) return NYX_E_PARAM;
  return launch_mlp_loss_grad(params, records, n, gamma, (float)inv_batch, grad, loss,
                              (hipStream_t)stream) == hipSuccess
             ? NYX_OK
             : NYX_E_HIP;
}

int nyx_mlp_adam(float* params, float* m, float* v, const float* grad, int t, double lr,
                 double beta1, double beta2, double eps, void* stream) {
  if (!params || !m || !v || !grad) return NYX_E_NULL;
  if (t < 1 || !finite_pos(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !finite_pos(eps))
    return NYX_E_PARAM;
  return launch_mlp_adam(params, m, v, grad, t, (float)lr, (float)beta1, (float)beta2, (float)eps,
                         (hipStream_t)stream) == hipSuccess
             ? NYX_OK
             : NYX_E_HIP;
}

int nyx_mlp_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return NYX_E_NULL;
  if ((uintptr_t)packed & 15) return NYX_E_PARAM;
  return launch_mlp_pack(params, packed, (hipStream_t)stream) == hipSuccess ? NYX_OK : NYX_E_HIP;
}

int nyx_mlp_predict(const void* packed, const float* records, long long n, double gamma,
                    float* out, void* stream) {
  if (!packed || !records || !out) return NYX_E_NULL;
  if ((uintptr_t)packed & 15) return NYX_E_PARAM;
  if (n < 0 || n > (1ll << 40) || !(gamma > 1.0)) return NYX_E_PARAM;
  return launch_mlp_predict(packed, records, n, gamma, out, (hipStream_t)stream) == hipSuccess
             ? NYX_OK
             : NYX_E_HIP;
}

int nyx_profile_enable(int on) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.on = on != 0;
  return NYX_OK;
}

int nyx_profile_read(double* ms, long long* sequences, int reset) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  for (hipEvent_t* ev : P.pending) {
    if (hipEventSynchronize(ev[kStages]) != hipSuccess) return NYX_E_HIP;
    for (int i = 0; i < kStages; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) return NYX_E_HIP;
      P.ms[i] += t;
    }
    P.seq += 1;
    P.free_.push_back(ev);
  }
  P.pending.clear();
  if (ms)
    for (int i = 0; i < kStages; ++i) ms[i] = P.ms[i];
  if (sequences) *sequences = P.seq;
  if (reset) {
    for (int i = 0; i < kStages; ++i) P.ms[i] = 0.0;
    P.seq = 0;
  }
  return NYX_OK;
}

}  // extern "C"

namespace {

// The plan's boxes tile a periodic domain as a gx x gy x gz grid of equal
// boxes, in box order, each at least ng cells across (NYX_OK or NYX_E_SHAPE).
int check_tiling(const nyx_batch* plan, int gx, int gy, int gz) {
  if (gx < 1 || gy < 1 || gz < 1 || (long long)gx * gy * gz != plan->nbox) return NYX_E_SHAPE;
  const nyx_box& b0 = plan->boxes[0];
  for (const auto& b : plan->boxes)
    if (b.n[0] != b0.n[0] || b.n[1] != b0.n[1] || b.n[2] != b0.n[2] || b.ng != b0.ng ||
        b.ng > b.n[0] || b.ng > b.n[1] || b.ng > b.n[2])
      return NYX_E_SHAPE;
  return NYX_OK;
}

}  // namespace

extern "C" {

int nyx_batch_set_ghost_source(nyx_batch* plan, int mode, int gx, int gy, int gz) {
  if (!plan) return NYX_E_NULL;
  if (mode < -1 || mode > 1) return NYX_E_PARAM;
  if (mode == 1) {
    const int rc = check_tiling(plan, gx, gy, gz);
    if (rc) return rc;
  }
  plan->gsrc = mode + 1;
  plan->gg[0] = mode == 1 ? gx : 1;
  plan->gg[1] = mode == 1 ? gy : 1;
  plan->gg[2] = mode == 1 ? gz : 1;
  return NYX_OK;
}

int nyx_batch_fill_ghosts(nyx_batch* plan, int mode, int gx, int gy, int gz, double* state,
                          void* stream) {
  if (!plan || !state) return NYX_E_NULL;
  if (mode != 0 && mode != 1) return NYX_E_PARAM;
  if (mode == 1) {
    const int rc = check_tiling(plan, gx, gy, gz);
    if (rc) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  for (const auto& g : plan->groups) {
    StepArgs A = group_args(plan, g);
    if (launch_fill_periodic(A, plan->table, state, 6, mode, gx, gy, gz, s) != hipSuccess)
      return NYX_E_HIP;
  }
  return NYX_OK;
}

}  // extern "C"
