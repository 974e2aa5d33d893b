// nyx_internal.h -- device-side box descriptors and launch arguments shared
// by the host ABI layer (nyx_abi.cpp) and the two precision builds of the
// stage kernels (nyx_step.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nyx_hydro.h"

namespace nyx {

constexpr int kBlock = 256;  // threads per block: 4 wavefronts of 64
// Threads per workgroup of the fused final-stage kernel (8 wavefronts): a
// tile of TX x TY cell columns of a box, TX = min(n_x, 64), TY = min(n_y,
// kFinBlock / TX), over a chunk of at most kFinPlanes planes in z (tall
// boxes are cut into several chunks so that the launch has enough tiles).
constexpr int kFinBlock = 512;
constexpr int kFinPlanes = 64;
// Fused front (tracing and stage-0 solves of x in one kernel): a wavefront
// holds 64 consecutive cells of the [-1, n]^3 range, the first of them the
// last of the previous wavefront, so a block owns kFrontOwn cells.
constexpr int kFrontOwn = kBlock / 64 * 63;
// Stored per face: the Godunov state (rho_g, u_g normal, v_g, w_g transverse,
// p_g) in the face's rotated frame; every flux is recomputed from it.
constexpr int kGod = 5;
// Device counters are accumulated per block into kStatSlots partial blocks
// (block index modulo kStatSlots) and summed once per step.
constexpr int kStatSlots = 64;
constexpr int kStatFields = 10;

// Division by a per-box invariant divisor d with a precomputed multiplier:
// q = (umulhi(n, m) + n) >> l, exact for every n < 2^31.
struct FastDiv {
  unsigned d, m, l;
};
inline FastDiv make_fastdiv(unsigned d) {
  unsigned l = 0;
  while ((1ull << l) < d) ++l;
  unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{d, (unsigned)m, l};
}

// One box as the kernels see it.  All offsets are element offsets.
struct BoxDev {
  int n[3];
  int ng;
  int px, py, pz;          // padded extents n + 2 ng
  int ex, ey, ez;          // extents of the cell range [-1, n]
  long long P, E, V;       // padded, [-1,n]^3 and valid cell counts
  long long soff, goff;    // state / gravity offset of padded cell 0
  long long sstride, gstride;
  long long w_prim, w_chi, w_edge, w_f0, w_f1, w_f2;  // stage arrays (elements)
  int gidx;                // index of the box in the caller's list
  int pad_;
  double dx;
  FastDiv dv[3][2];        // per Space: row length and plane size
  FastDiv dz[3];           // per Space: number of planes
  unsigned sy[3];          // per Space: rows per plane
  unsigned sc[3];          // per Space: cell count (< 2^31)
  int tx, ty, ntx, nty;    // fused final stage: tile shape, tiles along x and y,
  int ntiles, pad2_;       // tiles in all (z chunks of kFinPlanes planes included)
  int fbx, pad3_;          // fused front: blocks of kFrontOwn cells
};

// Stage-array element count for a box (before alignment padding).
inline long long align_elems(long long n) { return (n + 63) / 64 * 64; }

// Fill the derived fields and stage offsets of a box starting at `base`;
// returns the element offset just past its stage arrays.
inline long long box_layout(const nyx_box& b, int gidx, long long base, BoxDev* out) {
  BoxDev d{};
  for (int i = 0; i < 3; ++i) d.n[i] = b.n[i];
  d.ng = b.ng;
  d.px = b.n[0] + 2 * b.ng;
  d.py = b.n[1] + 2 * b.ng;
  d.pz = b.n[2] + 2 * b.ng;
  d.ex = b.n[0] + 2;
  d.ey = b.n[1] + 2;
  d.ez = b.n[2] + 2;
  d.P = (long long)d.px * d.py * d.pz;
  d.E = (long long)d.ex * d.ey * d.ez;
  d.V = (long long)b.n[0] * b.n[1] * b.n[2];
  d.soff = b.state_off;
  d.goff = b.grav_off;
  d.sstride = b.comp_stride;
  d.gstride = b.grav_stride;
  d.dx = b.dx;
  d.gidx = gidx;
  long long o = base;
  d.w_prim = o; o += align_elems(6 * d.P);
  d.w_chi = o;  o += align_elems(d.E);
  d.w_edge = o; o += align_elems(30 * d.E);
  d.w_f0 = o;   o += align_elems(3 * kGod * d.E);
  d.w_f1 = o;   o += align_elems(6 * kGod * d.E);
  d.w_f2 = o;   o += align_elems(3 * kGod * d.E);
  d.dv[0][0] = make_fastdiv((unsigned)d.px);
  d.dv[0][1] = make_fastdiv((unsigned)d.px * (unsigned)d.py);
  d.dv[1][0] = make_fastdiv((unsigned)d.ex);
  d.dv[1][1] = make_fastdiv((unsigned)d.ex * (unsigned)d.ey);
  d.dv[2][0] = make_fastdiv((unsigned)b.n[0]);
  d.dv[2][1] = make_fastdiv((unsigned)b.n[0] * (unsigned)b.n[1]);
  d.dz[0] = make_fastdiv((unsigned)d.pz);
  d.dz[1] = make_fastdiv((unsigned)d.ez);
  d.dz[2] = make_fastdiv((unsigned)b.n[2]);
  d.sy[0] = (unsigned)d.py;
  d.sy[1] = (unsigned)d.ey;
  d.sy[2] = (unsigned)b.n[1];
  d.sc[0] = (unsigned)d.P;
  d.sc[1] = (unsigned)d.E;
  d.sc[2] = (unsigned)d.V;
  d.tx = b.n[0] < 64 ? b.n[0] : 64;
  d.ty = b.n[1] < kFinBlock / d.tx ? b.n[1] : kFinBlock / d.tx;
  d.ntx = (b.n[0] + d.tx - 1) / d.tx;
  d.nty = (b.n[1] + d.ty - 1) / d.ty;
  d.ntiles = d.ntx * d.nty * ((b.n[2] + kFinPlanes - 1) / kFinPlanes);
  d.fbx = (int)((d.E + kFrontOwn - 1) / kFrontOwn);
  if (out) *out = d;
  return o;
}

// Per-box constants of a step, computed once per box by the step's prologue
// kernel (the same expressions the oracle evaluates on the host).
struct StepC {
  double dt, a_h, da, kh, hdt_a, hda_a, pexp, kap1, kap2, k, gm1;
  double xo, xn;  // expansion source of the energy equations at a_old / a_new
  double pad_;
};

// Which cell range a launch walks: padded cells, the [-1, n]^3 range, valid
// cells, the column tiles of the fused final stage (counted in tiles, not in
// blocks of cells; no cell coordinates of their own), and the fused front's
// blocks of kFrontOwn cells of the [-1, n]^3 range.
enum Space { kSpaceP = 0, kSpaceE = 1, kSpaceV = 2, kSpaceT = 3, kSpaceF = 4 };
constexpr int kSpaces = 5;

#ifdef __HIPCC__
// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Renumber them so that every XCD walks one contiguous
// range of the (linearised) grid: neighbouring rows and planes of a stage
// array are then read through the same L2.  A bijection for any grid size.
// With remap = false the hardware order is kept (the autotuner's other
// candidate).
__device__ __forceinline__ unsigned xcd_linear_block(bool remap = true) {
  const unsigned n = gridDim.x * gridDim.y;
  const unsigned lin = blockIdx.x + blockIdx.y * gridDim.x;
  if (!remap) return lin;
  const unsigned q = n >> 3, r = n & 7;
  const unsigned xcd = lin & 7, pos = lin >> 3;
  return xcd < r ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
}

// Raise *dst (bits of a non-negative double) to the bits of m.  The stored
// maximum only grows, so a read that already shows a value at least as large
// (even a stale one) makes the atomic unnecessary; most blocks of a box then
// skip it instead of queueing on one address.
__device__ __forceinline__ void max_bits(unsigned long long* dst, double m) {
  const unsigned long long v = (unsigned long long)__double_as_longlong(m);
  if (__hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(dst, v);
}

__device__ __forceinline__ unsigned fast_div(unsigned n, const FastDiv& f) {
  return (__umulhi(n, f.m) + n) >> f.l;
}
// Element i of an array through a 32-bit byte offset.  Every per-box array
// has fewer than 2^29 elements (checked on the host), so the byte offset fits
// 32 bits.  With a base that is uniform over the workgroup the compiler can
// use the scalar-base form of the memory instructions where the offset and
// the access sit in one block; elsewhere the access costs one 64-bit add.
template <class T>
__device__ __forceinline__ T ldu(const T* base, unsigned i) {
  return *(const T*)((const char*)base + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stu(T* base, unsigned i, T v) {
  *(T*)((char*)base + i * (unsigned)sizeof(T)) = v;
}

// Natural (x fastest, then y, then z) flat index of the cell at position q
// of a slab walk with 2^lg rows per slab (kTuneSlabShift); q >= the cell
// count is returned unchanged (lanes past the end of the box).
__device__ __forceinline__ unsigned slab_to_natural(const BoxDev& b, int space, unsigned q,
                                                    int lg) {
  if (q >= b.sc[space]) return q;
  const FastDiv& r = b.dv[space][0];
  const FastDiv& zd = b.dz[space];
  const unsigned ex = r.d, ey = b.sy[space], ez = zd.d;
  const unsigned t = fast_div(q, r);  // (slab, z, row) index
  const unsigned x = q - t * ex;
  const unsigned nfull = ey >> lg;    // whole slabs
  const unsigned tfull = (nfull << lg) * ez;
  unsigned y, z;
  if (t < tfull) {
    const unsigned yin = t & ((1u << lg) - 1u);
    const unsigned u = t >> lg;
    const unsigned sl = fast_div(u, zd);
    z = u - sl * ez;
    y = (sl << lg) + yin;
  } else {
    const unsigned t2 = t - tfull;
    const unsigned yin = fast_div(t2, zd);
    z = t2 - yin * ez;
    y = (nfull << lg) + yin;
  }
  return x + ex * (y + ey * z);
}

// (x, y, z) of flat index idx < 2^31 in the given Space of a box
__device__ __forceinline__ void space_coords(const BoxDev& b, int space, unsigned idx, int* c) {
  const FastDiv& r = b.dv[space][0];
  const FastDiv& pl = b.dv[space][1];
  unsigned q1 = fast_div(idx, r);
  unsigned q2 = fast_div(idx, pl);
  c[0] = (int)(idx - q1 * r.d);
  c[1] = (int)(q1 - q2 * b.sy[space]);
  c[2] = (int)q2;
}
#endif

// Stage kernels of a step, in launch order (also the order of the timing
// events and of the tuning entries).
constexpr int kStages = 7;
enum Stage { kStPrim = 0, kStFlat, kStTrace, kStRiem0, kStRiem1, kStRiem2, kStUpdate };
// Launch-order candidates of a stage (fields of a tuning entry):
//  bit 0 (kTuneCellMajor)  grids with one row per direction (or direction
//                  pair) walk the rows of one cell range back to back, so the
//                  stage arrays the directions share are reread from the same
//                  L2; otherwise one direction after the other;
//  bit 1 (kTuneHwOrder)    hardware workgroup order instead of the
//                  XCD-contiguous numbering;
//  bits 2-3 (kTuneSlabShift) cell order within a box: 0 plane by plane (x,
//                  then y, then z); s = 1, 2, 3: slabs of 2^(s+2) rows, each
//                  walked plane by plane along z (a z-pencil of row tiles), so
//                  a cell's z-neighbours are read shortly after it through
//                  the same L2; rows left over below a whole slab are walked
//                  one row at a time along z.
constexpr int kTuneCellMajor = 1;
constexpr int kTuneHwOrder = 2;
constexpr int kTuneSlabShift = 2;
constexpr int kTuneCandidates = 16;

// Control block of the persistent step (device, zeroed before each launch):
// per stage the heads of 8 work queues (one per eighth of the part of the
// stage's walk that is not handed out statically, drained first by the
// workgroups of one XCD); per stage boundary the arrival counts of the 8 XCD
// groups of workgroups and the count of XCD groups complete; the abort flag
// a barrier that timed out raises.
constexpr int kCtlXcdBar = kStages * 8;
constexpr int kCtlBarrier = kCtlXcdBar + kStages * 8;
constexpr int kCtlAbort = kCtlBarrier + kStages;
constexpr int kCtlWords = kCtlAbort + 1;

// Launch-wide arguments of a step.
struct StepArgs {
  // box selection: a device table + block prefix per Space (the single-box
  // entry points write a one-entry table in their prologue)
  BoxDev single;
  const BoxDev* table;     // device, nb entries (batched) or nullptr
  const int* prefix[kSpaces];  // device, nb+1 block prefixes per Space (batched)
  int nb;
  int nblocks[kSpaces];    // grid size per Space
  // physics
  const double* Uin;
  double* Uout;
  const void* grav;
  void* work;              // stage region base (real elements)
  unsigned long long* smax;  // per-box running max of |u|+c (bit pattern)
  const double* dt_dev;    // per-box dt (batched) or nullptr
  double dt_host;
  double a_old, a_new;
  double gamma, eta, small_dens, small_pres, riemann_tol, cfl;
  double igm1;   // 1 / (gamma - 1), for the mixed build's products
  float igm1f;   // the same in FP32 (the FP32 flux formulas)
  double mixed_stop;  // FP32-mixed stopping rule (see two_shock)
  int maxiter;
  nyx_stats* stats;
  unsigned long long* slots;  // kStatSlots x kStatFields partial counters (when stats)
  double* dt_next;
  hipEvent_t* ev;          // kStages + 1 events recorded around the stages, or nullptr
  const StepC* consts;     // per-box step constants, indexed by gidx
  // learned Riemann flux (FP32-mixed build only)
  const void* mlp;         // packed network, or nullptr
  int learned_mask;        // bit s: stage s (0, 1, 2) uses the network
  double mlp_tol;          // accepted two-shock residual
  // harvest of final-stage faces for training
  float* harvest;          // [cap][15] records, or nullptr
  unsigned long long* harvest_count;
  long long harvest_cap;
  unsigned harvest_keep;   // keep a face when its 32-bit hash < harvest_keep
  unsigned long long harvest_seed;
  int tune[kStages];       // launch-order candidate per stage (kTune* bits)
  // scheme variants (Sec. 3.2)
  int recon;               // NYX_RECON_PPM or NYX_RECON_PLM
  int grav_form;           // energy gravity term, 1 or 2
  int linear_riemann;      // 1: linearised solver instead of the two-shock one
  int expansion;           // 1: gamma != 5/3, apply the a adot (2 - 3(gamma-1)) rho e term
  // persistent step: control block (kCtlWords, zeroed before the launch)
  // and the grid barrier's time limit in wall-clock ticks
  unsigned long long* ctl;
  unsigned long long barrier_ticks;
  // 1: stages riem2 and update run fused (k_final) where the step allows it
  int fuse_final;
  // 1: stages trace and riem0 of x run fused (k_front) where the step
  // allows it; their launches then take y and z only
  int fuse_front;
  // direction of row 0 of the trace and riem0 launches (1 when k_front has
  // taken x)
  int dir0;
  // where stage 1 reads a ghost cell of the input state: 0 the input's own
  // ghost cell; 1 its periodic image in the same box; 2 its source cell in
  // the neighbouring box of boxes that tile a periodic domain as a
  // gg[0] x gg[1] x gg[2] grid (gfull: every box of the plan in box order)
  int gsrc;
  int gg[3];
  const BoxDev* gfull;
};


// Shape check of one box (NYX_OK or a negative nyx_status).
int validate_box(const nyx_box* b);

// One face of a flux register fed by a batched step (Sec. 4.3 reflux): the
// final flux of face f (box-local; f[d] in [0, n_d] along the normal d, a
// valid cell index across it) of box `box` is added, times scale * dt, to
// register slot `slot`.  nsub = 2 sums the 2 x 2 faces f, f + e_t1,
// f + e_t2, f + e_t1 + e_t2 (t1 < t2 the transverse axes) in that order.
struct FluxRec {
  int box, d, nsub, pad_;
  int f[3], pad2_;
  double scale;
  long long slot;
};

// The records of one level of a two-level sync plan (nyx_sync.hip), sorted
// by box, with the per-box prefix (host, nbox + 1 entries) and box shapes
// (host, 3 ints per box) for matching a batch plan.
struct SyncLevelView {
  const FluxRec* recs;
  const long long* prefix;
  const int* shapes;
  int nbox;
  long long nslots;
};

// The two precision builds of the stage kernels.
// launch_step_persistent: the seven stages of a group as one launch of
// co-resident workgroups (NYX_E_UNSUPPORTED-worthy cases return
// hipErrorNotSupported: harvesting, or a learned-stage mask other than 0 or
// 7); persistent_grid: the workgroups it launches on the current device.
namespace fp64 {
hipError_t launch_step(const StepArgs& a, hipStream_t s);
hipError_t launch_step_persistent(const StepArgs& a, hipStream_t s);
int persistent_grid(const StepArgs& a);
hipError_t launch_flux_record(const StepArgs& a, const BoxDev* table, const FluxRec* recs,
                              long long nrec, double* reg, long long nslots, hipStream_t s);
}
namespace mixed {
hipError_t launch_step(const StepArgs& a, hipStream_t s);
hipError_t launch_step_persistent(const StepArgs& a, hipStream_t s);
int persistent_grid(const StepArgs& a);
hipError_t launch_flux_record(const StepArgs& a, const BoxDev* table, const FluxRec* recs,
                              long long nrec, double* reg, long long nslots, hipStream_t s);
}
// Precision-independent kernels (in nyx_abi.cpp's companion nyx_util.hip).
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_dtmax(const StepArgs& a, double a_state, hipStream_t s);
hipError_t launch_dt_finalize(const StepArgs& a, double a_state, double cfl, double* dt_out,
                              hipStream_t s);
hipError_t launch_min_dt(double* dt, int n, hipStream_t s);
hipError_t launch_stats_reduce(const unsigned long long* slots, nyx_stats* stats, hipStream_t s);
// Step prologue: per-box step constants of boxes [0, nbox) of `a.table` (or
// of a.single when single_dst is given, which also receives a.single and the
// one-box block prefixes).
hipError_t launch_prologue(const StepArgs& a, int nbox, StepC* consts, BoxDev* single_dst,
                           int* prefix_dst, hipStream_t s);
// learned flux (nyx_mlp.hip)
hipError_t launch_mlp_init(float* P, unsigned long long seed, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float* P, const float* rec, long long n, double gamma,
                                float inv_n, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* P, float* m, float* v, const float* g, int t, float lr, float b1,
                           float b2, float eps, hipStream_t st);
hipError_t launch_mlp_pack(const float* P, void* packed, hipStream_t st);
hipError_t launch_mlp_predict(const void* packed, const float* rec, long long n, double gamma,
                              float* out, hipStream_t st);
hipError_t launch_fill_periodic(const StepArgs& a, const BoxDev* full, double* state, int ncomp,
                                int mode, int gx, int gy, int gz, hipStream_t s);

int sync_level_view(const nyx_sync_plan* p, int level, SyncLevelView* out);

}  // namespace nyx
