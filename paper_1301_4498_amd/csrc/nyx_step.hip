// nyx_step.hip -- stage kernels of the comoving unsplit PPM Godunov gas step
// for gfx950 (Almgren et al., Nyx: Sec. 3.2 Gas Dynamics; Sec. 3.6 Steps 2
// and 6).  This file is compiled twice:
//   NYX_PREC_FP64  : every stage in FP64, no contraction (parity build);
//   NYX_PREC_MIXED : primitives, flattening, PPM, tracing and the flux
//                    formulas in FP32; the two-shock iteration, the transverse
//                    corrections with their internal-energy recovery, the
//                    conservative accumulation, the gravity corrector and the
//                    dual-energy sync in FP64.
//
// Pipeline (one launch per stage, each over every box of a group):
//   prim    padded cells       primitives rho, u, v, w, p, c
//   flat    cells [-1,n]^3     flattening coefficient chi = min_d chi_d
//   trace   cells [-1,n]^3 x 3 PPM + characteristic tracing -> edge states
//   riem0   faces x 3          Riemann on stage-0 states -> F^d
//   riem1   faces x 6          states corrected by F^t (k/3) -> F^{d|t}
//   riem2   valid faces x 3    states corrected by F^{t1|t2}, F^{t2|t1} (k/2)
//                              -> final comoving fluxes
//   update  valid cells        flux differences, S_e, S_g^n, corrector, sync,
//                              optional CFL maximum of the new state
// Stage arrays are component-major over the [-1,n]^3 cell range (x fastest),
// so every load and store of a wavefront is contiguous.  A face stores only
// its Godunov state (5 values); fluxes are recomputed from it where needed
// with the same expressions, which keeps the HBM traffic of the Riemann
// stages low without changing a single bit of the result.
#include <hip/hip_runtime.h>

#include "nyx_internal.h"
#include "nyx_mlp_dev.h"

#if defined(NYX_PREC_FP64)
#define NYX_NS fp64
typedef double real;
#elif defined(NYX_PREC_MIXED)
#define NYX_NS mixed
typedef float real;
#else
#error "define NYX_PREC_FP64 or NYX_PREC_MIXED"
#endif

namespace nyx {
namespace NYX_NS {

// CW84 flattening constants (the PPM reference cited in Sec. 3.2)
#define FLAT_EPS 0.33
#define FLAT_OMEGA1 0.75
#define FLAT_OMEGA2 10.0

template <class T>
__device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
template <class T>
__device__ __forceinline__ T vmin(T a, T b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// block -> (box, local block) mapping
// ---------------------------------------------------------------------------
struct Loc {
  const BoxDev* bd;
  unsigned idx;  // cell index within the box's space (< 2^31)
};

// Box and cell index of this thread for the workgroup at walk position
// `lin` of a stage grid of gx blocks per row and gy rows; *ylane receives the
// row (direction or direction pair).  The walk follows the stage's tuning
// entry (kTune* bits).
__device__ __forceinline__ Loc locate_at(const StepArgs& A, int stage, int space, unsigned lin,
                                         unsigned gx, unsigned gy, int* ylane) {
  Loc L;
  const int tune = A.tune[stage];
  unsigned bx, yl;
  if (tune & kTuneCellMajor) {
    bx = lin / gy;
    yl = lin % gy;
  } else {
    bx = lin % gx;
    yl = lin / gx;
  }
  if (ylane) *ylane = (int)yl;
  const int* pre = A.prefix[space];
  int lo = 0, hi = A.nb;  // find b with pre[b] <= bx < pre[b+1]
  const int x = (int)bx;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pre[mid] <= x) lo = mid;
    else hi = mid;
  }
  L.bd = A.table + lo;
  L.idx = (unsigned)(x - pre[lo]) * (unsigned)kBlock + threadIdx.x;
  const int slab = (tune >> kTuneSlabShift) & 3;
  if (slab) L.idx = slab_to_natural(*L.bd, space, L.idx, slab + 2);
  return L;
}
// Where a work item of a stage sits: the walk position and grid shape of
// the stage's own launch (position from the hardware block index,
// XCD-contiguous unless the tuning says otherwise), or of one item of the
// persistent step's queue.
struct Item {
  unsigned lin, gx, gy;
};
__device__ __forceinline__ Item launch_item(const StepArgs& A, int stage) {
  return Item{xcd_linear_block(!(A.tune[stage] & kTuneHwOrder)), gridDim.x, gridDim.y};
}
__device__ __forceinline__ Loc locate(const StepArgs& A, int stage, int space, const Item& it,
                                      int* ylane = nullptr) {
  int y = 0;
  Loc L = locate_at(A, stage, space, it.lin, it.gx, it.gy, &y);
  if (ylane) *ylane = y;
  return L;
}

// per-box constants of the step, computed once per box by the prologue
__device__ __forceinline__ const StepC& step_consts(const StepArgs& A, const BoxDev& b) {
  return A.consts[b.gidx];
}

// ---------------------------------------------------------------------------
// counters: one atomic per wavefront
// ---------------------------------------------------------------------------
enum StatField {
  kNonfinite = 0, kNegDens, kNegEint, kFloorHits, kTransReverts, kSyncEfromE,
  kRiemannIters, kRiemannCalls, kMlpUsed, kMlpFallback
};
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Block-wide sum added into one of kStatSlots partial counter blocks; every
// thread of the block (NT threads) must call it (it synchronises the block).
template <int NT = kBlock>
__device__ __forceinline__ void count(const StepArgs& A, int field, unsigned v) {
  __shared__ unsigned red[NT / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int i = 0; i < NT / 64; ++i) t += red[i];
    const unsigned slot = (blockIdx.x + blockIdx.y * gridDim.x) % kStatSlots;
    if (t) atomicAdd(A.slots + slot * kStatFields + field, (unsigned long long)t);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// stage 1: primitives on every padded cell
// ---------------------------------------------------------------------------
// Where stage 1 reads padded cell id of box b when the input's ghost cells
// are not read (StepArgs::gsrc): a valid cell is itself; a ghost cell is its
// periodic image in the box (gsrc 1) or the cell of the neighbouring box of
// the tiling grid that a same-level ghost fill would copy into it (gsrc 2).
// Returns the source box's state, component stride and cell index.
__device__ __forceinline__ void ghost_source(const StepArgs& A, const BoxDev& b, unsigned id,
                                             const double*& U, long long& ss, unsigned& sid) {
  const unsigned px = (unsigned)b.px, pxy = px * (unsigned)b.py;
  const unsigned pk = id / pxy, r = id - pk * pxy, pj = r / px;
  int c[3] = {(int)(r - pj * px) - b.ng, (int)pj - b.ng, (int)pk - b.ng};
  if ((unsigned)c[0] < (unsigned)b.n[0] && (unsigned)c[1] < (unsigned)b.n[1] &&
      (unsigned)c[2] < (unsigned)b.n[2])
    return;
  const BoxDev* sb = &b;
  if (A.gsrc == 1) {
    for (int d = 0; d < 3; ++d) c[d] = ((c[d] % b.n[d]) + b.n[d]) % b.n[d];
  } else {
    const int gx = A.gg[0], gy = A.gg[1];
    const int bq[3] = {b.gidx % gx, (b.gidx / gx) % gy, b.gidx / (gx * gy)};
    int t[3];
    for (int d = 0; d < 3; ++d) {
      const int N = A.gg[d] * b.n[d];
      const int X = ((bq[d] * b.n[d] + c[d]) % N + N) % N;
      t[d] = X / b.n[d];
      c[d] = X - t[d] * b.n[d];
    }
    sb = &A.gfull[(t[2] * gy + t[1]) * gx + t[0]];
  }
  U = A.Uin + sb->soff;
  ss = sb->sstride;
  sid = ((unsigned)(c[2] + sb->ng) * (unsigned)sb->py + (unsigned)(c[1] + sb->ng)) * (unsigned)sb->px +
        (unsigned)(c[0] + sb->ng);
}

__device__ __forceinline__ void prim_body(const StepArgs& A, const Item& it) {
  Loc L = locate(A, kStPrim, kSpaceP, it);
  const BoxDev& b = *L.bd;
  unsigned floors = 0;
  if (L.idx < b.P) {
    const unsigned id = L.idx;
    const double* U = A.Uin + b.soff;
    long long ss = b.sstride;
    unsigned sid = id;  // the cell read for padded cell id
    if (A.gsrc) ghost_source(A, b, id, U, ss, sid);
    const double ao = A.a_old;
    double rho = ldu(U, sid);
    if (rho < A.small_dens) { rho = A.small_dens; floors++; }
    double u = ldu(U + ss, sid) / (ao * rho);
    double v = ldu(U + 2 * ss, sid) / (ao * rho);
    double w = ldu(U + 3 * ss, sid) / (ao * rho);
    double re = ldu(U + 5 * ss, sid) / (ao * ao);
    double p = (A.gamma - 1.0) * re;
    if (p < A.small_pres) { p = A.small_pres; floors++; }
    double c = sqrt((A.gamma * p) / rho);
    real* q = (real*)A.work + b.w_prim;
    stu(q, id, (real)rho);
    stu(q + b.P, id, (real)u);
    stu(q + 2 * b.P, id, (real)v);
    stu(q + 3 * b.P, id, (real)w);
    stu(q + 4 * b.P, id, (real)p);
    stu(q + 5 * b.P, id, (real)c);
  }
  if (A.stats) count(A, kFloorHits, floors);
}
__global__ __launch_bounds__(kBlock) void k_prim(StepArgs A) { prim_body(A, launch_item(A, kStPrim)); }

// padded index of the cell at E-array coordinates (ie, je, ke) (cell ie - 1)
__device__ __forceinline__ unsigned pidx_e(const BoxDev& b, int ie, int je, int ke) {
  return ((unsigned)(ke - 1 + b.ng) * (unsigned)b.py + (unsigned)(je - 1 + b.ng)) * (unsigned)b.px +
         (unsigned)(ie - 1 + b.ng);
}

// ---------------------------------------------------------------------------
// stage 2: flattening (O2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ real flat_tilde(real sp, real pm2, real pm1, real pp1, real pp2,
                                           real um1, real up1) {
  real dp1 = pp1 - pm1;
  real dp2 = pp2 - pm2;
#if defined(NYX_PREC_MIXED)
  // the ratio only places the coefficient on its ramp: the hardware
  // reciprocal (1 ulp) replaces the range-scaled division; a zero
  // denominator still gives z = inf where the detector fires (dp1 != 0)
  real z = fabs(dp1) * __builtin_amdgcn_rcpf(vmax(fabs(dp2), sp));
#else
  real z = fabs(dp1) / vmax(fabs(dp2), sp);
#endif
  bool w = (fabs(dp1) > (real)FLAT_EPS * vmin(pp1, pm1)) && ((up1 - um1) < (real)0);
  return w ? vmax((real)0, vmin((real)1, (real)FLAT_OMEGA2 * (z - (real)FLAT_OMEGA1))) : (real)0;
}

__device__ __forceinline__ void flat_body(const StepArgs& A, const Item& it) {
  Loc L = locate(A, kStFlat, kSpaceE, it);
  const BoxDev& b = *L.bd;
  if (L.idx >= b.E) return;
  const unsigned e = L.idx;
  int ec[3];
  space_coords(b, kSpaceE, L.idx, ec);
  const int ie = ec[0], je = ec[1], ke = ec[2];
  const real* prim = (const real*)A.work + b.w_prim;
  const real* P = prim + 4 * b.P;
  const real sp = (real)A.small_pres;
  const unsigned c0 = pidx_e(b, ie, je, ke);
  const unsigned sd[3] = {1u, (unsigned)b.px, (unsigned)b.px * (unsigned)b.py};
  // neighbour shifts go into the (uniform) base; all loads share c0 and are
  // issued before any arithmetic, so a wave waits once for all of them
  real pd[3][7], ud[3][5];
  const real pc = ldu(P, c0);
  for (int d = 0; d < 3; ++d) {
    const unsigned s = sd[d];
    const real* U = prim + (1 + d) * b.P;
    for (int o = -3; o <= 3; ++o) pd[d][o + 3] = o == 0 ? pc : ldu(P + (long long)o * s, c0);
    for (int o = -2; o <= 2; ++o) ud[d][o + 2] = ldu(U + (long long)o * s, c0);
  }
  real cmin = (real)1;
  for (int d = 0; d < 3; ++d) {
    const real* p = pd[d];
    const real* u = ud[d];
    real f0 = flat_tilde(sp, p[1], p[2], p[4], p[5], u[1], u[3]);
    real dp1 = p[4] - p[2];
#if defined(NYX_PREC_MIXED)
    // the one neighbour the pressure jump selects (cell j-1 for dp1 > 0,
    // j+1 for dp1 < 0) evaluated once on selected inputs: the same values
    // as evaluating both, with one evaluation fewer
    const bool lo = dp1 > (real)0;
    const real fn = flat_tilde(sp, lo ? p[0] : p[2], lo ? p[1] : p[3], lo ? p[3] : p[5],
                               lo ? p[4] : p[6], lo ? u[0] : u[2], lo ? u[2] : u[4]);
    const real f = (lo || dp1 < (real)0) ? vmax(f0, fn) : f0;  // f0 alone for dp1 = 0 or NaN
#else
    real fm = flat_tilde(sp, p[0], p[1], p[3], p[4], u[0], u[2]);
    real fp = flat_tilde(sp, p[2], p[3], p[5], p[6], u[2], u[4]);
    real f = f0;
    if (dp1 > (real)0) f = vmax(f0, fm);
    else if (dp1 < (real)0) f = vmax(f0, fp);
#endif
    real cd = (real)1 - f;
    cmin = (d == 0) ? cd : vmin(cmin, cd);
  }
  stu((real*)A.work + b.w_chi, e, cmin);
}
__global__ __launch_bounds__(kBlock) void k_flat(StepArgs A) { flat_body(A, launch_item(A, kStFlat)); }

// ---------------------------------------------------------------------------
// stage 3: PPM (O3) and characteristic tracing (O4)
// ---------------------------------------------------------------------------
#if defined(NYX_PREC_MIXED)
// The limited slope without the branch: with s the sign of d2 = q(j+1) -
// q(j-1), min(|dc|, 2|dl|, 2|dr|) = 2 min(|d2|/4, s dl, s dr) when dl dr > 0
// (then dl, dr and d2 share their sign), and that minimum is <= 0 otherwise,
// so clamping it at 0 gives the limiter's zero slope.  Scaling by 2 and 1/4
// is exact, so the value is the branchy form's (up to the sign of a zero
// slope, and slopes below the FP32 normal range).
__device__ __forceinline__ real lim_slope(real qm1, real q0, real qp1) {
  const real d2 = qp1 - qm1;
  const real dr = qp1 - q0;
  const real dl = q0 - qm1;
  const unsigned sg = __float_as_uint(d2) & 0x80000000u;
  const real sdl = __uint_as_float(__float_as_uint(dl) ^ sg);
  const real sdr = __uint_as_float(__float_as_uint(dr) ^ sg);
  const real m = (real)2 * fmaxf(fminf(fminf((real)0.25 * fabsf(d2), sdl), sdr), (real)0);
  return __uint_as_float(__float_as_uint(m) | sg);
}
#else
// Under dr dl > 0 neither dl nor dr is NaN, so fmin (one instruction) takes
// the same value as the compare-and-select minimum, infinite slopes included.
__device__ __forceinline__ real lim_slope(real qm1, real q0, real qp1) {
  real dc = (real)0.5 * (qp1 - qm1);
  real dr = qp1 - q0;
  real dl = q0 - qm1;
  if (dr * dl > (real)0) {
    const real m = fmin(fmin(fabs(dc), (real)2 * fabs(dl)), (real)2 * fabs(dr));
    return dc > (real)0 ? m : -m;
  }
  return (real)0;
}
#endif
// interface value between cells a and b from their limited slopes sa, sb
__device__ __forceinline__ real ppm_face(real qa, real qb, real sa, real sb) {
#if defined(NYX_PREC_MIXED)
  return (qa + (real)0.5 * (qb - qa)) - (sb - sa) * (real)(1.0 / 6.0);
#else
  return (qa + (real)0.5 * (qb - qa)) - (sb - sa) / (real)6;
#endif
}
__device__ __forceinline__ void ppm_edges(const real* q5, real chi, real& qm_o, real& qp_o) {
  real qj = q5[2];
  // slopes of cells j-1, j, j+1, each computed once
  const real sm = lim_slope(q5[0], q5[1], q5[2]);
  const real s0 = lim_slope(q5[1], q5[2], q5[3]);
  const real sp = lim_slope(q5[2], q5[3], q5[4]);
  real qp = ppm_face(q5[2], q5[3], s0, sp);
  real qm = ppm_face(q5[1], q5[2], sm, s0);
  qp = chi * qp + ((real)1 - chi) * qj;
  qm = chi * qm + ((real)1 - chi) * qj;
  if ((qp - qj) * (qj - qm) <= (real)0) {
    qp = qj;
    qm = qj;
  } else {
    real dq = qp - qm;
    real t = dq * (qj - (real)0.5 * (qm + qp));
#if defined(NYX_PREC_MIXED)
    real s = dq * dq * (real)(1.0 / 6.0);
#else
    real s = dq * dq / (real)6;
#endif
    if (t > s) qm = (real)3 * qj - (real)2 * qp;
    else if (-s > t) qp = (real)3 * qj - (real)2 * qm;
  }
  qm_o = qm;
  qp_o = qp;
}
// PLM variant (Sec. 3.2): the limited centred slope times the flattening
// coefficient gives the edge values q_j -/+ ds/2 (the tracing below then
// averages the linear profile: the parabola's q6 term vanishes)
__device__ __forceinline__ void plm_edges(const real* q5, real chi, real& qm_o, real& qp_o) {
  const real qj = q5[2];
  const real ds = chi * lim_slope(q5[1], q5[2], q5[3]);
  qm_o = qj - (real)0.5 * ds;
  qp_o = qj + (real)0.5 * ds;
}
__device__ __forceinline__ real avg_hi(real qp, real dq, real q6, real sig) {
  return qp - (real)0.5 * sig * (dq - ((real)1 - ((real)2 / (real)3) * sig) * q6);
}
__device__ __forceinline__ real avg_lo(real qm, real dq, real q6, real sig) {
  return qm + (real)0.5 * sig * (dq + ((real)1 - ((real)2 / (real)3) * sig) * q6);
}

// One side of the tracing: side = +1 (right face, waves with lam > 0) or -1.
// v[] indexes: 0 rho, nv normal velocity, t1/t2 transverse, 4 p.
template <int SIDE>
__device__ __forceinline__ void trace_side(const real* qc, real c, const real* qe,
                                           const real* dq, const real* q6, const real* lam,
                                           const real* sig, int nv, int t1, int t2,
                                           real* out) {
  const real rho = qc[0];
  const real csq = c * c;
  // averages over each wave's domain of dependence for rho, u_n, p
  real I[3][3];
  const int vid[3] = {0, nv, 4};
  for (int w = 0; w < 3; ++w)
    for (int k = 0; k < 3; ++k) {
      int v = vid[k];
      I[w][k] = SIDE > 0 ? avg_hi(qe[v], dq[v], q6[v], sig[w]) : avg_lo(qe[v], dq[v], q6[v], sig[w]);
    }
  const int fast = SIDE > 0 ? 2 : 0;  // fastest wave toward the face
  const bool fast_in = SIDE > 0 ? (lam[2] > (real)0) : (lam[0] < (real)0);
  real ref[3];
  for (int k = 0; k < 3; ++k) ref[k] = fast_in ? I[fast][k] : qe[vid[k]];
  real D[3][3];
  for (int w = 0; w < 3; ++w) {
    bool in = SIDE > 0 ? (lam[w] > (real)0) : (lam[w] < (real)0);
    for (int k = 0; k < 3; ++k) D[w][k] = in ? ref[k] - I[w][k] : (real)0;
  }
#if defined(NYX_PREC_MIXED)
  const real ic = (real)1 / c;
  const real icsq = ic * ic;
  real am = (real)0.5 * (D[0][2] * icsq - (rho * D[0][1]) * ic);
  real ap = (real)0.5 * (D[2][2] * icsq + (rho * D[2][1]) * ic);
  real a0 = D[1][0] - D[1][2] * icsq;
  out[0] = ref[0] - ((am + a0) + ap);
  out[nv] = ref[1] - (c * __builtin_amdgcn_rcpf(rho)) * (ap - am);
#else
  real am = (real)0.5 * (D[0][2] / csq - (rho * D[0][1]) / c);
  real ap = (real)0.5 * (D[2][2] / csq + (rho * D[2][1]) / c);
  real a0 = D[1][0] - D[1][2] / csq;
  out[0] = ref[0] - ((am + a0) + ap);
  out[nv] = ref[1] - (c / rho) * (ap - am);
#endif
  out[4] = ref[2] - csq * (am + ap);
  const bool c_in = SIDE > 0 ? (lam[1] > (real)0) : (lam[1] < (real)0);
  out[t1] = c_in ? (SIDE > 0 ? avg_hi(qe[t1], dq[t1], q6[t1], sig[1])
                             : avg_lo(qe[t1], dq[t1], q6[t1], sig[1]))
                 : qe[t1];
  out[t2] = c_in ? (SIDE > 0 ? avg_hi(qe[t2], dq[t2], q6[t2], sig[1])
                             : avg_lo(qe[t2], dq[t2], q6[t2], sig[1]))
                 : qe[t2];
}

// The direction of a launch row is uniform per workgroup; each stage body is
// instantiated per direction so that component and stride choices are
// compile-time constants instead of selects.
// The tracing of one cell of the [-1, n]^3 range in direction D (E-index e,
// E-coordinates ie, je, ke): its low- and high-side edge states after the
// half-step sources and the floors, in lo and hi; returns the floors applied.
template <int D>
__device__ __forceinline__ unsigned trace_cell(const StepArgs& A, const BoxDev& b, const StepC& C,
                                               unsigned e, int ie, int je, int ke, real* lo,
                                               real* hi) {
  constexpr int d = D;
  unsigned floors = 0;
  {
    const real* prim = (const real*)A.work + b.w_prim;
    const unsigned c0 = pidx_e(b, ie, je, ke);
    const unsigned s = d == 0 ? 1u : (d == 1 ? (unsigned)b.px : (unsigned)b.px * (unsigned)b.py);
    // every load of the cell is issued before any arithmetic, so a wave
    // waits once for all of them instead of once per variable
    const real chi = ldu((const real*)A.work + b.w_chi, e);
    real qs[5][5];
    for (int v = 0; v < 5; ++v)
      for (int o = -2; o <= 2; ++o) qs[v][o + 2] = ldu(prim + v * b.P + (long long)o * s, c0);
    const real c = ldu(prim + 5 * b.P, c0);
    const real* G = (const real*)A.grav + b.goff;
    const real g[3] = {ldu(G, c0), ldu(G + b.gstride, c0), ldu(G + 2 * b.gstride, c0)};
    real qc[5], qm[5], qp[5], dq[5], q6[5];
    for (int v = 0; v < 5; ++v) {
      const real* q5 = qs[v];
      qc[v] = q5[2];
      if (A.recon == NYX_RECON_PLM) plm_edges(q5, chi, qm[v], qp[v]);
      else ppm_edges(q5, chi, qm[v], qp[v]);
      dq[v] = qp[v] - qm[v];
      q6[v] = (real)6 * qc[v] - (real)3 * (qm[v] + qp[v]);
    }
    const int nv = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
    const real u = qc[nv];
    real lam[3] = {u - c, u, u + c};
    const real kh = (real)C.kh;
    real sig[3];
    for (int w = 0; w < 3; ++w) sig[w] = fabs(lam[w]) * kh;
    trace_side<+1>(qc, c, qp, dq, q6, lam, sig, nv, t1, t2, hi);
    trace_side<-1>(qc, c, qm, dq, q6, lam, sig, nv, t1, t2, lo);
    // half-step gravity and expansion sources, then floors
    const real hdt_a = (real)C.hdt_a, hda_a = (real)C.hda_a, pexp = (real)C.pexp;
    const real sd_ = (real)A.small_dens, sp_ = (real)A.small_pres;
    real* out[2] = {lo, hi};
    for (int sd = 0; sd < 2; ++sd) {
      real* q = out[sd];
      for (int dd = 0; dd < 3; ++dd) q[1 + dd] = q[1 + dd] + (hdt_a * g[dd] - hda_a * qc[1 + dd]);
      q[4] = q[4] - pexp * qc[4];
      if (q[0] < sd_) { q[0] = sd_; floors++; }
      if (q[4] < sp_) { q[4] = sp_; floors++; }
    }
  }
  return floors;
}
template <int D>
__device__ __forceinline__ void store_edges(const StepArgs& A, const BoxDev& b, unsigned e,
                                            const real* lo, const real* hi) {
  real* W = (real*)A.work + b.w_edge;
  for (int v = 0; v < 5; ++v) {
    stu(W + ((D * 2 + 0) * 5 + v) * b.E, e, lo[v]);
    stu(W + ((D * 2 + 1) * 5 + v) * b.E, e, hi[v]);
  }
}
template <int D>
__device__ __forceinline__ unsigned trace_dir(const StepArgs& A, const BoxDev& b, unsigned idx) {
  int ec[3];
  space_coords(b, kSpaceE, idx, ec);
  real lo[5], hi[5];
  const unsigned floors = trace_cell<D>(A, b, step_consts(A, b), idx, ec[0], ec[1], ec[2], lo, hi);
  store_edges<D>(A, b, idx, lo, hi);
  return floors;
}

__device__ __forceinline__ void trace_body(const StepArgs& A, const Item& it) {
  int d;
  Loc L = locate(A, kStTrace, kSpaceE, it, &d);
  d += A.dir0;
  const BoxDev& b = *L.bd;
  unsigned floors = 0;
  if (L.idx < b.E) {
    if (d == 0) floors = trace_dir<0>(A, b, L.idx);
    else if (d == 1) floors = trace_dir<1>(A, b, L.idx);
    else floors = trace_dir<2>(A, b, L.idx);
  }
  if (A.stats) count(A, kFloorHits, floors);
}
__global__ __launch_bounds__(kBlock) void k_trace(StepArgs A) { trace_body(A, launch_item(A, kStTrace)); }

// ---------------------------------------------------------------------------
// two-shock Riemann solver (O5), always FP64
// ---------------------------------------------------------------------------
struct RiemannOut {
  double r, u, v, w, p;          // Godunov state at x/t = 0 (rotated frame)
  double pstar, ustar, rsL, rsR;  // star pressure, velocity and densities
  int iters;
};

// Wave structure of a star state and its sample at x/t = 0 (O5, exact
// divisions and square roots): a shock (p* >= p_K) is one front at
// u_K -/+ W_K / rho_K; a rarefaction has its head at u_K -/+ c_K and its tail
// at u* -/+ c*_K with linear interpolation between them; u* = 0 takes the
// mean of both sides.
__device__ __forceinline__ void sample_star(double gam, const double* qL, const double* qR,
                                            double pstar, double ustar, double rsL, double rsR,
                                            double WL, double WR, RiemannOut& o) {
  const double rl = qL[0], ul = qL[1], pl = qL[4];
  const double rr = qR[0], ur = qR[1], pr = qR[4];
  const double cL = sqrt((gam * pl) / rl), cR = sqrt((gam * pr) / rr);
  const double csL = sqrt((gam * pstar) / rsL), csR = sqrt((gam * pstar) / rsR);
  double shdL, stlL, shdR, stlR;
  if (pstar >= pl) { shdL = ul - WL / rl; stlL = shdL; }
  else { shdL = ul - cL; stlL = ustar - csL; }
  if (pstar >= pr) { shdR = ur + WR / rr; stlR = shdR; }
  else { shdR = ur + cR; stlR = ustar + csR; }
  double sL0, sL1, sL2, sR0, sR1, sR2;
  if (shdL >= 0.0) { sL0 = rl; sL1 = ul; sL2 = pl; }
  else if (stlL <= 0.0) { sL0 = rsL; sL1 = ustar; sL2 = pstar; }
  else {
    double f = (0.0 - shdL) / (stlL - shdL);
    sL0 = rl + f * (rsL - rl);
    sL1 = ul + f * (ustar - ul);
    sL2 = pl + f * (pstar - pl);
  }
  if (shdR <= 0.0) { sR0 = rr; sR1 = ur; sR2 = pr; }
  else if (stlR >= 0.0) { sR0 = rsR; sR1 = ustar; sR2 = pstar; }
  else {
    double f = (0.0 - shdR) / (stlR - shdR);
    sR0 = rr + f * (rsR - rr);
    sR1 = ur + f * (ustar - ur);
    sR2 = pr + f * (pstar - pr);
  }
  if (ustar > 0.0) {
    o.r = sL0; o.u = sL1; o.p = sL2; o.v = qL[2]; o.w = qL[3];
  } else if (ustar < 0.0) {
    o.r = sR0; o.u = sR1; o.p = sR2; o.v = qR[2]; o.w = qR[3];
  } else {
    o.r = 0.5 * (sL0 + sR0);
    o.u = 0.5 * (sL1 + sR1);
    o.p = 0.5 * (sL2 + sR2);
    o.v = 0.5 * (qL[2] + qR[2]);
    o.w = 0.5 * (qL[3] + qR[3]);
  }
  o.pstar = pstar;
  o.ustar = ustar;
  o.rsL = rsL;
  o.rsR = rsR;
}

#if !defined(NYX_PREC_MIXED)
// Linearised approximate solver (the alternative Sec. 3.2 compares the
// two-shock solver against): acoustic star state with impedances
// W_K = sqrt(gamma p_K rho_K), rho*_K = rho_K + (p* - p_K)/c_K^2
// (>= (1 - 1/gamma) rho_K once p* is floored), sampled with the two-shock
// wave structure; no iteration.
__device__ __forceinline__ RiemannOut lin_solve(const StepArgs& A, const double* qL,
                                                const double* qR) {
  const double gam = A.gamma;
  const double g2 = 0.5 * (gam + 1.0);
  const double rl = qL[0], ul = qL[1], pl = qL[4];
  const double rr = qR[0], ur = qR[1], pr = qR[4];
  const double CL = (gam * pl) * rl;
  const double CR = (gam * pr) * rr;
  const double W0L = sqrt(CL), W0R = sqrt(CR);
  double p = ((W0R * pl + W0L * pr) + (W0L * W0R) * (ul - ur)) / (W0L + W0R);
  p = vmax(p, A.small_pres);
  const double ustar = ((W0L * ul + W0R * ur) + (pl - pr)) / (W0L + W0R);
  const double rsL = rl + (p - pl) / ((gam * pl) / rl);
  const double rsR = rr + (p - pr) / ((gam * pr) / rr);
  const double WL = sqrt(CL + (g2 * rl) * (p - pl));
  const double WR = sqrt(CR + (g2 * rr) * (p - pr));
  RiemannOut o;
  sample_star(gam, qL, qR, p, ustar, rsL, rsR, WL, WR, o);
  o.iters = 0;
  return o;
}
#endif

#if defined(NYX_PREC_MIXED)
// FP64 reciprocal and reciprocal square root from the hardware estimates
// (relative error below 2^-24, measured on gfx950) refined by one
// Newton-Raphson step each: relative error about 2^-47, not correctly
// rounded.  Arguments are positive and finite where used.
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = x * y;
  double r = fma(-h, y, 1.0);
  return fma(0.5 * y, r, y);
}
// Raw hardware estimates (relative error below 2^-24, FP64 range) for
// quantities that only scale a Newton step or feed the FP32-stored sample of
// the wave fan.
__device__ __forceinline__ double rcp_est(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ double rsq_est(double x) { return __builtin_amdgcn_rsq(x); }

// The two-shock Newton iteration, rearranged so that each evaluation needs
// one reciprocal and two reciprocal square roots: with
// X_K = W_K^2 = C_K + (gamma+1)/2 rho_K (p - p_K) and w_K = 1/W_K,
//   u*_L = u_L - (p - p_L) w_L,  u*_R = u_R + (p - p_R) w_R,
//   1/Z_K = (X_K + C_K) w_K^3 / 2 = w_K (1/2 + (C_K/2) w_K^2),
//   p' = p - (u*_R - u*_L) / (1/Z_L + 1/Z_R),
//   u* = (u*_L / Z_R + u*_R / Z_L) / (1/Z_L + 1/Z_R),
//   1/rho*_K = 1/rho_K - (p* - p_K) w_K^2.
// The converged pressure is the root of u*_R - u*_L: under the default
// stopping rule it takes the raw w_K estimates, which shift that root by
// about their own relative error (2^-24, the FP32 rounding of the stored
// state); tighter rules take the refined w_K (ts_iterate).  The slope
// 1/Z_L + 1/Z_R only scales the step, so its reciprocal is always the raw
// estimate: a relative error of 2^-24 in a step that the stopping rule bounds
// by 2^-12 p moves p' by less than 2^-36 p.
struct TwoShock {
  double gam, sp, rl, ul, pl, rr, ur, pr, CL, CR, hCL, hCR, gl, gr;
};
struct TwoShockEval {
  double XL, XR, wL, wR, usL, usR, zL, zR;
};
__device__ __forceinline__ TwoShock ts_setup(const StepArgs& A, const double* qL,
                                             const double* qR) {
  TwoShock t;
  t.gam = A.gamma;
  t.sp = A.small_pres;
  t.rl = qL[0]; t.ul = qL[1]; t.pl = qL[4];
  t.rr = qR[0]; t.ur = qR[1]; t.pr = qR[4];
  t.CL = (t.gam * t.pl) * t.rl;
  t.CR = (t.gam * t.pr) * t.rr;
  t.hCL = 0.5 * t.CL;
  t.hCR = 0.5 * t.CR;
  const double g2 = 0.5 * (t.gam + 1.0);
  t.gl = g2 * t.rl;
  t.gr = g2 * t.rr;
  return t;
}
__device__ __forceinline__ TwoShockEval ts_eval(const TwoShock& t, double p) {
  TwoShockEval e;
  e.XL = t.CL + t.gl * (p - t.pl);
  e.XR = t.CR + t.gr * (p - t.pr);
  e.wL = rsq64(e.XL);
  e.wR = rsq64(e.XR);
  e.usL = t.ul - (p - t.pl) * e.wL;
  e.usR = t.ur + (p - t.pr) * e.wR;
  e.zL = (0.5 + t.hCL * (e.wL * e.wL)) * e.wL;
  e.zR = (0.5 + t.hCR * (e.wR * e.wR)) * e.wR;
  return e;
}
// fmax is the floor max(p', small_pres): small_pres is never NaN
__device__ __forceinline__ double ts_newton(const TwoShock& t, const TwoShockEval& e, double p) {
  return fmax(p - (e.usR - e.usL) * rcp_est(e.zL + e.zR), t.sp);
}
// The two-shock relations at the converged pressure for the sample: the same
// expressions as ts_eval with estimate-only reciprocal square roots.
__device__ __forceinline__ TwoShockEval ts_eval_est(const TwoShock& t, double p) {
  TwoShockEval e;
  e.XL = t.CL + t.gl * (p - t.pl);
  e.XR = t.CR + t.gr * (p - t.pr);
  e.wL = rsq_est(e.XL);
  e.wR = rsq_est(e.XR);
  e.usL = t.ul - (p - t.pl) * e.wL;
  e.usR = t.ur + (p - t.pr) * e.wR;
  e.zL = (0.5 + t.hCL * (e.wL * e.wL)) * e.wL;
  e.zR = (0.5 + t.hCR * (e.wR * e.wR)) * e.wR;
  return e;
}

// Sample at x/t = 0 of the wave of one side, written for the left side:
// (r, u, p) is the side's state with its normal velocity mirrored for the
// right side (u -> -u, and likewise u*), X and w from the two-shock
// relations, D = 1/rho* of that side.  Shock: one front at u - W/rho;
// rarefaction: head u - c, tail u* - c*, linear in between.
__device__ __forceinline__ void sample_side(double gam, double r, double ir, double u, double p,
                                            double X, double w, double D, double rs, double us,
                                            double ps, double* out) {
  double shd, stl;
  if (ps >= p) {
    shd = u - (X * w) * ir;
    stl = shd;
  } else {
    const double x0 = (gam * p) * ir, x1 = (gam * ps) * D;
    shd = u - x0 * rsq_est(x0);
    stl = us - x1 * rsq_est(x1);
  }
  if (shd >= 0.0) {
    out[0] = r; out[1] = u; out[2] = p;
  } else if (stl <= 0.0) {
    out[0] = rs; out[1] = us; out[2] = ps;
  } else {
    const double f = (0.0 - shd) * rcp_est(stl - shd);
    out[0] = r + f * (rs - r);
    out[1] = u + f * (us - u);
    out[2] = p + f * (ps - p);
  }
}

// Star state from the converged pressure p (u* with a refined reciprocal,
// star densities from the estimates) and the sample at x/t = 0: only the
// side the contact moves away from is sampled, both sides (and their mean)
// when u* = 0.
// Sample of a star state (p*, u*, 1/rho*_K = D_K) with the wave data X_K,
// w_K = X_K^-1/2 of each side: only the side the contact moves away from,
// both sides (and their mean) when u* = 0.
__device__ __forceinline__ RiemannOut sample_upwind(const TwoShock& t, double XL, double XR,
                                                   double wL, double wR, double irl,
                                                   double irr, double DL, double DR,
                                                   double rsL, double rsR, double ustar,
                                                   double pstar, const double* qL,
                                                   const double* qR) {
  const bool left = !(ustar < 0.0);  // u* > 0 samples the left wave, u* = 0 both
  const double sg = left ? 1.0 : -1.0;
  double s1[3];
  sample_side(t.gam, left ? t.rl : t.rr, left ? irl : irr, sg * (left ? t.ul : t.ur),
              left ? t.pl : t.pr, left ? XL : XR, left ? wL : wR, left ? DL : DR,
              left ? rsL : rsR, sg * ustar, pstar, s1);
  RiemannOut o;
  if (ustar != 0.0) {
    o.r = s1[0]; o.u = sg * s1[1]; o.p = s1[2];
    o.v = left ? qL[2] : qR[2];
    o.w = left ? qL[3] : qR[3];
  } else {
    double s2[3];
    sample_side(t.gam, t.rr, irr, -t.ur, t.pr, XR, wR, DR, rsR, -ustar, pstar, s2);
    o.r = 0.5 * (s1[0] + s2[0]);
    o.u = 0.5 * (s1[1] - s2[1]);
    o.p = 0.5 * (s1[2] + s2[2]);
    o.v = 0.5 * (qL[2] + qR[2]);
    o.w = 0.5 * (qL[3] + qR[3]);
  }
  o.pstar = pstar;
  o.ustar = ustar;
  o.rsL = rsL;
  o.rsR = rsR;
  o.iters = 0;
  return o;
}

// star state from the converged pressure p (u* with a refined reciprocal,
// star densities from the Hugoniot relation with the estimates) and its sample
__device__ __forceinline__ RiemannOut ts_finish(const TwoShock& t, const TwoShockEval& e,
                                                double p, const double* qL, const double* qR) {
  const double ustar = (e.usL * e.zR + e.usR * e.zL) * rcp64(e.zL + e.zR);
  const double irl = rcp_est(t.rl), irr = rcp_est(t.rr);
  const double DL = irl - (p - t.pl) * (e.wL * e.wL);
  const double DR = irr - (p - t.pr) * (e.wR * e.wR);
  return sample_upwind(t, e.XL, e.XR, e.wL, e.wR, irl, irr, DL, DR, rcp_est(DL), rcp_est(DR),
                       ustar, p, qL, qR);
}

// The same star state and sample for the plain solver, with the reciprocal
// and star density of the sampled (upwind) side only, both sides when u* = 0:
// the same expressions as ts_finish and sample_upwind, so the same Godunov
// state, two reciprocal estimates fewer per face.  The star density of the
// side not sampled is returned as 0.
__device__ __forceinline__ RiemannOut ts_finish_upwind(const TwoShock& t, const TwoShockEval& e,
                                                       double p, const double* qL,
                                                       const double* qR) {
  const double ustar = (e.usL * e.zR + e.usR * e.zL) * rcp64(e.zL + e.zR);
  const bool left = !(ustar < 0.0);  // u* > 0 samples the left wave, u* = 0 both
  const double r = left ? t.rl : t.rr, pk = left ? t.pl : t.pr, w = left ? e.wL : e.wR;
  const double ir = rcp_est(r);
  const double D = ir - (p - pk) * (w * w);
  const double rs = rcp_est(D);
  double s1[3];
  sample_side(t.gam, r, ir, left ? t.ul : -t.ur, pk, left ? e.XL : e.XR, w, D, rs,
              left ? ustar : -ustar, p, s1);
  RiemannOut o;
  if (ustar != 0.0) {
    o.r = s1[0]; o.u = left ? s1[1] : -s1[1]; o.p = s1[2];
    o.v = left ? qL[2] : qR[2];
    o.w = left ? qL[3] : qR[3];
  } else {
    const double irr = rcp_est(t.rr);
    const double DR = irr - (p - t.pr) * (e.wR * e.wR);
    double s2[3];
    sample_side(t.gam, t.rr, irr, -t.ur, t.pr, e.XR, e.wR, DR, rcp_est(DR), -ustar, p, s2);
    o.r = 0.5 * (s1[0] + s2[0]);
    o.u = 0.5 * (s1[1] - s2[1]);
    o.p = 0.5 * (s1[2] + s2[2]);
    o.v = 0.5 * (qL[2] + qR[2]);
    o.w = 0.5 * (qL[3] + qR[3]);
  }
  o.pstar = p;
  o.ustar = ustar;
  o.rsL = left ? rs : 0.0;
  o.rsR = left ? 0.0 : rs;
  o.iters = 0;
  return o;
}

// Linearised solver of this build: the acoustic star state (refined
// reciprocals), linearised star densities rho*_K = rho_K + (p* - p_K) rho_K^2
// / C_K, and the same upwind sample as the two-shock solver.
__device__ __forceinline__ RiemannOut lin_solve(const StepArgs& A, const double* qL,
                                                const double* qR) {
  const TwoShock t = ts_setup(A, qL, qR);
  const double W0L = t.CL * rsq64(t.CL), W0R = t.CR * rsq64(t.CR);
  const double iW = rcp64(W0L + W0R);
  double p = ((W0R * t.pl + W0L * t.pr) + (W0L * W0R) * (t.ul - t.ur)) * iW;
  p = vmax(p, t.sp);
  const double ustar = ((W0L * t.ul + W0R * t.ur) + (t.pl - t.pr)) * iW;
  const double rsL = t.rl + (p - t.pl) * ((t.rl * t.rl) * rcp_est(t.CL));
  const double rsR = t.rr + (p - t.pr) * ((t.rr * t.rr) * rcp_est(t.CR));
  const double XL = t.CL + t.gl * (p - t.pl), XR = t.CR + t.gr * (p - t.pr);
  RiemannOut o = sample_upwind(t, XL, XR, rsq_est(XL), rsq_est(XR), rcp_est(t.rl),
                               rcp_est(t.rr), rcp_est(rsL), rcp_est(rsR), rsL, rsR, ustar, p,
                               qL, qR);
  o.iters = 0;
  return o;
}

// Newton iterations from p until a step falls below mixed_stop p (at most
// maxiter in all).  RAW evaluates the two-shock relations with the raw
// reciprocal square-root estimates: their relative error (below 2^-24) moves
// the root of u*_R - u*_L by about that much, the size of the FP32 rounding of
// the stored Godunov state, and lies far below a stopping step of 2^-20 or
// more; tighter stopping rules take the refined w_K.
// true where the stopping step lies far enough above the raw estimates'
// error for the iteration to use them (see ts_iterate)
__host__ __device__ __forceinline__ bool raw_stop(const StepArgs& A) { return A.mixed_stop >= 0x1p-20; }
template <bool RAW>
__device__ __forceinline__ double ts_iterate(const StepArgs& A, const TwoShock& t, double p,
                                             int& it) {
  while (it < A.maxiter) {
    const TwoShockEval e = RAW ? ts_eval_est(t, p) : ts_eval(t, p);
    const double pn = ts_newton(t, e, p);
    ++it;
    const bool conv = fabs(pn - p) <= A.mixed_stop * pn;
    p = pn;
    if (conv) break;
  }
  return p;
}

// BOTH: the star densities of both sides (training records); otherwise the
// sampled side's only.  RS selects the iteration's w_K: 0 by the stopping
// rule at run time, 1 the raw estimates, 2 the refined ones (a kernel that
// fixes RS holds one copy of the loop instead of two).
template <bool BOTH = false, int RS = 0>
__device__ __forceinline__ RiemannOut two_shock(const StepArgs& A, const double* qL,
                                                const double* qR) {
  const TwoShock t = ts_setup(A, qL, qR);
  // acoustic initial guess (estimates suffice for a starting point)
  const double W0L = t.CL * rsq_est(t.CL), W0R = t.CR * rsq_est(t.CR);
  double p = ((W0R * t.pl + W0L * t.pr) + (W0L * W0R) * (t.ul - t.ur)) * rcp_est(W0L + W0R);
  p = vmax(p, t.sp);
  // Newton converges quadratically here (Z_K is the exact slope of the
  // two-shock velocity curves), with relative error e' ~ K e^2 and K about
  // 1/4 on a shock branch.  This build stores the Godunov state in FP32, so
  // once a step is below s p (s = max(sqrt(tol), 2^-12)) the accepted
  // pressure is already resolved below FP32 rounding and the iteration stops
  // there.
  int it = 0;
  if constexpr (RS == 1) p = ts_iterate<true>(A, t, p, it);
  else if constexpr (RS == 2) p = ts_iterate<false>(A, t, p, it);
  else p = raw_stop(A) ? ts_iterate<true>(A, t, p, it) : ts_iterate<false>(A, t, p, it);
  const TwoShockEval e = ts_eval_est(t, p);
  RiemannOut o = BOTH ? ts_finish(t, e, p, qL, qR) : ts_finish_upwind(t, e, p, qL, qR);
  o.iters = it;
  return o;
}

// Learned solve.  The network's pressure guess p0 = Pbar exp(y0) is corrected
// by one Newton step of the two-shock relations; the result is accepted when
// the network's output is finite, the face's inputs lie in the training
// domain (`in_domain`), the two-shock velocity residual |u*_R(p1) -
// u*_L(p1)| / cbar at the corrected pressure is below tol and the star state
// is positive and finite.  Otherwise the plain two-shock solver decides the
// face (*used = false).  The Newton step and the residual are two
// evaluations of the two-shock relations, counted as two iterations, on top
// of the fallback solver's own.
constexpr int kLearnedEvals = 2;
__device__ __forceinline__ RiemannOut learned_solve(const StepArgs& A, const double* qL,
                                                    const double* qR, float y0, double pbar,
                                                    double cbar, bool in_domain, bool* used) {
  const TwoShock t = ts_setup(A, qL, qR);
  const bool out_finite = isfinite(y0);  // NaN or infinite weights never pass
  const double y = (double)(y0 < -40.0f ? -40.0f : (y0 > 40.0f ? 40.0f : y0));
  const double p0 = vmax(pbar * exp(y), t.sp);
  const double p1 = ts_newton(t, ts_eval(t, p0), p0);
  const TwoShockEval e = ts_eval(t, p1);
  const double resid = fabs(e.usR - e.usL) * rcp64(cbar);
  // never true for tol = 0 or a NaN residual
  bool ok = out_finite && in_domain && resid < A.mlp_tol;
  if (ok) {
    RiemannOut o = ts_finish(t, e, p1, qL, qR);
    ok = o.rsL > 0.0 && o.rsR > 0.0 && isfinite(o.rsL) && isfinite(o.rsR) && isfinite(o.r) &&
         isfinite(o.u) && isfinite(o.p) && o.r > 0.0 && o.p > 0.0;
    if (ok) {
      *used = true;
      o.iters = kLearnedEvals;
      return o;
    }
  }
  *used = false;
  RiemannOut o = two_shock(A, qL, qR);
  o.iters += kLearnedEvals;
  return o;
}
#else

// BOTH and RS are the mixed build's choices of star densities and of the
// iteration's reciprocal square roots; this build always computes both
// densities with correctly rounded arithmetic
template <bool BOTH = true, int RS = 0>
__device__ __forceinline__ RiemannOut two_shock(const StepArgs& A, const double* qL,
                                                const double* qR) {
  const double gam = A.gamma;
  const double g2 = 0.5 * (gam + 1.0);
  const double sp = A.small_pres;
  const double rl = qL[0], ul = qL[1], pl = qL[4];
  const double rr = qR[0], ur = qR[1], pr = qR[4];
  const double CL = (gam * pl) * rl;
  const double CR = (gam * pr) * rr;
  const double W0L = sqrt(CL), W0R = sqrt(CR);
  double p = ((W0R * pl + W0L * pr) + (W0L * W0R) * (ul - ur)) / (W0L + W0R);
  p = vmax(p, sp);
  int it = 0;
  double WL, WR, usL, usR, ZL, ZR;
  while (it < A.maxiter) {
    WL = sqrt(CL + (g2 * rl) * (p - pl));
    WR = sqrt(CR + (g2 * rr) * (p - pr));
    usL = ul - (p - pl) / WL;
    usR = ur + (p - pr) / WR;
    ZL = ((2.0 * WL) * WL) * WL / (WL * WL + CL);
    ZR = ((2.0 * WR) * WR) * WR / (WR * WR + CR);
    double pn = p - ((ZL * ZR) * (usR - usL)) / (ZL + ZR);
    pn = vmax(pn, sp);
    ++it;
    bool conv = fabs(pn - p) <= A.riemann_tol * pn;
    p = pn;
    if (conv) break;
  }
  WL = sqrt(CL + (g2 * rl) * (p - pl));
  WR = sqrt(CR + (g2 * rr) * (p - pr));
  usL = ul - (p - pl) / WL;
  usR = ur + (p - pr) / WR;
  ZL = ((2.0 * WL) * WL) * WL / (WL * WL + CL);
  ZR = ((2.0 * WR) * WR) * WR / (WR * WR + CR);
  const double ustar = (ZL * usL + ZR * usR) / (ZL + ZR);
  const double pstar = p;
  const double rsL = 1.0 / (1.0 / rl - (pstar - pl) / (WL * WL));
  const double rsR = 1.0 / (1.0 / rr - (pstar - pr) / (WR * WR));
  RiemannOut o;
  sample_star(gam, qL, qR, pstar, ustar, rsL, rsR, WL, WR, o);
  o.iters = it;
  return o;
}
#endif  // NYX_PREC_MIXED

// Godunov state of a d-face as stored (rotated frame: rho, u_n, v_t1, w_t2, p)
__device__ __forceinline__ void store_god(real* G, long long E, unsigned i, const RiemannOut& g) {
  stu(G, i, (real)g.r);
  stu(G + E, i, (real)g.u);
  stu(G + 2 * E, i, (real)g.v);
  stu(G + 3 * E, i, (real)g.w);
  stu(G + 4 * E, i, (real)g.p);
}

// A stored Godunov state of a face, in the rotated frame of that face.
struct God {
  real r, u, v, w, p;
};
__device__ __forceinline__ God ld_god(const real* G, long long E, unsigned i) {
  return God{ldu(G, i), ldu(G + E, i), ldu(G + 2 * E, i), ldu(G + 3 * E, i), ldu(G + 4 * E, i)};
}

// O6: lab-frame fluxes of a d-face from its Godunov state (flux arithmetic
// in real): f = (f_rho, f_mx, f_my, f_mz, f_E, f_e, p_g, u_g).
__device__ __forceinline__ void face_flux(const StepArgs& A, int d, const God& g, real* f) {
  const real gm1 = (real)(A.gamma - 1.0);
  const real r = g.r, u = g.u, v = g.v, w = g.w, p = g.p;
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const real ru = r * u;
  f[0] = ru;
  f[1 + d] = ru * u + p;
  f[1 + t1] = ru * v;
  f[1 + t2] = ru * w;
#if defined(NYX_PREC_MIXED)
  const real igm1 = A.igm1f;  // (real)1 / gm1, computed on the host
  const real rE = p * igm1 + ((real)0.5 * r) * ((u * u + v * v) + w * w);
  f[4] = u * (rE + p);
  f[5] = (u * p) * igm1;
#else
  const real rE = p / gm1 + ((real)0.5 * r) * ((u * u + v * v) + w * w);
  f[4] = u * (rE + p);
  f[5] = (u * p) / gm1;
#endif
  f[6] = p;
  f[7] = u;
}
__device__ __forceinline__ void face_flux(const StepArgs& A, int d, const real* G, long long E,
                                          unsigned i, real* f) {
  face_flux(A, d, ld_god(G, E, i), f);
}

__device__ __forceinline__ void e_coords(const BoxDev& b, unsigned e, int* c) {
  space_coords(b, kSpaceE, e, c);
}
__device__ __forceinline__ unsigned e_stride(const BoxDev& b, int d) {
  return d == 0 ? 1u : (d == 1 ? (unsigned)b.ex : (unsigned)b.ex * (unsigned)b.ey);
}

// ---------------------------------------------------------------------------
// O7: transverse correction of a lab-frame edge state (FP64 arithmetic).
// Dc[5]: summed flux differences (high minus low t-face) of rho, m, E;
// De: summed differences of the internal-energy flux plus the p div u term.
// ---------------------------------------------------------------------------
// add the differences of one transverse direction t (stored Godunov states
// at the low and high t-faces of a cell) to Dc, De; the first direction sets
// them, a second one is added, in that order
template <bool FIRST>
__device__ __forceinline__ void tdiff(const StepArgs& A, int t, const God& glo, const God& ghi,
                                      double* Dc, double& De) {
  real fm[8], fp[8];
  face_flux(A, t, glo, fm);
  face_flux(A, t, ghi, fp);
#if defined(NYX_PREC_MIXED)
  // flux differences are flux arithmetic: FP32, widened once
  for (int c = 0; c < 5; ++c) {
    const double dd = (double)(fp[c] - fm[c]);
    Dc[c] = FIRST ? dd : Dc[c] + dd;
  }
  const double de = (double)((fp[5] - fm[5]) + (0.5f * (fp[6] + fm[6])) * (fp[7] - fm[7]));
#else
  for (int c = 0; c < 5; ++c) {
    const double dd = (double)fp[c] - (double)fm[c];
    Dc[c] = FIRST ? dd : Dc[c] + dd;
  }
  const double de = ((double)fp[5] - (double)fm[5]) +
                    (0.5 * ((double)fp[6] + (double)fm[6])) * ((double)fp[7] - (double)fm[7]);
#endif
  De = FIRST ? de : De + de;
}
template <bool FIRST>
__device__ __forceinline__ void tdiff(const StepArgs& A, int t, const real* Glo, const real* Ghi,
                                      unsigned i, long long E, double* Dc, double& De) {
  tdiff<FIRST>(A, t, ld_god(Glo, E, i), ld_god(Ghi, E, i), Dc, De);
}

__device__ __forceinline__ bool trans_correct(const StepArgs& A, const double* q,
                                              const double* Dc, double De, double kap,
                                              double* out) {
  const double gm1 = A.gamma - 1.0;
  const double rho = q[0], ux = q[1], uy = q[2], uz = q[3], p = q[4];
  double U[5];
  U[0] = rho;
  U[1] = rho * ux;
  U[2] = rho * uy;
  U[3] = rho * uz;
#if defined(NYX_PREC_MIXED)
  const double Ue = p * A.igm1;  // p * (1 / gm1), the reciprocal from the host
#else
  const double Ue = p / gm1;
#endif
  U[4] = Ue + (0.5 * rho) * ((ux * ux + uy * uy) + uz * uz);
  double Un[5];
  for (int c = 0; c < 5; ++c) Un[c] = U[c] - kap * Dc[c];
  const double Uen = Ue - kap * De;
#if defined(NYX_PREC_MIXED)
  const double iU0 = rcp64(Un[0]);
  const double ke = (0.5 * ((Un[1] * Un[1] + Un[2] * Un[2]) + Un[3] * Un[3])) * iU0;
#else
  const double ke = (0.5 * ((Un[1] * Un[1] + Un[2] * Un[2]) + Un[3] * Un[3])) / Un[0];
#endif
  double pn;
  if (Un[4] - ke > A.eta * Un[4]) pn = gm1 * (Un[4] - ke);
  else pn = gm1 * Uen;
  double r[5];
  r[0] = Un[0];
#if defined(NYX_PREC_MIXED)
  r[1] = Un[1] * iU0;
  r[2] = Un[2] * iU0;
  r[3] = Un[3] * iU0;
#else
  r[1] = Un[1] / Un[0];
  r[2] = Un[2] / Un[0];
  r[3] = Un[3] / Un[0];
#endif
  r[4] = pn;
  bool ok = (r[0] > 0.0) && (r[4] > 0.0);
  for (int c = 0; c < 5; ++c) ok = ok && isfinite(r[c]);
  if (!ok) {
    for (int c = 0; c < 5; ++c) out[c] = q[c];
    return true;
  }
  for (int c = 0; c < 5; ++c) out[c] = r[c];
  return false;
}

__device__ __forceinline__ int pair_index(int d, int t) { return d * 2 + (t == (d + 1) % 3 ? 0 : 1); }

// rotate lab-frame states into the frame of a d-face
__device__ __forceinline__ void rotate(int d, const double* L, double* q) {
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  q[0] = L[0];
  q[1] = L[1 + d];
  q[2] = L[1 + t1];
  q[3] = L[1 + t2];
  q[4] = L[4];
}

#if defined(NYX_PREC_MIXED)
constexpr bool kHasLearned = true;
#else
constexpr bool kHasLearned = false;
#endif

// Riemann solve of one face of the wave.  LEARNED: every lane of the
// wavefront must call it (the network runs wave-wide); `active` marks lanes
// with a real face.  Returns the solution for active lanes.
template <bool LEARNED, bool BOTH = false, int RS = 0>
__device__ __forceinline__ RiemannOut solve(const StepArgs& A, bool active, const double* qL,
                                            const double* qR, __bf16* lds, unsigned* used,
                                            unsigned* fallback) {
  RiemannOut g{};
#if defined(NYX_PREC_MIXED)
  if constexpr (LEARNED) {
    const double one[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    const double* a = active ? qL : one;
    const double* b = active ? qR : one;
    float x[kMlpIn], y[kMlpOut];
    double rbar, cbar, ubar;
    mlp_inputs(A.gamma, a, b, x, &rbar, &cbar, &ubar);
    bool in_domain = true;
    for (int k = 0; k < kMlpIn; ++k) {
      const bool inside = fabsf(x[k]) <= kMlpDomain;  // false for NaN
      in_domain = in_domain && inside;
      x[k] = inside ? x[k] : 0.0f;
    }
    mlp_wave_forward(A.mlp, x, lds, y);
    if (active) {
      bool u = false;
      g = learned_solve(A, qL, qR, y[0], rbar * cbar * cbar, cbar, in_domain, &u);
      *used += u ? 1u : 0u;
      *fallback += u ? 0u : 1u;
    }
    return g;
  }
#endif
  if (active) g = A.linear_riemann ? lin_solve(A, qL, qR) : two_shock<BOTH, RS>(A, qL, qR);
  return g;
}

// ---------------------------------------------------------------------------
// stage 4: Riemann on stage-0 states, faces between cells of [-1, n]
// ---------------------------------------------------------------------------
struct Tally {
  unsigned calls = 0, iters = 0, reverts = 0, used = 0, fb = 0;
};

template <bool LEARNED, int D>
__device__ __forceinline__ void riem0_dir(const StepArgs& A, const BoxDev& b, unsigned idx,
                                          __bf16* lds, Tally& T) {
  constexpr int d = D;
  int c[3] = {0, 0, 0};
  if (idx < b.E) e_coords(b, idx, c);
  const bool active = idx < b.E && c[d] >= 1;  // face f = c[d] - 1 in [0, n_d]
  const unsigned e = idx;
  double ql[5], qr[5];
  if (active) {
    const long long sL = e_stride(b, d);  // left cell: shift in the base, same offset e
    const real* W = (const real*)A.work + b.w_edge;
    double Ls[5], Rs[5];
    for (int v = 0; v < 5; ++v) {
      Ls[v] = (double)ldu(W + ((d * 2 + 1) * 5 + v) * b.E - sL, e);
      Rs[v] = (double)ldu(W + ((d * 2 + 0) * 5 + v) * b.E, e);
    }
    rotate(d, Ls, ql);
    rotate(d, Rs, qr);
  }
  RiemannOut g = solve<LEARNED>(A, active, ql, qr, lds, &T.used, &T.fb);
  if (active) {
    T.calls = 1;
    T.iters = g.iters;
    store_god((real*)A.work + b.w_f0 + (long long)d * kGod * b.E, b.E, e, g);
  }
}

template <bool LEARNED>
__device__ __forceinline__ void count_tally(const StepArgs& A, const Tally& T, bool reverts) {
  if (A.stats) {
    count(A, kRiemannCalls, T.calls);
    count(A, kRiemannIters, T.iters);
    if (reverts) count(A, kTransReverts, T.reverts);
    if (LEARNED) {
      count(A, kMlpUsed, T.used);
      count(A, kMlpFallback, T.fb);
    }
  }
}

// mlp_lds: the block's (kBlock / 64) x kMlpWaveLds network tile (learned)
template <bool LEARNED>
__device__ __forceinline__ void riem0_body(const StepArgs& A, const Item& it, __bf16* mlp_lds) {
  int d;
  Loc L = locate(A, kStRiem0, kSpaceE, it, &d);
  d += A.dir0;
  const BoxDev& b = *L.bd;
  __bf16* lds = mlp_lds + (threadIdx.x >> 6) * kMlpWaveLds * LEARNED;
  Tally T;
  if (d == 0) riem0_dir<LEARNED, 0>(A, b, L.idx, lds, T);
  else if (d == 1) riem0_dir<LEARNED, 1>(A, b, L.idx, lds, T);
  else riem0_dir<LEARNED, 2>(A, b, L.idx, lds, T);
  count_tally<LEARNED>(A, T, false);
}
template <bool LEARNED>
__global__ __launch_bounds__(kBlock) void k_riem0(StepArgs A) {
  __shared__ __bf16 mlp_lds[LEARNED ? (kBlock / 64) * kMlpWaveLds : 1];
  riem0_body<LEARNED>(A, launch_item(A, kStRiem0), mlp_lds);
}

// ---------------------------------------------------------------------------
// fused front (launch mode NYX_LAUNCH_FUSED): stages 3 and 4 of x in one
// kernel.  Each cell is traced as k_trace traces it and its edge states are
// stored, and each x-face is solved as k_riem0 solves it, from the high-side
// state of the cell below and the low-side state of the cell above, which
// the kernel still holds instead of reading them back.  (A thread walking a
// column along y or z, carrying the high-side state in registers, was
// slower than the staged kernels for those directions.)
// ---------------------------------------------------------------------------
// the stage-0 solve of the D-face at E-index e from the stage-array states L
// (high side of the cell below) and R (low side of the cell above)
template <int D>
__device__ __forceinline__ void riem0_face(const StepArgs& A, const BoxDev& b, unsigned e,
                                           bool active, const real* L, const real* R, Tally& T) {
  double ql[5], qr[5];
  if (active) {
    double Ls[5], Rs[5];
    for (int v = 0; v < 5; ++v) {
      Ls[v] = (double)L[v];
      Rs[v] = (double)R[v];
    }
    rotate(D, Ls, ql);
    rotate(D, Rs, qr);
  }
  RiemannOut g = solve<false>(A, active, ql, qr, nullptr, &T.used, &T.fb);
  if (active) {
    T.calls += 1;
    T.iters += g.iters;
    store_god((real*)A.work + b.w_f0 + (long long)D * kGod * b.E, b.E, e, g);
  }
}

// x: wavefront w of block bb holds E-cells bb kFrontOwn + 63 w - 1 + lane.
// Lane 0's cell is the previous wavefront's last: lane 0 only traces it,
// for the high-side state lane 1 takes.  Every other lane stores its
// cell's edge states and solves the x-face below the cell (none at the
// range's first column) with the state of lane - 1.
__device__ __forceinline__ void front_x(const StepArgs& A, const BoxDev& b, const StepC& C,
                                        unsigned bb, unsigned& floors, Tally& T) {
  const int lane = (int)(threadIdx.x & 63);
  const long long e = (long long)bb * kFrontOwn + (long long)(threadIdx.x >> 6) * 63 + lane - 1;
  const bool on = e >= 0 && e < b.E;
  const bool own = on && lane > 0;
  int ec[3] = {0, 0, 0};
  real lo[5] = {}, hi[5] = {};
  unsigned fl = 0;
  if (on) {
    space_coords(b, kSpaceE, (unsigned)e, ec);
    fl = trace_cell<0>(A, b, C, (unsigned)e, ec[0], ec[1], ec[2], lo, hi);
  }
  if (own) {
    floors += fl;
    store_edges<0>(A, b, (unsigned)e, lo, hi);
  }
  real left[5];
  for (int v = 0; v < 5; ++v) left[v] = __shfl_up(hi[v], 1, 64);
  riem0_face<0>(A, b, (unsigned)e, own && ec[0] >= 1, left, lo, T);
}

__global__ __launch_bounds__(kBlock) void k_front(StepArgs A) {
  const unsigned x = xcd_linear_block(true);
  const int* pre = A.prefix[kSpaceF];
  int lo = 0, hi = A.nb;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= (int)x) lo = mid;
    else hi = mid;
  }
  const BoxDev& b = A.table[lo];
  unsigned floors = 0;
  Tally T;
  front_x(A, b, step_consts(A, b), x - (unsigned)pre[lo], floors, T);
  if (A.stats) count(A, kFloorHits, floors);
  count_tally<false>(A, T, false);
}

// ---------------------------------------------------------------------------
// stage 5: for one direction d, the d-states of a face's two cells corrected
// by stage-0 t-fluxes (t = t1 and t = t2), Riemann -> F^{d|t1}, F^{d|t2}.
// Both pairs share the loads of the d-states.
// ---------------------------------------------------------------------------
// Learned form: grid.y = 6, one (direction, pair K) per thread (fewer live
// registers next to the network's accumulators).  The plain form takes both
// pairs of a direction per thread (riem1_both below).
template <int D, int K>
__device__ __forceinline__ void riem1_pair(const StepArgs& A, const BoxDev& b, unsigned idx,
                                           __bf16* lds, Tally& T) {
  constexpr int d = D;
  constexpr int t = K == 0 ? (D + 1) % 3 : (D + 2) % 3;
  int c[3] = {0, 0, 0};
  if (idx < b.E) e_coords(b, idx, c);
  const unsigned e = idx;
  const bool active = idx < b.E && c[d] >= 1 && c[t] >= 1 && c[t] <= b.n[t];
  // the left cell's arrays are read through bases shifted by -sdd, so every
  // load of the thread uses the one offset e
  const long long sdd = e_stride(b, d);
  double ql[5], qr[5];
  if (active) {
    const StepC& C = step_consts(A, b);
    const real* W = (const real*)A.work + b.w_edge;
    const long long stt = e_stride(b, t);
    const real* G0 = (const real*)A.work + b.w_f0 + (long long)t * kGod * b.E;
    double qs[2][5];
    for (int s = 0; s < 2; ++s) {
      const long long sh = s == 0 ? -sdd : 0;
      const int side = s == 0 ? 1 : 0;  // left cell gives its right-face state
      double q[5];
      for (int v = 0; v < 5; ++v) q[v] = (double)ldu(W + ((d * 2 + side) * 5 + v) * b.E + sh, e);
      const real* Gc = G0 + sh;
      double Dc[5], De;
      tdiff<true>(A, t, Gc, Gc + stt, e, b.E, Dc, De);
      T.reverts += trans_correct(A, q, Dc, De, C.kap1, qs[s]) ? 1u : 0u;
    }
    rotate(d, qs[0], ql);
    rotate(d, qs[1], qr);
  }
  RiemannOut g = solve<true>(A, active, ql, qr, lds, &T.used, &T.fb);
  if (active) {
    T.calls += 1;
    T.iters += g.iters;
    store_god((real*)A.work + b.w_f1 + (long long)pair_index(d, t) * kGod * b.E, b.E, e, g);
  }
}

// Plain form, both pairs of direction D: the corrected states of both pairs
// come first, so the second pair's loads are in flight during the first
// pair's arithmetic instead of after its solve; the second pair's rotated
// states wait in LDS (park, kPark doubles per thread, lane-strided) across
// the first solve, where they would otherwise add live registers and cost
// a wave per SIMD.
constexpr int kPark = 10;
template <int D>
__device__ __forceinline__ void riem1_both(const StepArgs& A, const BoxDev& b, unsigned idx,
                                           double* park, Tally& T) {
  constexpr int d = D;
  int c[3] = {0, 0, 0};
  if (idx < b.E) e_coords(b, idx, c);
  const unsigned e = idx;
  constexpr int ts[2] = {(D + 1) % 3, (D + 2) % 3};
  const bool inb = idx < b.E && c[d] >= 1;
  const bool want[2] = {inb && c[ts[0]] >= 1 && c[ts[0]] <= b.n[ts[0]],
                        inb && c[ts[1]] >= 1 && c[ts[1]] <= b.n[ts[1]]};
  const long long sdd = e_stride(b, d);
  double ql[2][5], qr[2][5];
  if (want[0] || want[1]) {
    const StepC& C = step_consts(A, b);
    const real* W = (const real*)A.work + b.w_edge;
    double q[2][5];
    for (int s = 0; s < 2; ++s) {
      const long long sh = s == 0 ? -sdd : 0;
      const int side = s == 0 ? 1 : 0;  // left cell gives its right-face state
      for (int v = 0; v < 5; ++v) q[s][v] = (double)ldu(W + ((d * 2 + side) * 5 + v) * b.E + sh, e);
    }
    for (int k = 0; k < 2; ++k) {
      if (!want[k]) continue;
      const int t = ts[k];
      const long long stt = e_stride(b, t);
      const real* G0 = (const real*)A.work + b.w_f0 + (long long)t * kGod * b.E;
      double qs[2][5];
      for (int s = 0; s < 2; ++s) {
        const real* Gc = G0 + (s == 0 ? -sdd : 0);
        double Dc[5], De;
        tdiff<true>(A, t, Gc, Gc + stt, e, b.E, Dc, De);
        T.reverts += trans_correct(A, q[s], Dc, De, C.kap1, qs[s]) ? 1u : 0u;
      }
      rotate(d, qs[0], ql[k]);
      rotate(d, qs[1], qr[k]);
    }
    if (want[1])
      for (int v = 0; v < 5; ++v) {
        park[v * kBlock + threadIdx.x] = ql[1][v];
        park[(5 + v) * kBlock + threadIdx.x] = qr[1][v];
      }
  }
  // the plain solver needs no wave-wide participation: lanes without a
  // face of pair k skip it
  for (int k = 0; k < 2; ++k) {
    if (!want[k]) continue;
    double l[5], r[5];
    for (int v = 0; v < 5; ++v) {
      l[v] = k == 0 ? ql[0][v] : park[v * kBlock + threadIdx.x];
      r[v] = k == 0 ? qr[0][v] : park[(5 + v) * kBlock + threadIdx.x];
    }
    RiemannOut g = solve<false>(A, true, l, r, nullptr, &T.used, &T.fb);
    T.calls += 1;
    T.iters += g.iters;
    store_god((real*)A.work + b.w_f1 + (long long)pair_index(d, ts[k]) * kGod * b.E, b.E, e, g);
  }
}

// park: kPark x kBlock doubles (plain form); mlp_lds as in riem0_body
template <bool LEARNED>
__device__ __forceinline__ void riem1_body(const StepArgs& A, const Item& it, __bf16* mlp_lds,
                                           double* park) {
  int y;
  Loc L = locate(A, kStRiem1, kSpaceE, it, &y);
  const BoxDev& b = *L.bd;
  __bf16* lds = mlp_lds + (threadIdx.x >> 6) * kMlpWaveLds * LEARNED;
  Tally T;
  if constexpr (LEARNED) {
    switch (y) {
      case 0: riem1_pair<0, 0>(A, b, L.idx, lds, T); break;
      case 1: riem1_pair<0, 1>(A, b, L.idx, lds, T); break;
      case 2: riem1_pair<1, 0>(A, b, L.idx, lds, T); break;
      case 3: riem1_pair<1, 1>(A, b, L.idx, lds, T); break;
      case 4: riem1_pair<2, 0>(A, b, L.idx, lds, T); break;
      default: riem1_pair<2, 1>(A, b, L.idx, lds, T); break;
    }
  } else {
    if (y == 0) riem1_both<0>(A, b, L.idx, park, T);
    else if (y == 1) riem1_both<1>(A, b, L.idx, park, T);
    else riem1_both<2>(A, b, L.idx, park, T);
  }
  count_tally<LEARNED>(A, T, true);
}
template <bool LEARNED>
__global__ __launch_bounds__(kBlock) void k_riem1(StepArgs A) {
  __shared__ __bf16 mlp_lds[LEARNED ? (kBlock / 64) * kMlpWaveLds : 1];
  __shared__ double park[LEARNED ? 1 : kPark * kBlock];
  riem1_body<LEARNED>(A, launch_item(A, kStRiem1), mlp_lds, park);
}

// 32-bit hash of a face for the training-sample harvest
__device__ __forceinline__ unsigned face_hash(unsigned long long seed, int box, long long e, int d) {
  unsigned long long z = seed ^ ((unsigned long long)box << 40) ^ ((unsigned long long)e << 2) ^
                         (unsigned long long)d;
  z = (z ^ (z >> 33)) * 0xff51afd7ed558ccdull;
  z = (z ^ (z >> 33)) * 0xc4ceb9fe1a85ec53ull;
  z ^= z >> 33;
  return (unsigned)z;
}

// ---------------------------------------------------------------------------
// stage 6: final d-states and comoving fluxes on valid faces
// ---------------------------------------------------------------------------
// The final d-states of the face at E-index e (between the cells at E-index
// e - e_d and e; c[d] >= 1 and the transverse coordinates in [1, n]): both
// cells' edge states corrected by the t1- and t2-differences of the stage-1
// states, rotated into the face's frame.  Adds the reverts to *reverts.
// A cell's differences are the same for both of its d-faces, so a caller
// walking faces along d carries them: CARRY = 1 stores the upper cell's
// differences (Dc, De) in carry[6]; CARRY = 2 also takes the lower cell's
// from it instead of loading and differencing its stage-1 states.
template <int D, int CARRY = 0>
__device__ __forceinline__ void final_states(const StepArgs& A, const BoxDev& b, const StepC& C,
                                             unsigned e, double* ql, double* qr,
                                             unsigned* reverts, double* carry = nullptr) {
  constexpr int d = D;
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const long long sdd = e_stride(b, d), s1 = e_stride(b, t1), s2 = e_stride(b, t2);
  const real* W = (const real*)A.work + b.w_edge;
  const real* G1a = (const real*)A.work + b.w_f1 + (long long)pair_index(t1, t2) * kGod * b.E;
  const real* G1b = (const real*)A.work + b.w_f1 + (long long)pair_index(t2, t1) * kGod * b.E;
  // both cells' loads are issued before any arithmetic, so a wave waits
  // once for all of them
  real qe[2][5];
  God ga[2][2], gb[2][2];
  for (int s = 0; s < 2; ++s) {
    const long long sh = s == 0 ? -sdd : 0;  // cell shift in the bases, offset e
    const int side = s == 0 ? 1 : 0;
    for (int v = 0; v < 5; ++v) qe[s][v] = ldu(W + ((d * 2 + side) * 5 + v) * b.E + sh, e);
    if (CARRY == 2 && s == 0) continue;
    ga[s][0] = ld_god(G1a + sh, b.E, e);
    ga[s][1] = ld_god(G1a + sh + s1, b.E, e);
    gb[s][0] = ld_god(G1b + sh, b.E, e);
    gb[s][1] = ld_god(G1b + sh + s2, b.E, e);
  }
  double qs[2][5];
  for (int s = 0; s < 2; ++s) {
    double q[5];
    for (int v = 0; v < 5; ++v) q[v] = (double)qe[s][v];
    double Dc[5], De;
    if (CARRY == 2 && s == 0) {
      for (int c = 0; c < 5; ++c) Dc[c] = carry[c];
      De = carry[5];
    } else {
      tdiff<true>(A, t1, ga[s][0], ga[s][1], Dc, De);   // t1-flux corrected by t2
      tdiff<false>(A, t2, gb[s][0], gb[s][1], Dc, De);  // t2-flux corrected by t1
    }
    if (CARRY != 0 && s == 1) {
      for (int c = 0; c < 5; ++c) carry[c] = Dc[c];
      carry[5] = De;
    }
    *reverts += trans_correct(A, q, Dc, De, C.kap2, qs[s]) ? 1u : 0u;
  }
  rotate(d, qs[0], ql);
  rotate(d, qs[1], qr);
}

template <int MODE, int D>
__device__ __forceinline__ void riem2_dir(const StepArgs& A, const BoxDev& b, unsigned idx,
                                          __bf16* lds, Tally& T) {
  constexpr bool LEARNED = MODE == 1;
  constexpr int d = D;
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  int c[3] = {0, 0, 0};
  if (idx < b.E) e_coords(b, idx, c);
  const unsigned e = idx;
  const bool active = idx < b.E && c[d] >= 1 && c[t1] >= 1 && c[t1] <= b.n[t1] && c[t2] >= 1 &&
                      c[t2] <= b.n[t2];
  double ql[5], qr[5];
  if (active) final_states<D>(A, b, step_consts(A, b), e, ql, qr, &T.reverts);
  RiemannOut g = solve<LEARNED, MODE == 2>(A, active, ql, qr, lds, &T.used, &T.fb);
  if (active) {
    T.calls = 1;
    T.iters = g.iters;
    store_god((real*)A.work + b.w_f2 + (long long)d * kGod * b.E, b.E, e, g);
    if (MODE == 2 && face_hash(A.harvest_seed, b.gidx, e, d) < A.harvest_keep) {
      const unsigned long long slot = atomicAdd(A.harvest_count, 1ull);
      if (slot < (unsigned long long)A.harvest_cap) {
        float* r = A.harvest + 15 * slot;
        for (int v = 0; v < 5; ++v) {
          r[v] = (float)ql[v];
          r[5 + v] = (float)qr[v];
        }
        r[10] = (float)g.pstar;
        r[11] = (float)g.ustar;
        r[12] = (float)g.rsL;
        r[13] = (float)g.rsR;
        r[14] = (float)g.r;
      }
    }
  }
}

// MODE 0: plain; 1: learned; 2: plain and harvest training records
template <int MODE>
__device__ __forceinline__ void riem2_body(const StepArgs& A, const Item& it, __bf16* mlp_lds) {
  constexpr bool LEARNED = MODE == 1;
  int d;
  Loc L = locate(A, kStRiem2, kSpaceE, it, &d);
  const BoxDev& b = *L.bd;
  __bf16* lds = mlp_lds + (threadIdx.x >> 6) * kMlpWaveLds * LEARNED;
  Tally T;
  if (d == 0) riem2_dir<MODE, 0>(A, b, L.idx, lds, T);
  else if (d == 1) riem2_dir<MODE, 1>(A, b, L.idx, lds, T);
  else riem2_dir<MODE, 2>(A, b, L.idx, lds, T);
  count_tally<LEARNED>(A, T, true);
}
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_riem2(StepArgs A) {
  __shared__ __bf16 mlp_lds[MODE == 1 ? (kBlock / 64) * kMlpWaveLds : 1];
  riem2_body<MODE>(A, launch_item(A, kStRiem2), mlp_lds);
}

// O9: comoving flux vector of a final face (Sec. 3.2): F_rho = f_rho/a_h,
// F_m = f_m, F_E = a_h f_E, F_e = a_h f_e; p_g and u_g kept for S_e.
__device__ __forceinline__ void final_flux(const StepArgs& A, int d, const God& g, real ah, real* f) {
  face_flux(A, d, g, f);
  f[0] = f[0] / ah;
  f[4] = ah * f[4];
  f[5] = ah * f[5];
}

// ---------------------------------------------------------------------------
// CFL maximum of one cell (Sec. 3.5), shared by update and estimate_dt
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_speed(const StepArgs& A, double U0, double m0, double m1,
                                             double m2, double Ue, double a) {
  const double gm1 = A.gamma - 1.0;
  double rho = vmax(U0, A.small_dens);
#if defined(NYX_PREC_MIXED)
  const double iar = rcp64(a * rho);
  double re = Ue * rcp64(a * a);
  double p = vmax(gm1 * re, A.small_pres);
  const double x = (A.gamma * p) * rcp64(rho);
  double c = x * rsq64(x);
  double s = 0.0;
  s = vmax(s, fabs(m0 * iar) + c);
  s = vmax(s, fabs(m1 * iar) + c);
  s = vmax(s, fabs(m2 * iar) + c);
#else
  double re = Ue / (a * a);
  double p = vmax(gm1 * re, A.small_pres);
  double c = sqrt((A.gamma * p) / rho);
  double s = 0.0;
  s = vmax(s, fabs(m0 / (a * rho)) + c);
  s = vmax(s, fabs(m1 / (a * rho)) + c);
  s = vmax(s, fabs(m2 / (a * rho)) + c);
#endif
  return s;
}

// kinetic energy |m|^2 / (2 rho) of a momentum in the stored variables
__device__ __forceinline__ double kinetic(const double* m, double rho) {
#if defined(NYX_PREC_MIXED)
  return (0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2])) * rcp64(rho);
#else
  return (0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2])) / rho;
#endif
}

template <int NT = kBlock>
__device__ __forceinline__ void block_max_atomic(double s, unsigned long long* dst) {
  __shared__ double red[NT / 64];
  for (int o = 32; o > 0; o >>= 1) s = vmax(s, __shfl_xor(s, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < NT / 64; ++i) m = vmax(m, red[i]);
    if (m > 0.0) max_bits(dst, m);
  }
  __syncthreads();  // red is free again when the block's next item reduces
}

// ---------------------------------------------------------------------------
// stage 7: conservative update, gravity corrector, dual-energy sync
// ---------------------------------------------------------------------------
// The stored state and the gravity of a valid cell (padded index id).
struct CellIn {
  double U0, Um[3], UE, Ue, g[3];
};
__device__ __forceinline__ CellIn load_cell(const StepArgs& A, const BoxDev& b, unsigned id) {
  CellIn x;
  const double* U = A.Uin + b.soff;
  x.U0 = ldu(U, id);
  x.Um[0] = ldu(U + b.sstride, id);
  x.Um[1] = ldu(U + 2 * b.sstride, id);
  x.Um[2] = ldu(U + 3 * b.sstride, id);
  x.UE = ldu(U + 4 * b.sstride, id);
  x.Ue = ldu(U + 5 * b.sstride, id);
  const real* G = (const real*)A.grav + b.goff;
  x.g[0] = (double)ldu(G, id);
  x.g[1] = (double)ldu(G + b.gstride, id);
  x.g[2] = (double)ldu(G + 2 * b.gstride, id);
  return x;
}

// Flux differences D (rho, m, E, e: high minus low face, summed over the
// directions x, y, z in that order) and the p div u sum Pi of a cell, from
// the final states of its low and high faces (O9).
__device__ __forceinline__ void flux_diff(const StepArgs& A, real ah, const God* gl, const God* gh,
                                          double* D, double& Pi) {
  Pi = 0.0;
  for (int d = 0; d < 3; ++d) {
    real fl[8], fh[8];
    final_flux(A, d, gl[d], ah, fl);
    final_flux(A, d, gh[d], ah, fh);
    for (int c = 0; c < 6; ++c) {
      double dF = (double)fh[c] - (double)fl[c];
      D[c] = (d == 0) ? dF : D[c] + dF;
    }
    double pd = (0.5 * ((double)fh[6] + (double)fl[6])) * ((double)fh[7] - (double)fl[7]);
    Pi = (d == 0) ? pd : Pi + pd;
  }
}

struct CellCount {
  unsigned nsync = 0, nnf = 0, nnd = 0, nne = 0;
};
// Predictor (Step 2), gravity corrector and dual-energy sync (Step 6) of one
// cell from its flux differences; stores the new state at padded index id
// and returns its CFL speed (0 when no dt_next is asked for).
__device__ __forceinline__ double update_apply(const StepArgs& A, const StepC& C, const BoxDev& b,
                                               unsigned id, const CellIn& x, const double* D,
                                               double Pi, CellCount& n) {
  const double U0 = x.U0, UE = x.UE, Ue = x.Ue;
  const double* Um = x.Um;
  const double* g = x.g;
  const double dt = C.dt, kk = C.k;
  // predictor (Step 2)
  const double s0 = U0 - kk * D[0];
  double mh[3], sm[3];
  for (int d = 0; d < 3; ++d) {
    mh[d] = Um[d] - kk * D[1 + d];
    sm[d] = mh[d] + (dt * U0) * g[d];
  }
  double sE;
  if (A.grav_form == 2) {
    // form 2 (Sec. 3.2): E changes by the kinetic energy the gravity
    // momentum update causes, at the new density
    sE = (UE - kk * D[4]) + (kinetic(sm, s0) - kinetic(mh, s0));
  } else {
    sE = (UE - kk * D[4]) + dt * ((Um[0] * g[0] + Um[1] * g[1]) + Um[2] * g[2]);
  }
  double se = (Ue - kk * D[5]) - (kk * C.a_h) * Pi;
  if (A.expansion) {
    // expansion source of both energy equations (Sec. 2.2), predictor part
    sE = sE + C.xo * Ue;
    se = se + C.xo * Ue;
  }
  // corrector (Step 6), same g
  double nm[3];
  for (int d = 0; d < 3; ++d) nm[d] = sm[d] + ((0.5 * dt) * (s0 - U0)) * g[d];
  double nE;
  if (A.grav_form == 2) {
    nE = sE + (kinetic(nm, s0) - kinetic(sm, s0));
  } else {
    nE = sE + (0.5 * dt) * (((sm[0] - Um[0]) * g[0] + (sm[1] - Um[1]) * g[1]) +
                            (sm[2] - Um[2]) * g[2]);
  }
  double ne = se;
  if (A.expansion) {
    // time-centred expansion source: + (S* - S^n) dt / 2
    const double cx = 0.5 * (C.xn * se - C.xo * Ue);
    nE = nE + cx;
    ne = ne + cx;
  }
  // dual-energy sync (Step 6)
#if defined(NYX_PREC_MIXED)
  const double ke = (0.5 * ((nm[0] * nm[0] + nm[1] * nm[1]) + nm[2] * nm[2])) * rcp64(s0);
#else
  const double ke = (0.5 * ((nm[0] * nm[0] + nm[1] * nm[1]) + nm[2] * nm[2])) / s0;
#endif
  if (nE - ke > A.eta * nE) {
    ne = nE - ke;
  } else {
    nE = ne + ke;
    n.nsync += 1;
  }
  double* O = A.Uout + b.soff;
  stu(O, id, s0);
  stu(O + b.sstride, id, nm[0]);
  stu(O + 2 * b.sstride, id, nm[1]);
  stu(O + 3 * b.sstride, id, nm[2]);
  stu(O + 4 * b.sstride, id, nE);
  stu(O + 5 * b.sstride, id, ne);
  bool fin = isfinite(s0) && isfinite(nm[0]) && isfinite(nm[1]) && isfinite(nm[2]) &&
             isfinite(nE) && isfinite(ne);
  n.nnf += fin ? 0 : 1;
  n.nnd += s0 <= 0.0 ? 1 : 0;
  n.nne += ne <= 0.0 ? 1 : 0;
  return A.dt_next ? cell_speed(A, s0, nm[0], nm[1], nm[2], ne, A.a_new) : 0.0;
}

template <int NT = kBlock>
__device__ __forceinline__ void count_cells(const StepArgs& A, const CellCount& n) {
  if (A.stats) {
    count<NT>(A, kSyncEfromE, n.nsync);
    count<NT>(A, kNonfinite, n.nnf);
    count<NT>(A, kNegDens, n.nnd);
    count<NT>(A, kNegEint, n.nne);
  }
}

__device__ __forceinline__ void update_body(const StepArgs& A, const Item& it) {
  Loc L = locate(A, kStUpdate, kSpaceV, it);
  const BoxDev& b = *L.bd;
  CellCount n;
  double smax = 0.0;
  if (L.idx < b.V) {
    int vc[3];
    space_coords(b, kSpaceV, L.idx, vc);
    const int i = vc[0], j = vc[1], k = vc[2];
    const StepC& C = step_consts(A, b);
    const unsigned e = ((unsigned)(k + 1) * (unsigned)b.ey + (unsigned)(j + 1)) * (unsigned)b.ex +
                       (unsigned)(i + 1);
    const real* G2 = (const real*)A.work + b.w_f2;
    const unsigned id = ((unsigned)(k + b.ng) * (unsigned)b.py + (unsigned)(j + b.ng)) *
                            (unsigned)b.px + (unsigned)(i + b.ng);
    // every load of the cell is issued before any arithmetic
    God gl[3], gh[3];
    for (int d = 0; d < 3; ++d) {
      const real* G = G2 + (long long)d * kGod * b.E;
      gl[d] = ld_god(G, b.E, e);
      gh[d] = ld_god(G + (long long)e_stride(b, d), b.E, e);
    }
    const CellIn x = load_cell(A, b, id);
    double D[6], Pi;
    flux_diff(A, (real)C.a_h, gl, gh, D, Pi);
    smax = update_apply(A, C, b, id, x, D, Pi, n);
  }
  count_cells(A, n);
  if (A.dt_next) block_max_atomic(smax, A.smax + b.gidx);
}
__global__ __launch_bounds__(kBlock) void k_update(StepArgs A) {
  update_body(A, launch_item(A, kStUpdate));
}

// ---------------------------------------------------------------------------
// stages 6 and 7 fused (plain solver, no harvest).  A workgroup takes a tile
// of TX x TY cell columns of a box and marches up one chunk of at most
// kFinPlanes planes in z (a chunk above the first solves its bottom z-face
// again: the chunk below owns it).  Per plane it
// solves the low x- and y-faces of its cells and each cell's high z-face,
// and also the x-faces past the tile's last column and the y-faces past its
// last row (solved again by the neighbouring tile unless they bound the box;
// only the tile that owns a face counts it).  The x- and y-face states meet
// in LDS, the z-face state stays in registers for the next plane, and each
// cell is updated as soon as its six faces are known: the final face states
// never reach HBM.  Every face and every cell runs the code of the staged
// riem2 and update kernels, so the new state, the counters and dt_next are
// those of the staged launches bit for bit.
// ---------------------------------------------------------------------------
constexpr int kFinXs = kFinBlock + kFinBlock / 2;  // x-face slots: TY (TX + 1), TX >= 2
constexpr int kFinYs = kFinBlock + 64;             // y-face slots: (TY + 1) TX, TX <= 64

__device__ __forceinline__ void lds_put(real* L, int stride, int slot, const God& g) {
  L[slot] = g.r;
  L[stride + slot] = g.u;
  L[2 * stride + slot] = g.v;
  L[3 * stride + slot] = g.w;
  L[4 * stride + slot] = g.p;
}
__device__ __forceinline__ God lds_get(const real* L, int stride, int slot) {
  return God{L[slot], L[stride + slot], L[2 * stride + slot], L[3 * stride + slot],
             L[4 * stride + slot]};
}

// The final face at E-index e in direction D when `on`, as the staged riem2
// stores it (real); counted in T when `own`.
template <int D, int CARRY = 0, int RS = 0>
__device__ __forceinline__ God final_face(const StepArgs& A, const BoxDev& b, const StepC& C,
                                          bool on, bool own, unsigned e, Tally& T,
                                          double* carry = nullptr) {
  double ql[5], qr[5];
  unsigned rv = 0;
  if (on) final_states<D, CARRY>(A, b, C, e, ql, qr, &rv, carry);
  const RiemannOut g = solve<false, false, RS>(A, on, ql, qr, nullptr, &T.used, &T.fb);
  God o{};
  if (on) {
    o = God{(real)g.r, (real)g.u, (real)g.v, (real)g.w, (real)g.p};
    if (own) {
      T.calls += 1;
      T.iters += g.iters;
      T.reverts += rv;
    }
  }
  return o;
}

// Waves per SIMD k_final is compiled for: two workgroups per CU in the mixed
// build (128 VGPRs, no spill); the FP64 build would spill at that count.
#if defined(NYX_PREC_MIXED)
constexpr int kFinWaves = 4;
#else
constexpr int kFinWaves = 2;
#endif
template <int RS>
__global__ __launch_bounds__(kFinBlock, kFinWaves) void k_final(StepArgs A) {
  __shared__ real fx[5 * kFinXs];
  __shared__ real fy[5 * kFinYs];
  // box and tile of the workgroup (tiles numbered XCD-contiguously)
  const int lin = (int)xcd_linear_block(true);
  const int* pre = A.prefix[kSpaceT];
  int lo = 0, hi = A.nb;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= lin) lo = mid;
    else hi = mid;
  }
  const BoxDev& b = A.table[lo];
  const StepC& C = step_consts(A, b);
  const int TX = b.tx, TY = b.ty;
  const int tile = lin - pre[lo];
  const int txy = b.ntx * b.nty;
  const int tzi = tile / txy;
  const int tyi = (tile - tzi * txy) / b.ntx;
  const int i0 = (tile - tzi * txy - tyi * b.ntx) * TX, j0 = tyi * TY;
  const int nx = b.n[0], ny = b.n[1];
  const int k0 = tzi * kFinPlanes;
  const int k1 = b.n[2] < k0 + kFinPlanes ? b.n[2] : k0 + kFinPlanes;
  const int t = (int)threadIdx.x;
  const int tj = t / TX, ti = t - tj * TX;
  const bool lane = t < TX * TY;
  const int i = i0 + ti, j = j0 + tj;
  const bool cell = lane && i < nx && j < ny;
  const bool xon = lane && i <= nx && j < ny;  // the x-face below column i (i = nx: the box's last)
  const bool yon = lane && i < nx && j <= ny;
  // faces past the tile: x-faces at i0 + TX of rows j0 + t (threads [0, TY)),
  // y-faces at j0 + TY of columns i0 + t - yo (threads [yo, yo + TX)); yo is
  // a multiple of 64, so each wavefront solves one direction
  const int yo = (TY + 63) & ~63;
  const bool xe = t < TY && i0 + TX <= nx && j0 + t < ny;
  const bool ye = t >= yo && t < yo + TX && j0 + TY <= ny && i0 + (t - yo) < nx;
  const bool xe_own = i0 + TX == nx, ye_own = j0 + TY == ny;
  const unsigned ex = (unsigned)b.ex, exy = (unsigned)b.ex * (unsigned)b.ey;
  const unsigned pxy = (unsigned)b.px * (unsigned)b.py;
  // E-indices at plane k0 (cell (i, j, k) is E-cell (i + 1, j + 1, k + 1));
  // lanes without the face never use theirs
  const unsigned ez0 = (unsigned)(k0 + 1) * exy;
  unsigned e = ez0 + (unsigned)(j + 1) * ex + (unsigned)(i + 1);
  unsigned exe = ez0 + (unsigned)(j0 + t + 1) * ex + (unsigned)(i0 + TX + 1);
  unsigned eye = ez0 + (unsigned)(j0 + TY + 1) * ex + (unsigned)(i0 + (t - yo) + 1);
  unsigned id = (unsigned)(k0 + b.ng) * pxy + (unsigned)(j + b.ng) * (unsigned)b.px +
                (unsigned)(i + b.ng);
  const real ah = (real)C.a_h;
  Tally T;
  CellCount n;
  double smax = 0.0;
  // the z-faces carry each cell's differences from the face below it to
  // the face above
  double zc[6];
  God zl = final_face<2, 1, RS>(A, b, C, cell, k0 == 0, e, T, zc);  // below the first plane
  for (int k = k0; k < k1; ++k) {
    {
      const God g = final_face<0, 0, RS>(A, b, C, xon, true, e, T);
      if (xon) lds_put(fx, kFinXs, tj * (TX + 1) + ti, g);
    }
    {
      const God g = final_face<1, 0, RS>(A, b, C, yon, true, e, T);
      if (yon) lds_put(fy, kFinYs, tj * TX + ti, g);
    }
    if (t < yo) {
      const God g = final_face<0, 0, RS>(A, b, C, xe, xe_own, exe, T);
      if (xe) lds_put(fx, kFinXs, t * (TX + 1) + TX, g);
    } else if (t < yo + TX) {
      const God g = final_face<1, 0, RS>(A, b, C, ye, ye_own, eye, T);
      if (ye) lds_put(fy, kFinYs, TY * TX + (t - yo), g);
    }
    const God zh = final_face<2, 2, RS>(A, b, C, cell, true, e + exy, T, zc);
    CellIn x{};
    if (cell) x = load_cell(A, b, id);
    __syncthreads();
    if (cell) {
      const God gl[3] = {lds_get(fx, kFinXs, tj * (TX + 1) + ti), lds_get(fy, kFinYs, tj * TX + ti),
                         zl};
      const God gh[3] = {lds_get(fx, kFinXs, tj * (TX + 1) + ti + 1),
                         lds_get(fy, kFinYs, (tj + 1) * TX + ti), zh};
      double D[6], Pi;
      flux_diff(A, ah, gl, gh, D, Pi);
      smax = vmax(smax, update_apply(A, C, b, id, x, D, Pi, n));
    }
    zl = zh;
    e += exy;
    exe += exy;
    eye += exy;
    id += pxy;
    // the face slots are free for the next plane (two LDS buffers with one
    // barrier per plane measured slower: 14.3 against 13.7 ms on the stress
    // patches)
    __syncthreads();
  }
  if (A.stats) {
    count<kFinBlock>(A, kRiemannCalls, T.calls);
    count<kFinBlock>(A, kRiemannIters, T.iters);
    count<kFinBlock>(A, kTransReverts, T.reverts);
  }
  count_cells<kFinBlock>(A, n);
  if (A.dt_next) block_max_atomic<kFinBlock>(smax, A.smax + b.gidx);
}

// ---------------------------------------------------------------------------
// flux registers (Sec. 4.3 reflux): after a group's update, each record
// adds scale * dt times the final flux of its face (or the sum of its 2 x 2
// fine faces) to its register slot.  One lane per record; a slot belongs to
// one record, so no two lanes write the same slot.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_flux_record(StepArgs A, const BoxDev* table,
                                                        const FluxRec* recs, long long nrec,
                                                        double* reg, long long nslots) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrec) return;
  const FluxRec R = recs[r];
  const BoxDev& b = table[R.box];
  const StepC& C = step_consts(A, b);
  const int d = R.d;
  const unsigned e = ((unsigned)(R.f[2] + 1) * (unsigned)b.ey + (unsigned)(R.f[1] + 1)) *
                         (unsigned)b.ex + (unsigned)(R.f[0] + 1);
  const real* G = (const real*)A.work + b.w_f2 + (long long)d * kGod * b.E;
  const real ah = (real)C.a_h;
  double acc[6];
  real f[8];
  final_flux(A, d, ld_god(G, b.E, e), ah, f);
  for (int c = 0; c < 6; ++c) acc[c] = (double)f[c];
  if (R.nsub == 2) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const unsigned o1 = e_stride(b, t1), o2 = e_stride(b, t2);
    const unsigned sub[3] = {e + o1, e + o2, e + o1 + o2};
    for (int q = 0; q < 3; ++q) {
      final_flux(A, d, ld_god(G, b.E, sub[q]), ah, f);
      for (int c = 0; c < 6; ++c) acc[c] = acc[c] + (double)f[c];
    }
  }
  const double w = R.scale * C.dt;
  for (int c = 0; c < 6; ++c) {
    double* g = reg + (long long)c * nslots + R.slot;
    *g = *g + w * acc[c];
  }
}

hipError_t launch_flux_record(const StepArgs& a, const BoxDev* table, const FluxRec* recs,
                              long long nrec, double* reg, long long nslots, hipStream_t s) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flux_record, dim3((unsigned)((nrec + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, a, table, recs, nrec, reg, nslots);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, hipStream_t s) {
  const dim3 blk(kBlock);
  auto mark = [&](int i) {
    if (a.ev) (void)hipEventRecord(a.ev[i], s);
  };
  auto learned = [&](int stage) { return kHasLearned && a.mlp && (a.learned_mask >> stage & 1); };
  mark(0);
  hipLaunchKernelGGL(k_prim, dim3(a.nblocks[kSpaceP]), blk, 0, s, a);
  mark(1);
  hipLaunchKernelGGL(k_flat, dim3(a.nblocks[kSpaceE]), blk, 0, s, a);
  mark(2);
  if (a.fuse_front && !learned(0)) {
    // trace and riem0 of x fused, then the staged kernels for y and z
    // (rows 0 and 1 of their grids); stage 3's time holds k_front and the
    // y, z tracing, stage 4's the y, z solves
    StepArgs yz = a;
    yz.dir0 = 1;
    hipLaunchKernelGGL(k_front, dim3(a.nblocks[kSpaceF]), blk, 0, s, a);
    hipLaunchKernelGGL(k_trace, dim3(a.nblocks[kSpaceE], 2), blk, 0, s, yz);
    mark(3);
    hipLaunchKernelGGL(k_riem0<false>, dim3(a.nblocks[kSpaceE], 2), blk, 0, s, yz);
  } else {
    hipLaunchKernelGGL(k_trace, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
    mark(3);
    if (learned(0)) hipLaunchKernelGGL(k_riem0<kHasLearned>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
    else hipLaunchKernelGGL(k_riem0<false>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
  }
  mark(4);
  if (learned(1)) hipLaunchKernelGGL(k_riem1<kHasLearned>, dim3(a.nblocks[kSpaceE], 6), blk, 0, s, a);
  else hipLaunchKernelGGL(k_riem1<false>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
  mark(5);
  if (a.fuse_final && !learned(2) && !a.harvest) {
    // riem2 and update as one launch; its time is stage 6's, stage 7's is 0
#if defined(NYX_PREC_MIXED)
    // the instantiation whose Newton loop matches the stopping rule
    if (raw_stop(a)) hipLaunchKernelGGL(k_final<1>, dim3(a.nblocks[kSpaceT]), dim3(kFinBlock), 0, s, a);
    else hipLaunchKernelGGL(k_final<2>, dim3(a.nblocks[kSpaceT]), dim3(kFinBlock), 0, s, a);
#else
    hipLaunchKernelGGL(k_final<0>, dim3(a.nblocks[kSpaceT]), dim3(kFinBlock), 0, s, a);
#endif
    mark(6);
    mark(7);
    return hipGetLastError();
  }
  if (learned(2)) hipLaunchKernelGGL(k_riem2<kHasLearned ? 1 : 0>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
  else if (a.harvest) hipLaunchKernelGGL(k_riem2<2>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
  else hipLaunchKernelGGL(k_riem2<0>, dim3(a.nblocks[kSpaceE], 3), blk, 0, s, a);
  mark(6);
  hipLaunchKernelGGL(k_update, dim3(a.nblocks[kSpaceV]), blk, 0, s, a);
  mark(7);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// persistent step: the seven stages of a group in one launch.  The grid holds
// as many workgroups as the device keeps resident at once; each stage's
// work items (the blocks of its own launch) are handed out by atomic queues,
// and a grid barrier separates the stages (a stage reads its neighbours'
// results of the previous one).  Every item runs the same stage body as the
// stage's own kernel, so the results are those of the staged launches, bit
// for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int stage_space(int s) {
  return s == kStPrim ? kSpaceP : (s == kStUpdate ? kSpaceV : kSpaceE);
}
__device__ __forceinline__ unsigned stage_rows(int s, bool learned1) {
  if (s == kStPrim || s == kStFlat || s == kStUpdate) return 1u;
  return (s == kStRiem1 && learned1) ? 6u : 3u;
}

template <int LMASK>
__device__ __forceinline__ void run_item(const StepArgs& A, int s, const Item& it, __bf16* mlp,
                                         double* park) {
  switch (s) {
    case kStPrim: prim_body(A, it); break;
    case kStFlat: flat_body(A, it); break;
    case kStTrace: trace_body(A, it); break;
    case kStRiem0: riem0_body<(LMASK & 1) != 0>(A, it, mlp); break;
    case kStRiem1: riem1_body<(LMASK & 2) != 0>(A, it, mlp, park); break;
    case kStRiem2: riem2_body<(LMASK & 4) ? 1 : 0>(A, it, mlp); break;
    default: update_body(A, it); break;
  }
}

// Walk position of workgroup w among G when the workgroups of each XCD
// (dispatched round-robin, w mod 8) take one contiguous range: the same
// numbering the staged launches use.
__device__ __forceinline__ unsigned xcd_position(unsigned w, unsigned G) {
  const unsigned q = G >> 3, r = G & 7;
  const unsigned x = w & 7, k = w >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// How a stage's n work items are handed out to G workgroups.  The first
// S = min(n, G c0) items are split statically: the workgroup at XCD
// position p takes [p c0, (p + 1) c0), c0 = max(1, n / 2G), so a stage with
// no more items than workgroups needs no atomic at all.  The rest [S, n) is
// cut into nr contiguous ranges (8, or 1 with the hardware-order tuning bit
// or when it is small), each with an atomic queue head; a workgroup drains
// the range of its own XCD first, then takes from the others, `chunk` items
// at a time.
struct Share {
  unsigned S, c0, nr, chunk;
};
__device__ __forceinline__ Share share_of(unsigned n, unsigned G, bool hw_order) {
  Share h;
  h.c0 = n / (2u * G);
  h.c0 = h.c0 < 1u ? 1u : h.c0;
  const unsigned long long s = (unsigned long long)G * h.c0;
  h.S = s < n ? (unsigned)s : n;
  const unsigned rest = n - h.S;
  h.nr = (hw_order || rest < 64u * G) ? 1u : 8u;
  h.chunk = rest / (16u * G);
  h.chunk = h.chunk < 1u ? 1u : (h.chunk > 64u ? 64u : h.chunk);
  return h;
}
// Next chunk [b0, b1) of the queued part, taken by one thread; *done marks
// ranges found empty.
__device__ __forceinline__ bool grab(unsigned long long* head, unsigned n, const Share& h,
                                     unsigned home, unsigned* done, unsigned* b0,
                                     unsigned* b1) {
  const unsigned rest = n - h.S;
  for (unsigned k = 0; k < h.nr; ++k) {
    const unsigned r = (home + k) % h.nr;
    if (*done >> r & 1u) continue;
    const unsigned lo = h.S + (unsigned)((unsigned long long)rest * r / h.nr);
    const unsigned hi = h.S + (unsigned)((unsigned long long)rest * (r + 1) / h.nr);
    const unsigned long long v =
        lo < hi ? atomicAdd(head + r, (unsigned long long)h.chunk) : 0ull;
    if (lo < hi && (unsigned long long)lo + v < hi) {
      *b0 = lo + (unsigned)v;
      *b1 = hi - *b0 < h.chunk ? hi : *b0 + h.chunk;
      return true;
    }
    *done |= 1u << r;
  }
  return false;
}

// Grid barrier after stage s.  Each workgroup counts itself in its XCD
// group's counter; the last of a group counts the group as complete; all
// wait for every group.  The fences make every workgroup's stage results
// visible to every XCD before any workgroup goes on.  A barrier that has not
// filled after `ticks` of the wall clock (a workgroup that never became
// resident) raises the abort flag; every workgroup that sees it leaves, so
// each wait ends.  Returns false on abort.
__device__ __forceinline__ bool grid_barrier(unsigned long long* ctl, int s,
                                             unsigned long long ticks) {
  __shared__ int ok_sh;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned G = gridDim.x, x = blockIdx.x & 7u;
    const unsigned long long members = (G + 7u - x) / 8u;
    const unsigned long long groups = G < 8u ? G : 8u;
    if (atomicAdd(ctl + kCtlXcdBar + 8 * s + x, 1ull) + 1ull == members)
      atomicAdd(ctl + kCtlBarrier + s, 1ull);
    const unsigned long long t0 = (unsigned long long)wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(ctl + kCtlBarrier + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           groups) {
      if (__hip_atomic_load(ctl + kCtlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if ((unsigned long long)wall_clock64() - t0 > ticks) {
        atomicExch(ctl + kCtlAbort, 1ull);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

// Waves per SIMD the persistent kernel is compiled for: with all seven stage
// bodies inlined the plain FP32-mixed build needs 132 VGPRs (3 waves), and
// asking for 4 fits it in 128 with a 12-byte spill.  The FP64 build (171
// VGPRs; 4 waves would spill) and the learned form (4 waves would spill 472
// bytes) keep 2.
#if defined(NYX_PREC_MIXED)
constexpr int kPersistWaves = 4;
#else
constexpr int kPersistWaves = 2;
#endif
template <int LMASK>
__global__ __launch_bounds__(kBlock, LMASK ? 2 : kPersistWaves) void k_step_persistent(StepArgs A) {
  __shared__ __bf16 mlp_lds[LMASK ? (kBlock / 64) * kMlpWaveLds : 1];
  __shared__ double park[(LMASK & 2) ? 1 : kPark * kBlock];
  __shared__ unsigned q_sh[3];
  unsigned long long* ctl = A.ctl;
  const unsigned G = gridDim.x;
  const unsigned home = blockIdx.x & 7u;
  const unsigned pos = xcd_position(blockIdx.x, G);
  for (int s = 0; s < kStages; ++s) {
    const unsigned gx = (unsigned)A.nblocks[stage_space(s)];
    const unsigned gy = stage_rows(s, (LMASK & 2) != 0);
    const unsigned n = gx * gy;
    const Share h = share_of(n, G, (A.tune[s] & kTuneHwOrder) != 0);
    // the static share (uniform over the workgroup)
    const unsigned long long f0 = (unsigned long long)pos * h.c0;
    const unsigned s0 = f0 < h.S ? (unsigned)f0 : h.S;
    const unsigned s1 = f0 + h.c0 < h.S ? (unsigned)(f0 + h.c0) : h.S;
    // items need no barrier between them: a body's block-wide scratch
    // (counter and maximum reductions) synchronises itself, the parked
    // states are per thread and the network's tiles per wave
    for (unsigned lin = s0; lin < s1; ++lin) run_item<LMASK>(A, s, Item{lin, gx, gy}, mlp_lds, park);
    unsigned done = 0;
    while (h.S < n) {
      if (threadIdx.x == 0) {
        unsigned b0 = 0, b1 = 0;
        const bool got = grab(ctl + 8 * s, n, h, home, &done, &b0, &b1);
        q_sh[0] = b0;
        q_sh[1] = b1;
        q_sh[2] = got ? 1u : 0u;
      }
      __syncthreads();
      const unsigned b0 = q_sh[0], b1 = q_sh[1];
      const bool got = q_sh[2] != 0;
      __syncthreads();  // every thread has read q_sh before the next take
      if (!got) break;
      for (unsigned lin = b0; lin < b1; ++lin) run_item<LMASK>(A, s, Item{lin, gx, gy}, mlp_lds, park);
    }
    if (s + 1 < kStages && !grid_barrier(ctl, s, A.barrier_ticks)) return;
  }
}

namespace {
template <int LMASK>
int resident_grid() {
  // per device: workgroups of this kernel the device keeps resident at once
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cache[dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_persistent<LMASK>, kBlock,
                                                     0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev] = per_cu * cus;
  }
  return cache[dev];
}
int lmask_of(const StepArgs& a) { return kHasLearned && a.mlp ? a.learned_mask : 0; }
}  // namespace

int persistent_grid(const StepArgs& a) {
  if (a.harvest) return 0;
  const int m = lmask_of(a);
  if (m == 0) return resident_grid<0>();
#if defined(NYX_PREC_MIXED)
  if (m == 7) return resident_grid<7>();
#endif
  return 0;
}

hipError_t launch_step_persistent(const StepArgs& a, hipStream_t s) {
  int grid = persistent_grid(a);
  if (grid <= 0) return hipErrorNotSupported;
  // no more workgroups than the largest stage has items
  long long most = 0;
  const bool l1 = (lmask_of(a) & 2) != 0;
  const long long rows[kStages] = {1, 1, 3, 3, l1 ? 6 : 3, 3, 1};
  const int space[kStages] = {kSpaceP, kSpaceE, kSpaceE, kSpaceE, kSpaceE, kSpaceE, kSpaceV};
  for (int st = 0; st < kStages; ++st) {
    const long long n = (long long)a.nblocks[space[st]] * rows[st];
    most = n > most ? n : most;
  }
  if (most < grid) grid = (int)(most > 0 ? most : 1);
  if (!a.ctl) return hipErrorInvalidValue;
  hipError_t e = launch_zero_u64(a.ctl, kCtlWords, s);
  if (e != hipSuccess) return e;
  if (lmask_of(a) == 0)
    hipLaunchKernelGGL(k_step_persistent<0>, dim3(grid), dim3(kBlock), 0, s, a);
#if defined(NYX_PREC_MIXED)
  else
    hipLaunchKernelGGL(k_step_persistent<7>, dim3(grid), dim3(kBlock), 0, s, a);
#endif
  return hipGetLastError();
}

}  // namespace NYX_NS
}  // namespace nyx
