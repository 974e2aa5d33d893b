// nyx_internal.h -- device-side box descriptors and launch arguments shared
// by the host ABI layer (nyx_abi.cpp) and the two precision builds of the
// stage kernels (nyx_step.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nyx_hydro.h"

namespace nyx {

constexpr int kBlock = 256;  // threads per block: 4 wavefronts of 64
constexpr int kFaceVals = 8; // f_rho, f_mx, f_my, f_mz, f_E, f_e, p_g, u_g

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
  d.w_f0 = o;   o += align_elems(3 * kFaceVals * d.E);
  d.w_f1 = o;   o += align_elems(6 * kFaceVals * d.E);
  d.w_f2 = o;   o += align_elems(3 * kFaceVals * d.E);
  if (out) *out = d;
  return o;
}

// Which cell range a launch walks.
enum Space { kSpaceP = 0, kSpaceE = 1, kSpaceV = 2 };

// Launch-wide arguments of a step.
struct StepArgs {
  // box selection: either one box by value, or a device table + block prefix
  BoxDev single;
  const BoxDev* table;     // device, nb entries (batched) or nullptr
  const int* prefix[3];    // device, nb+1 block prefixes per Space (batched)
  int nb;
  int nblocks[3];          // grid size per Space
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
  int maxiter;
  nyx_stats* stats;
  double* dt_next;
  hipEvent_t* ev;          // kStages + 1 events recorded around the stages, or nullptr
};

// stage order of launch_step (for timing)
constexpr int kStages = 7;

// The two precision builds of the stage kernels.
namespace fp64 {
hipError_t launch_step(const StepArgs& a, hipStream_t s);
}
namespace mixed {
hipError_t launch_step(const StepArgs& a, hipStream_t s);
}
// Precision-independent kernels (in nyx_abi.cpp's companion nyx_util.hip).
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_dtmax(const StepArgs& a, double a_state, hipStream_t s);
hipError_t launch_dt_finalize(const StepArgs& a, double a_state, double cfl, double* dt_out,
                              hipStream_t s);
hipError_t launch_min_dt(double* dt, int n, hipStream_t s);
hipError_t launch_fill_periodic(const StepArgs& a, const BoxDev* full, double* state, int ncomp,
                                int mode, int gx, int gy, int gz, hipStream_t s);

}  // namespace nyx
