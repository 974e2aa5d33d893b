// nyx_util.hip -- precision-independent kernels: the hydro CFL reduction
// (Sec. 3.5), the per-box dt finalisation, the level minimum and the ghost
// fills that prepare a step's inputs (Sec. 4.1).  Built without contraction.
#include <hip/hip_runtime.h>

#include "nyx_internal.h"

namespace nyx {

__device__ __forceinline__ double dmaxd(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmind(double a, double b) { return a < b ? a : b; }

__global__ void k_zero_u64(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__device__ __forceinline__ const BoxDev* locate_box(const StepArgs& A, int space, long long& idx,
                                                   bool remap = true) {
  const unsigned bx = xcd_linear_block(remap);  // 1-D grids here
  if (A.table == nullptr) {
    idx = (long long)bx * kBlock + threadIdx.x;
    return &A.single;
  }
  const int* pre = A.prefix[space];
  int lo = 0, hi = A.nb;
  int x = (int)bx;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pre[mid] <= x) lo = mid;
    else hi = mid;
  }
  idx = (long long)(x - pre[lo]) * kBlock + threadIdx.x;
  return A.table + lo;
}

// maximum over valid cells and axes of |U_d| + c (Sec. 3.5), per box
__global__ __launch_bounds__(kBlock) void k_dtmax(StepArgs A, double a) {
  long long v;
  const BoxDev& b = *locate_box(A, kSpaceV, v);
  double s = 0.0;
  if (v < b.V) {
    int vc[3];
    space_coords(b, kSpaceV, (unsigned)v, vc);
    const int i = vc[0], j = vc[1], k = vc[2];
    const long long id = ((long long)(k + b.ng) * b.py + (j + b.ng)) * b.px + (i + b.ng);
    const double* U = A.Uin + b.soff + id;
    const double gm1 = A.gamma - 1.0;
    double rho = dmaxd(U[0], A.small_dens);
    double re = U[5 * b.sstride] / (a * a);
    double p = dmaxd(gm1 * re, A.small_pres);
    double c = sqrt((A.gamma * p) / rho);
    s = dmaxd(s, fabs(U[b.sstride] / (a * rho)) + c);
    s = dmaxd(s, fabs(U[2 * b.sstride] / (a * rho)) + c);
    s = dmaxd(s, fabs(U[3 * b.sstride] / (a * rho)) + c);
  }
  __shared__ double red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) s = dmaxd(s, __shfl_xor(s, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kBlock / 64; ++w) m = dmaxd(m, red[w]);
    if (m > 0.0) max_bits(A.smax + b.gidx, m);
  }
}

hipError_t launch_dtmax(const StepArgs& a, double a_state, hipStream_t s) {
  hipLaunchKernelGGL(k_dtmax, dim3(a.nblocks[kSpaceV]), dim3(kBlock), 0, s, a, a_state);
  return hipGetLastError();
}

// dt = cfl a dx / s_max for each box (one thread per box)
__global__ void k_dt_finalize(StepArgs A, double a, double cfl, double* dt, int nbox) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const BoxDev& b = A.table ? A.table[i] : A.single;
  double smax = __longlong_as_double((long long)A.smax[b.gidx]);
  dt[b.gidx] = ((cfl * a) * b.dx) / smax;
}

hipError_t launch_dt_finalize(const StepArgs& a, double a_state, double cfl, double* dt_out,
                              hipStream_t s) {
  int n = a.table ? a.nb : 1;
  hipLaunchKernelGGL(k_dt_finalize, dim3((n + 255) / 256), dim3(256), 0, s, a, a_state, cfl,
                     dt_out, n);
  return hipGetLastError();
}

__global__ void k_prologue(StepArgs A, int nbox, StepC* consts, BoxDev* single_dst,
                           int* prefix_dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const BoxDev& b = single_dst ? A.single : A.table[i];
  if (single_dst && i == 0) {
    *single_dst = A.single;
    for (int s = 0; s < kSpaces; ++s) {
      prefix_dst[2 * s] = 0;
      prefix_dst[2 * s + 1] = A.nblocks[s];
    }
  }
  StepC c;
  c.dt = A.dt_dev ? A.dt_dev[b.gidx] : A.dt_host;
  c.gm1 = A.gamma - 1.0;
  c.a_h = 0.5 * (A.a_old + A.a_new);
  c.da = A.a_new - A.a_old;
  c.kh = c.dt / (c.a_h * b.dx);
  c.hdt_a = (0.5 * c.dt) / c.a_h;
  c.hda_a = (0.5 * c.da) / c.a_h;
  c.pexp = (1.5 * c.gm1) * (c.da / c.a_h);
  c.kap1 = c.kh / 3.0;
  c.kap2 = c.kh / 2.0;
  c.k = c.dt / b.dx;
  // a adot (2 - 3(gamma-1)) rho e = (adot / a) cgam U_e; integrated over the
  // step at a_old (predictor) and a_new (corrector)
  const double cgam = 2.0 - 3.0 * c.gm1;
  c.xo = cgam * (c.da / A.a_old);
  c.xn = cgam * (c.da / A.a_new);
  c.pad_ = 0.0;
  consts[b.gidx] = c;
}

hipError_t launch_prologue(const StepArgs& a, int nbox, StepC* consts, BoxDev* single_dst,
                           int* prefix_dst, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue, dim3((nbox + 63) / 64), dim3(64), 0, s, a, nbox, consts, single_dst,
                     prefix_dst);
  return hipGetLastError();
}

// sum the per-slot partial counters into the caller's nyx_stats
__global__ void k_stats_reduce(const unsigned long long* slots, unsigned long long* stats) {
  const int f = threadIdx.x;
  if (f >= kStatFields) return;
  unsigned long long t = 0;
  for (int i = 0; i < kStatSlots; ++i) t += slots[i * kStatFields + f];
  if (t) atomicAdd(stats + f, t);
}

hipError_t launch_stats_reduce(const unsigned long long* slots, nyx_stats* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(64), 0, s, slots, (unsigned long long*)stats);
  return hipGetLastError();
}

// level time step: every entry becomes the minimum (one block)
__global__ __launch_bounds__(1024) void k_min_dt(double* dt, int n) {
  __shared__ double red[1024 / 64];
  double m = 1.0 / 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = dmind(m, dt[i]);
  for (int o = 32; o > 0; o >>= 1) m = dmind(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) r = dmind(r, red[w]);
    red[0] = r;
  }
  __syncthreads();
  double r = red[0];
  for (int i = threadIdx.x; i < n; i += blockDim.x) dt[i] = r;
}

hipError_t launch_min_dt(double* dt, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_min_dt, dim3(1), dim3(1024), 0, s, dt, n);
  return hipGetLastError();
}

// Ghost cell q of a box, q < P - V, as box-local coordinates (ghosts negative
// or >= n): first the 2 ng whole padded planes below and above the box in z,
// then the 2 ng padded rows below and above it in y on each valid plane, then
// the ng cells at each end of every valid row.  Planes and rows are
// contiguous in memory across consecutive q.
__device__ __forceinline__ void ghost_coords(const BoxDev& b, unsigned q, int* c) {
  const unsigned ng = (unsigned)b.ng, px = (unsigned)b.px, py = (unsigned)b.py;
  const unsigned n0 = (unsigned)b.n[0], n1 = (unsigned)b.n[1], n2 = (unsigned)b.n[2];
  const unsigned nz = 2u * ng * px * py, ny = 2u * ng * px * n2;
  unsigned pi, pj, pk;
  if (q < nz) {
    const unsigned plane = q / (px * py), r = q - plane * (px * py);
    pj = r / px;
    pi = r - pj * px;
    pk = plane < ng ? plane : n2 + plane;
  } else if (q < nz + ny) {
    const unsigned r = q - nz, row = r / px;
    pi = r - row * px;
    const unsigned kk = row / (2u * ng), jj = row - kk * (2u * ng);
    pj = jj < ng ? jj : n1 + jj;
    pk = kk + ng;
  } else {
    const unsigned r = q - nz - ny, row = r / (2u * ng), ii = r - row * (2u * ng);
    pi = ii < ng ? ii : n0 + ii;
    const unsigned kk = row / n1;
    pj = row - kk * n1 + ng;
    pk = kk + ng;
  }
  c[0] = (int)pi - b.ng;
  c[1] = (int)pj - b.ng;
  c[2] = (int)pk - b.ng;
}

// Ghost fill.  mode 0: periodic within the box.  mode 1: boxes tile a
// periodic domain as a gx*gy*gz grid of equal boxes; `A.table` then points at
// the group's boxes and `full` at the whole list in box order.  The grid is
// the padded-cell grid; the first P - V work items of each box take its ghost
// cells (ghost_coords) and the rest return at once.  Blocks keep the hardware
// order, so the ghost blocks at the start of each box spread over the XCDs.
__global__ __launch_bounds__(kBlock) void k_fill(StepArgs A, const BoxDev* full, double* state,
                                                 int ncomp, int mode, int gx, int gy, int gz) {
  long long id;
  const BoxDev& b = *locate_box(A, kSpaceP, id, false);
  if (id >= b.P - b.V) return;
  int gc[3];
  ghost_coords(b, (unsigned)id, gc);
  const int i = gc[0], j = gc[1], k = gc[2];
  long long src, ss = b.sstride;  // the source cell and its box's component stride
  if (mode == 0) {
    const int si = ((i % b.n[0]) + b.n[0]) % b.n[0];
    const int sj = ((j % b.n[1]) + b.n[1]) % b.n[1];
    const int sk = ((k % b.n[2]) + b.n[2]) % b.n[2];
    src = b.soff + ((long long)(sk + b.ng) * b.py + (sj + b.ng)) * b.px + (si + b.ng);
  } else {
    const int bx = b.gidx % gx, by = (b.gidx / gx) % gy, bz = b.gidx / (gx * gy);
    const int NX = gx * b.n[0], NY = gy * b.n[1], NZ = gz * b.n[2];
    const int X = ((bx * b.n[0] + i) % NX + NX) % NX;
    const int Y = ((by * b.n[1] + j) % NY + NY) % NY;
    const int Z = ((bz * b.n[2] + k) % NZ + NZ) % NZ;
    const int sbx = X / b.n[0], sby = Y / b.n[1], sbz = Z / b.n[2];
    const BoxDev& sb = full[(sbz * gy + sby) * gx + sbx];
    const int si = X - sbx * b.n[0], sj = Y - sby * b.n[1], sk = Z - sbz * b.n[2];
    src = sb.soff + ((long long)(sk + sb.ng) * sb.py + (sj + sb.ng)) * sb.px + (si + sb.ng);
    ss = sb.sstride;
  }
  const long long dst = b.soff + ((long long)(k + b.ng) * b.py + (j + b.ng)) * b.px + (i + b.ng);
  const long long cs = b.sstride;
  if (ncomp == 6) {
    // the gas state: every component is loaded before any is stored (sources
    // are valid cells, destinations ghost cells, so no store feeds a load)
    double v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = state[src + c * ss];
#pragma unroll
    for (int c = 0; c < 6; ++c) state[dst + c * cs] = v[c];
  } else {
    for (int c = 0; c < ncomp; ++c) state[dst + c * cs] = state[src + c * ss];
  }
}

hipError_t launch_fill_periodic(const StepArgs& a, const BoxDev* full, double* state, int ncomp,
                                int mode, int gx, int gy, int gz, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(a.nblocks[kSpaceP]), dim3(kBlock), 0, s, a, full, state, ncomp,
                     mode, gx, gy, gz);
  return hipGetLastError();
}

}  // namespace nyx
