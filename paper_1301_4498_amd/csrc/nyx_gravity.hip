// nyx_gravity.hip -- the mesh side of the gravity input of the gas step
// (Sec. 2.4 and Sec. 3.4 Self-gravity): cloud-in-cell deposit of particle
// mass, the periodic Poisson equation lap(phi) = coef (rho - mean(rho))
// discretised with the 7-point stencil and solved by geometric multigrid
// V-cycles with red-black Gauss-Seidel relaxation, and g = -grad(phi) by
// centred differences, written in the step's padded gravity layout.
//
// Fields of the periodic domain are stored x fastest without ghost cells.
// Every kernel is a plain stencil over HBM-resident arrays, one lane per
// cell (or per cell of one colour); reductions are deterministic (fixed
// block partials, then one block), so a solve gives the same bits on every
// run.  The deposit adds with hardware FP64 atomics and is therefore exact
// only up to the order of the additions.  Built without contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "nyx_internal.h"

namespace nyx {
namespace grav {

constexpr int kRedBlocks = 4096;  // block partials of a reduction

__device__ __forceinline__ unsigned wrap_dec(unsigned i, unsigned n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ unsigned wrap_inc(unsigned i, unsigned n) { return i + 1 == n ? 0 : i + 1; }

struct Grid {
  unsigned nx, ny, nz;
};

// natural order (the caller's mesh fields): x fastest
__device__ __forceinline__ unsigned nat(const Grid& g, unsigned i, unsigned j, unsigned k) {
  return (k * g.ny + j) * g.nx + i;
}

// the solver's own arrays keep the two colours of the red-black ordering
// apart: colour (i + j + k) & 1 holds its cells x fastest with half-length
// rows, so a half sweep reads the other colour's neighbours, its own rhs
// and writes its own cells, each contiguous across the lanes of a row
__device__ __forceinline__ unsigned at(const Grid& g, unsigned i, unsigned j, unsigned k) {
  const unsigned half = g.nx >> 1;
  return ((i + j + k) & 1) * (half * g.ny * g.nz) + (k * g.ny + j) * half + (i >> 1);
}

__device__ __forceinline__ void coords(const Grid& g, unsigned c, unsigned* i, unsigned* j,
                                       unsigned* k) {
  *i = c % g.nx;
  *j = (c / g.nx) % g.ny;
  *k = c / (g.nx * g.ny);
}

// the six-neighbour sum of the 7-point stencil, (x pair + y pair) + z pair
__device__ __forceinline__ double nb_sum(const double* p, const Grid& g, unsigned i, unsigned j,
                                         unsigned k) {
  const double sx = p[at(g, wrap_dec(i, g.nx), j, k)] + p[at(g, wrap_inc(i, g.nx), j, k)];
  const double sy = p[at(g, i, wrap_dec(j, g.ny), k)] + p[at(g, i, wrap_inc(j, g.ny), k)];
  const double sz = p[at(g, i, j, wrap_dec(k, g.nz))] + p[at(g, i, j, wrap_inc(k, g.nz))];
  return (sx + sy) + sz;
}

// ---- cloud-in-cell deposit: one lane per particle, 8 atomic adds ----
__global__ __launch_bounds__(kBlock) void k_cic(const double* __restrict__ pos,
                                                const double* __restrict__ mass, long long np,
                                                Grid g, double dx, double inv_vol,
                                                double* __restrict__ rho) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  const unsigned n[3] = {g.nx, g.ny, g.nz};
  unsigned lo[3], hi[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    const double s = pos[d * np + p] / dx - 0.5;
    if (!(fabs(s) < 1e15)) return;  // non-finite or absurd position: the particle is skipped
    const double fl = floor(s);
    f[d] = s - fl;
    long long i0 = (long long)fl % (long long)n[d];
    if (i0 < 0) i0 += n[d];
    lo[d] = (unsigned)i0;
    hi[d] = lo[d] + 1 == n[d] ? 0 : lo[d] + 1;
  }
  const double m = mass[p] * inv_vol;
  for (int q = 0; q < 8; ++q) {
    const int b0 = q & 1, b1 = (q >> 1) & 1, b2 = q >> 2;
    double w = 1.0;
    w = w * (b0 ? f[0] : 1.0 - f[0]);
    w = w * (b1 ? f[1] : 1.0 - f[1]);
    w = w * (b2 ? f[2] : 1.0 - f[2]);
    unsafeAtomicAdd(rho + nat(g, b0 ? hi[0] : lo[0], b1 ? hi[1] : lo[1], b2 ? hi[2] : lo[2]),
                    m * w);
  }
}

// total density of a cell: the deposited field plus, when given, the gas
// density of the state (component 0 of a padded box covering the domain)
struct RhoSrc {
  const double* rho;
  const double* state;  // or nullptr
  long long soff;
  unsigned px, py, ng;
};

__device__ __forceinline__ double rho_total(const RhoSrc& R, const Grid& g, unsigned c) {
  double r = R.rho[c];
  if (R.state) {
    const unsigned i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    r = r + R.state[R.soff + ((long long)(k + R.ng) * R.py + (j + R.ng)) * R.px + (i + R.ng)];
  }
  return r;
}

// ---- deterministic reductions: fixed block partials, then one block ----
template <int OP>  // 0: sum, 1: max
__device__ __forceinline__ double combine(double a, double b) {
  return OP == 0 ? a + b : fmax(a, b);
}

template <int OP>
__device__ double block_reduce(double v) {
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = combine<OP>(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

// MODE 0: sum of rho_total (natural order); 1: max |f - L phi|; 2: max |f|;
// 3: sum of phi (solver order)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_partial(RhoSrc R, const double* __restrict__ phi,
                                                    const double* __restrict__ f, Grid g,
                                                    double inv_h2, double* __restrict__ part) {
  constexpr int OP = (MODE == 0 || MODE == 3) ? 0 : 1;
  const unsigned n = g.nx * g.ny * g.nz;
  double acc = 0.0;
  for (unsigned c = blockIdx.x * kBlock + threadIdx.x; c < n; c += gridDim.x * kBlock) {
    double v;
    if (MODE == 0) {
      v = rho_total(R, g, c);
    } else if (MODE == 1) {
      // c walks the solver's order: the cell's colour, row and half index
      const unsigned half = g.nx >> 1, hn = n >> 1;
      const unsigned color = c / hn, r = c - color * hn;
      const unsigned ih = r % half, row = r / half;
      const unsigned j = row % g.ny, k = row / g.ny;
      const unsigned i = 2 * ih + ((j + k + color) & 1);
      const double lap = (nb_sum(phi, g, i, j, k) - 6.0 * phi[c]) * inv_h2;
      v = fabs(f[c] - lap);
    } else if (MODE == 2) {
      v = fabs(f[c]);
    } else {
      v = phi[c];
    }
    acc = combine<OP>(acc, v);
  }
  const double b = block_reduce<OP>(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

template <int OP>
__global__ __launch_bounds__(kBlock) void k_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) acc = combine<OP>(acc, part[i]);
  const double b = block_reduce<OP>(acc);
  if (threadIdx.x == 0) *out = b;
}

// f = coef (rho_total - sum / n) in the solver's order; the initial guess
// copied into it
__global__ __launch_bounds__(kBlock) void k_rhs(RhoSrc R, Grid g, double coef,
                                                const double* __restrict__ sum,
                                                double* __restrict__ f,
                                                const double* __restrict__ phi_in,
                                                double* __restrict__ phi) {
  const unsigned n = g.nx * g.ny * g.nz;
  const unsigned c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  unsigned i, j, k;
  coords(g, c, &i, &j, &k);
  const unsigned a = at(g, i, j, k);
  const double mean = *sum / (double)n;
  f[a] = coef * (rho_total(R, g, c) - mean);
  phi[a] = phi_in[c];
}

// the caller's phi (natural order) = the solution minus sum / n
__global__ __launch_bounds__(kBlock) void k_sub_mean(const double* __restrict__ phi, Grid g,
                                                     const double* __restrict__ sum,
                                                     double* __restrict__ out) {
  const unsigned n = g.nx * g.ny * g.nz;
  const unsigned c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  unsigned i, j, k;
  coords(g, c, &i, &j, &k);
  out[c] = phi[at(g, i, j, k)] - *sum / (double)n;
}

// ---- multigrid kernels ----
// one Gauss-Seidel half sweep: cells with (i + j + k) % 2 == color
__global__ __launch_bounds__(kBlock) void k_rbgs(double* __restrict__ phi,
                                                 const double* __restrict__ f, Grid g, double h2,
                                                 unsigned color) {
  const unsigned half = g.nx >> 1;
  const unsigned t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= half * g.ny * g.nz) return;
  const unsigned ih = t % half, r = t / half;
  const unsigned j = r % g.ny, k = r / g.ny;
  const unsigned i = 2 * ih + ((j + k + color) & 1);
  const unsigned c = at(g, i, j, k);
  phi[c] = (nb_sum(phi, g, i, j, k) - h2 * f[c]) / 6.0;
}

// All sweeps of a small level in one workgroup (the half sweeps separated
// by barriers): the same updates, in the same order, as k_rbgs launches.
__global__ __launch_bounds__(kBlock) void k_rbgs_small(double* __restrict__ phi,
                                                       const double* __restrict__ f, Grid g,
                                                       double h2, int sweeps) {
  const unsigned half = g.nx >> 1, n = half * g.ny * g.nz;
  for (int it = 0; it < sweeps; ++it)
    for (unsigned color = 0; color < 2; ++color) {
      for (unsigned t = threadIdx.x; t < n; t += kBlock) {
        const unsigned ih = t % half, r = t / half;
        const unsigned j = r % g.ny, k = r / g.ny;
        const unsigned i = 2 * ih + ((j + k + color) & 1);
        const unsigned c = at(g, i, j, k);
        phi[c] = (nb_sum(phi, g, i, j, k) - h2 * f[c]) / 6.0;
      }
      __syncthreads();
    }
}

// coarse f = mean of the eight children's residuals f - L phi; coarse phi = 0
__global__ __launch_bounds__(kBlock) void k_restrict(const double* __restrict__ phi,
                                                     const double* __restrict__ f, Grid g,
                                                     double inv_h2, Grid gc,
                                                     double* __restrict__ fc,
                                                     double* __restrict__ phic) {
  const unsigned C = blockIdx.x * kBlock + threadIdx.x;
  if (C >= gc.nx * gc.ny * gc.nz) return;
  const unsigned I = C % gc.nx, J = (C / gc.nx) % gc.ny, K = C / (gc.nx * gc.ny);
  double s = 0.0;
  for (int q = 0; q < 8; ++q) {
    const unsigned i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
    const unsigned c = at(g, i, j, k);
    const double r = f[c] - (nb_sum(phi, g, i, j, k) - 6.0 * phi[c]) * inv_h2;
    s = q == 0 ? r : s + r;
  }
  const unsigned a = at(gc, I, J, K);
  fc[a] = 0.125 * s;
  phic[a] = 0.0;
}

// fine phi += trilinear (cell-centred) interpolation of the coarse
// correction: one lane per coarse cell reads its 3 x 3 x 3 neighbourhood
// once and corrects its eight children; child (a, b, c) takes the parent
// with weight 27/64, the three face neighbours on its side 9/64, the three
// edge neighbours 3/64 and the corner 1/64
__global__ __launch_bounds__(kBlock) void k_prolong(double* __restrict__ phi, Grid g,
                                                    const double* __restrict__ ec, Grid gc) {
  const unsigned C = blockIdx.x * kBlock + threadIdx.x;
  if (C >= gc.nx * gc.ny * gc.nz) return;
  unsigned I, J, K;
  coords(gc, C, &I, &J, &K);
  const unsigned xs[3] = {wrap_dec(I, gc.nx), I, wrap_inc(I, gc.nx)};
  const unsigned ys[3] = {wrap_dec(J, gc.ny), J, wrap_inc(J, gc.ny)};
  const unsigned zs[3] = {wrap_dec(K, gc.nz), K, wrap_inc(K, gc.nz)};
  double e[3][3][3];
  for (int z = 0; z < 3; ++z)
    for (int y = 0; y < 3; ++y)
      for (int x = 0; x < 3; ++x) e[z][y][x] = ec[at(gc, xs[x], ys[y], zs[z])];
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const int X = a ? 2 : 0, Y = b ? 2 : 0, Z = c ? 2 : 0;  // the neighbour on the child's side
    const double c000 = e[1][1][1];
    const double c100 = e[1][1][X], c010 = e[1][Y][1], c001 = e[Z][1][1];
    const double c110 = e[1][Y][X], c101 = e[Z][1][X], c011 = e[Z][Y][1];
    const double c111 = e[Z][Y][X];
    const double v = (27.0 * c000 + 9.0 * ((c100 + c010) + c001) + 3.0 * ((c110 + c101) + c011) +
                      c111) *
                     (1.0 / 64.0);
    const unsigned f = at(g, 2 * I + a, 2 * J + b, 2 * K + c);
    phi[f] = phi[f] + v;
  }
}

// ---- g = -grad(phi) into the padded layout of a box covering the domain ----
template <class T>
__global__ __launch_bounds__(kBlock) void k_gradient(const double* __restrict__ phi, Grid g,
                                                     double two_dx, BoxDev b,
                                                     T* __restrict__ grav) {
  const unsigned c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= (unsigned)b.P) return;
  const unsigned px = (unsigned)b.px, py = (unsigned)b.py;
  const int pi = (int)(c % px), pj = (int)((c / px) % py), pk = (int)(c / (px * py));
  // the periodic image of the padded cell in the domain
  auto wrapc = [](int x, unsigned n) { return (unsigned)(((x % (int)n) + (int)n) % (int)n); };
  const unsigned i = wrapc(pi - b.ng, g.nx), j = wrapc(pj - b.ng, g.ny), k = wrapc(pk - b.ng, g.nz);
  const double gx = -(phi[nat(g, wrap_inc(i, g.nx), j, k)] - phi[nat(g, wrap_dec(i, g.nx), j, k)]) / two_dx;
  const double gy = -(phi[nat(g, i, wrap_inc(j, g.ny), k)] - phi[nat(g, i, wrap_dec(j, g.ny), k)]) / two_dx;
  const double gz = -(phi[nat(g, i, j, wrap_inc(k, g.nz))] - phi[nat(g, i, j, wrap_dec(k, g.nz))]) / two_dx;
  T* out = grav + b.goff;
  out[c] = (T)gx;
  out[b.gstride + c] = (T)gy;
  out[2 * b.gstride + c] = (T)gz;
}

static unsigned blocks_for(unsigned long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Level {
  Grid g;
  double h2, inv_h2;
  double* phi;
  double* f;
};

static int check_dom(const int32_t* dom) {
  if (!dom) return NYX_E_NULL;
  unsigned long long n = 1;
  for (int d = 0; d < 3; ++d) {
    if (dom[d] < 2 || (dom[d] & 1) || dom[d] > (1 << 16)) return NYX_E_SHAPE;
    n *= (unsigned long long)dom[d];
  }
  if (n > (1ull << 31) - 1) return NYX_E_SHAPE;
  return NYX_OK;
}

// level sizes: halve while every extent stays even (red-black sweeps pair
// the cells of a row), down to extents of 2
static std::vector<Grid> levels_of(const int32_t* dom) {
  std::vector<Grid> L;
  Grid g{(unsigned)dom[0], (unsigned)dom[1], (unsigned)dom[2]};
  L.push_back(g);
  while (g.nx % 4 == 0 && g.ny % 4 == 0 && g.nz % 4 == 0) {
    g = Grid{g.nx / 2, g.ny / 2, g.nz / 2};
    L.push_back(g);
  }
  return L;
}

static size_t cells(const Grid& g) { return (size_t)g.nx * g.ny * g.nz; }
static size_t r256(size_t x) { return (x + 255) / 256 * 256; }

// workspace: block partials, 8 scalars, then phi and f of every level in the
// solver's colour-split order, each 256-byte aligned
constexpr size_t kOffScalars = (size_t)kRedBlocks * sizeof(double);
constexpr size_t kOffLevels = kOffScalars + 256;

static size_t mg_bytes(const int32_t* dom) {
  const auto L = levels_of(dom);
  size_t b = kOffLevels;
  for (size_t l = 0; l < L.size(); ++l) b += 2 * r256(cells(L[l]) * sizeof(double));
  return b;
}

template <int MODE, int OP>
static void reduce(const RhoSrc& R, const double* phi, const double* f, const Grid& g, double inv_h2,
            unsigned nb, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_partial<MODE>, dim3(nb), dim3(kBlock), 0, s, R, phi, f, g, inv_h2, part);
  hipLaunchKernelGGL(k_final<OP>, dim3(1), dim3(kBlock), 0, s, part, (int)nb, out);
}

constexpr int kPre = 2, kPost = 2, kCoarseSweeps = 32;

// levels up to this many cells are smoothed by one workgroup
constexpr size_t kSmallCells = 4096;

static hipError_t smooth(const Level& v, int iters, hipStream_t s) {
  if (cells(v.g) <= kSmallCells) {
    hipLaunchKernelGGL(k_rbgs_small, dim3(1), dim3(kBlock), 0, s, v.phi, v.f, v.g, v.h2, iters);
    return hipGetLastError();
  }
  const unsigned nb = blocks_for((unsigned long long)(v.g.nx / 2) * v.g.ny * v.g.nz);
  for (int it = 0; it < iters; ++it)
    for (unsigned color = 0; color < 2; ++color)
      hipLaunchKernelGGL(k_rbgs, dim3(nb), dim3(kBlock), 0, s, v.phi, v.f, v.g, v.h2, color);
  return hipGetLastError();
}

static hipError_t vcycle(std::vector<Level>& L, size_t l, hipStream_t s) {
  if (l + 1 == L.size()) return smooth(L[l], kCoarseSweeps, s);
  hipError_t e = smooth(L[l], kPre, s);
  if (e != hipSuccess) return e;
  const Level& f = L[l];
  Level& c = L[l + 1];
  hipLaunchKernelGGL(k_restrict, dim3(blocks_for(cells(c.g))), dim3(kBlock), 0, s, f.phi, f.f,
                     f.g, f.inv_h2, c.g, c.f, c.phi);
  if ((e = vcycle(L, l + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(cells(c.g))), dim3(kBlock), 0, s, f.phi, f.g,
                     c.phi, c.g);
  return smooth(f, kPost, s);
}

}  // namespace grav
}  // namespace nyx

using namespace nyx;
using namespace nyx::grav;

extern "C" {

int nyx_cic_deposit(const double* pos, const double* mass, long long np, const int32_t* dom,
                    double dx, double* rho, void* stream) {
  int rc = check_dom(dom);
  if (rc) return rc;
  if (!rho) return NYX_E_NULL;
  if (np < 0 || !(dx > 0.0) || !std::isfinite(dx)) return NYX_E_PARAM;
  if (np == 0) return NYX_OK;
  if (!pos || !mass) return NYX_E_NULL;
  Grid g{(unsigned)dom[0], (unsigned)dom[1], (unsigned)dom[2]};
  hipLaunchKernelGGL(k_cic, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     (hipStream_t)stream, pos, mass, np, g, dx, 1.0 / ((dx * dx) * dx), rho);
  return hipGetLastError() == hipSuccess ? NYX_OK : NYX_E_HIP;
}

int nyx_poisson_workspace_bytes(const int32_t* dom, size_t* bytes) {
  int rc = check_dom(dom);
  if (rc) return rc;
  if (!bytes) return NYX_E_NULL;
  *bytes = mg_bytes(dom);
  return NYX_OK;
}

int nyx_poisson_solve(const int32_t* dom, double dx, double coef, const double* rho,
                      const double* state, const nyx_box* box, double* phi, double tol,
                      int max_vcycles, void* workspace, size_t ws_bytes, void* stream,
                      int* vcycles, double* rel_resid) {
  int rc = check_dom(dom);
  if (rc) return rc;
  if (!rho || !phi || !workspace) return NYX_E_NULL;
  if (!(dx > 0.0) || !std::isfinite(dx) || !std::isfinite(coef) || !(tol >= 0.0) ||
      max_vcycles < 1 || max_vcycles > 1000)
    return NYX_E_PARAM;
  if ((uintptr_t)workspace & 255) return NYX_E_WORKSPACE;
  if (ws_bytes < mg_bytes(dom)) return NYX_E_WORKSPACE;
  RhoSrc R{rho, nullptr, 0, 0, 0, 0};
  if (state) {
    if (!box) return NYX_E_NULL;
    if ((rc = validate_box(box))) return rc;
    for (int d = 0; d < 3; ++d)
      if (box->n[d] != dom[d]) return NYX_E_SHAPE;
    R.state = state;
    R.soff = box->state_off;
    R.ng = (unsigned)box->ng;
    R.px = (unsigned)(box->n[0] + 2 * box->ng);
    R.py = (unsigned)(box->n[1] + 2 * box->ng);
  }
  hipStream_t s = (hipStream_t)stream;
  const auto G = levels_of(dom);
  double* part = (double*)workspace;
  double* scal = (double*)((char*)workspace + kOffScalars);  // sum rho, max|f|, max|r|, sum phi
  char* w = (char*)workspace + kOffLevels;
  std::vector<Level> L(G.size());
  double h = dx;
  for (size_t l = 0; l < G.size(); ++l) {
    L[l].g = G[l];
    L[l].h2 = h * h;
    L[l].inv_h2 = 1.0 / (h * h);
    L[l].phi = (double*)w;
    w += r256(cells(G[l]) * sizeof(double));
    L[l].f = (double*)w;
    w += r256(cells(G[l]) * sizeof(double));
    h *= 2.0;
  }
  const Level& F = L[0];
  const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(cells(F.g)));
  // right-hand side and its size
  reduce<0, 0>(R, F.phi, F.f, F.g, F.inv_h2, nb, part, scal + 0, s);
  hipLaunchKernelGGL(k_rhs, dim3(blocks_for(cells(F.g))), dim3(kBlock), 0, s, R, F.g, coef,
                     scal + 0, F.f, phi, F.phi);
  if (hipGetLastError() != hipSuccess) return NYX_E_HIP;
  // with tol > 0 or a residual requested the stream is synchronised (once,
  // then once per V-cycle); otherwise only kernels are enqueued
  const bool check = tol > 0.0 || rel_resid;
  auto read = [&](const double* src, double* dst) {
    return hipMemcpyAsync(dst, src, sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
  };
  double fnorm = 0.0, rmax = 0.0, rel = 0.0;
  if (check) {
    reduce<2, 1>(R, F.phi, F.f, F.g, F.inv_h2, nb, part, scal + 1, s);
    if (!read(scal + 1, &fnorm)) return NYX_E_HIP;
  }
  int done = 0;
  for (int cyc = 0; cyc < max_vcycles; ++cyc) {
    if (vcycle(L, 0, s) != hipSuccess) return NYX_E_HIP;
    ++done;
    if (tol > 0.0 || (check && cyc + 1 == max_vcycles)) {
      reduce<1, 1>(R, F.phi, F.f, F.g, F.inv_h2, nb, part, scal + 2, s);
      if (!read(scal + 2, &rmax)) return NYX_E_HIP;
      rel = fnorm > 0.0 ? rmax / fnorm : rmax;
      if (tol > 0.0 && rel <= tol) break;
    }
  }
  // the periodic problem fixes phi up to a constant: remove its mean
  reduce<3, 0>(R, F.phi, F.f, F.g, F.inv_h2, nb, part, scal + 3, s);
  hipLaunchKernelGGL(k_sub_mean, dim3(blocks_for(cells(F.g))), dim3(kBlock), 0, s, F.phi, F.g,
                     scal + 3, phi);
  if (hipGetLastError() != hipSuccess) return NYX_E_HIP;
  if (vcycles) *vcycles = done;
  if (rel_resid) *rel_resid = rel;
  return NYX_OK;
}

int nyx_gravity_from_phi(const int32_t* dom, double dx, const double* phi, const nyx_box* box,
                         void* grav, int precision, void* stream) {
  int rc = check_dom(dom);
  if (rc) return rc;
  if (!phi || !box || !grav) return NYX_E_NULL;
  if ((rc = validate_box(box))) return rc;
  for (int d = 0; d < 3; ++d)
    if (box->n[d] != dom[d]) return NYX_E_SHAPE;
  if (!(dx > 0.0) || !std::isfinite(dx)) return NYX_E_PARAM;
  if (precision != NYX_FP64 && precision != NYX_MIXED) return NYX_E_PARAM;
  BoxDev b;
  box_layout(*box, 0, 0, &b);
  Grid g{(unsigned)dom[0], (unsigned)dom[1], (unsigned)dom[2]};
  const double two_dx = 2.0 * dx;
  hipStream_t s = (hipStream_t)stream;
  if (precision == NYX_FP64)
    hipLaunchKernelGGL(k_gradient<double>, dim3(blocks_for(b.P)), dim3(kBlock), 0, s, phi, g,
                       two_dx, b, (double*)grav);
  else
    hipLaunchKernelGGL(k_gradient<float>, dim3(blocks_for(b.P)), dim3(kBlock), 0, s, phi, g,
                       two_dx, b, (float*)grav);
  return hipGetLastError() == hipSuccess ? NYX_OK : NYX_E_HIP;
}

}  // extern "C"
