/*
 * gravity_oracle.c -- FP64 CPU reference of the mesh side of the gravity
 * input path (Sec. 2.4 and Sec. 3.4 Self-gravity).  TEST INFRASTRUCTURE
 * ONLY; shares no code with the HIP library.
 *
 * A periodic domain of dom[3] cells of size dx, cell (i, j, k) centred at
 * ((i + 1/2) dx, ...), fields stored x fastest without ghost cells.
 *
 *   - cloud-in-cell deposit: a particle's mass is spread uniformly over a
 *     cube of side dx centred at the particle; each cell receives the mass
 *     times the volume of its intersection with the cube over dx^3, divided
 *     by dx^3 (a comoving density).  Per axis the cube meets the cells
 *     i0 = floor(x / dx - 1/2) and i0 + 1 with fractions 1 - f and f,
 *     f = x / dx - 1/2 - i0.  Particles are taken in index order; the eight
 *     cells of one particle in the order (0,0,0), (1,0,0), (0,1,0), ...,
 *     x fastest.
 *   - centred gradient: g_d(c) = -(phi(c + e_d) - phi(c - e_d)) / (2 dx).
 *   - cloud-in-cell interpolation of a cell field to particle positions
 *     with the same weights (used by the pins only: together with the
 *     deposit and the centred gradient it makes a particle's force on
 *     itself vanish).
 * The Poisson solve itself is defined in the Python wrapper by the exact
 * solution of the discrete 7-point system (a library FFT).
 */
#include <math.h>
#include <stdint.h>

static long wrapl(long x, long m) {
  long r = x % m;
  return r < 0 ? r + m : r;
}

static long cidx(const int32_t* dom, long i, long j, long k) {
  return (wrapl(k, dom[2]) * dom[1] + wrapl(j, dom[1])) * dom[0] + wrapl(i, dom[0]);
}

/* lower cell and the fraction given to the upper one, per axis */
static void cic_axis(double x, double dx, long* i0, double* f) {
  const double s = x / dx - 0.5;
  const double fl = floor(s);
  *i0 = (long)fl;
  *f = s - fl;
}

int nyxo_cic_deposit(long np, const double* pos, const double* mass, const int32_t* dom,
                     double dx, double* rho) {
  if (np < 0 || !dom || !(dx > 0.0) || (np > 0 && (!pos || !mass)) || !rho) return -1;
  const double inv_vol = 1.0 / ((dx * dx) * dx);
  for (long p = 0; p < np; ++p) {
    long i0[3];
    double f[3];
    for (int d = 0; d < 3; ++d) cic_axis(pos[d * np + p], dx, &i0[d], &f[d]);
    const double m = mass[p] * inv_vol;
    for (int q = 0; q < 8; ++q) {
      const int b[3] = {q & 1, (q >> 1) & 1, q >> 2};
      double w = 1.0;
      for (int d = 0; d < 3; ++d) w = w * (b[d] ? f[d] : 1.0 - f[d]);
      rho[cidx(dom, i0[0] + b[0], i0[1] + b[1], i0[2] + b[2])] += m * w;
    }
  }
  return 0;
}

int nyxo_cic_interp(long np, const double* pos, const int32_t* dom, double dx,
                    const double* field, double* out) {
  if (np < 0 || !dom || !(dx > 0.0) || (np > 0 && (!pos || !field || !out))) return -1;
  for (long p = 0; p < np; ++p) {
    long i0[3];
    double f[3];
    for (int d = 0; d < 3; ++d) cic_axis(pos[d * np + p], dx, &i0[d], &f[d]);
    double v = 0.0;
    for (int q = 0; q < 8; ++q) {
      const int b[3] = {q & 1, (q >> 1) & 1, q >> 2};
      double w = 1.0;
      for (int d = 0; d < 3; ++d) w = w * (b[d] ? f[d] : 1.0 - f[d]);
      v = v + w * field[cidx(dom, i0[0] + b[0], i0[1] + b[1], i0[2] + b[2])];
    }
    out[p] = v;
  }
  return 0;
}

int nyxo_gradient(const int32_t* dom, double dx, const double* phi, double* g) {
  if (!dom || !(dx > 0.0) || !phi || !g) return -1;
  const long n = (long)dom[0] * dom[1] * dom[2];
  for (long k = 0; k < dom[2]; ++k)
    for (long j = 0; j < dom[1]; ++j)
      for (long i = 0; i < dom[0]; ++i) {
        const long c = cidx(dom, i, j, k);
        g[c] = -(phi[cidx(dom, i + 1, j, k)] - phi[cidx(dom, i - 1, j, k)]) / (2.0 * dx);
        g[n + c] = -(phi[cidx(dom, i, j + 1, k)] - phi[cidx(dom, i, j - 1, k)]) / (2.0 * dx);
        g[2 * n + c] = -(phi[cidx(dom, i, j, k + 1)] - phi[cidx(dom, i, j, k - 1)]) / (2.0 * dx);
      }
  return 0;
}
