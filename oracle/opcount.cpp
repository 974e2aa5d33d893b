// opcount.cpp -- operation-count build of the step oracle (TEST AND
// MEASUREMENT INFRASTRUCTURE ONLY; see nyx_oracle.c).
//
// nyx_oracle.c is compiled here unchanged, as C++, with `double` replaced by a
// counting number type.  Every +, -, *, / and sqrt the oracle evaluates is
// counted against the stage marked by NYXO_STAGE and, inside the two-shock
// solver, against its Newton iterations (NYXO_ITER).  Comparisons, fabs,
// min/max and selects are counted separately and are not flops.  The values
// computed are the oracle's own (the type carries an IEEE double and does the
// same operation), so the counts are those of the published algorithm as the
// oracle evaluates it, on the caller's data.
//
// Stages: 1 primitives (O1), 2 flattening (O2), 3 PPM + tracing (O3, O4),
// 4 stage-0 Riemann (O5, O6), 5 stage-1 corrections + Riemann (O7, O5),
// 6 stage-2 corrections + Riemann (O7, O5, O9), 7 update, corrector, sync
// (O10-O12), 8 CFL (O13).
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

namespace opc {
enum { kAdd = 0, kMul, kDiv, kSqrt, kCmp, kNops };
constexpr int kStages = 9;
static long long counts[kStages][2][kNops];
static int stage = 0;
static int iter = 0;
static inline void tick(int op) { counts[stage][iter][op]++; }
}  // namespace opc

struct cdouble {
  double v;
  cdouble() = default;
  cdouble(double x) : v(x) {}  // NOLINT: implicit from literals and ints
  cdouble& operator+=(cdouble o) { opc::tick(opc::kAdd); v += o.v; return *this; }
  cdouble& operator-=(cdouble o) { opc::tick(opc::kAdd); v -= o.v; return *this; }
  cdouble& operator*=(cdouble o) { opc::tick(opc::kMul); v *= o.v; return *this; }
  cdouble& operator/=(cdouble o) { opc::tick(opc::kDiv); v /= o.v; return *this; }
  cdouble operator-() const { return cdouble(-v); }
  explicit operator long() const { return (long)v; }
  explicit operator int() const { return (int)v; }
};
static inline cdouble operator+(cdouble a, cdouble b) { opc::tick(opc::kAdd); return cdouble(a.v + b.v); }
static inline cdouble operator-(cdouble a, cdouble b) { opc::tick(opc::kAdd); return cdouble(a.v - b.v); }
static inline cdouble operator*(cdouble a, cdouble b) { opc::tick(opc::kMul); return cdouble(a.v * b.v); }
static inline cdouble operator/(cdouble a, cdouble b) { opc::tick(opc::kDiv); return cdouble(a.v / b.v); }
static inline bool operator<(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v < b.v; }
static inline bool operator>(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v > b.v; }
static inline bool operator<=(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v <= b.v; }
static inline bool operator>=(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v >= b.v; }
static inline bool operator==(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v == b.v; }
static inline bool operator!=(cdouble a, cdouble b) { opc::tick(opc::kCmp); return a.v != b.v; }
static inline cdouble sqrt(cdouble a) { opc::tick(opc::kSqrt); return cdouble(std::sqrt(a.v)); }
static inline cdouble fabs(cdouble a) { return cdouble(std::fabs(a.v)); }
static inline bool isfinite(cdouble a) { return std::isfinite(a.v); }

#define NYXO_STAGE(s) (opc::stage = (s))
#define NYXO_ITER(on) (opc::iter = (on))
#define double cdouble
#include "nyx_oracle.c"
#undef double

extern "C" {

// Counts of the last calls since nyxo_opcount_reset: out[stage][iter][op],
// stage 0..8, iter 0 (outside) / 1 (inside a Newton iteration), op = add/sub,
// mul, div, sqrt, comparison.
void nyxo_opcount_reset(void) {
  std::memset(opc::counts, 0, sizeof opc::counts);
  opc::stage = 0;
  opc::iter = 0;
}
void nyxo_opcount_read(long long* out) {
  std::memcpy(out, opc::counts, sizeof opc::counts);
}

// The step and the CFL estimate on plain double arrays; same arguments and
// results as nyxo_hydro_step / nyxo_estimate_dt.
int nyxo_opcount_step(const void* prm_in, int nx, int ny, int nz, int ng, const double* Uin,
                      const double* grav, double dt, double dx, double a_old, double a_new,
                      double* Uout, long long* stats8) {
  static_assert(sizeof(cdouble) == sizeof(double), "cdouble must be one double");
  const struct {
    double gamma, eta, small_dens, small_pres, riemann_tol;
    int32_t riemann_maxiter, recon, riemann, grav_form;
  }* in = static_cast<const decltype(in)>(prm_in);
  nyxo_params prm;
  prm.gamma = in->gamma;
  prm.eta = in->eta;
  prm.small_dens = in->small_dens;
  prm.small_pres = in->small_pres;
  prm.riemann_tol = in->riemann_tol;
  prm.riemann_maxiter = in->riemann_maxiter;
  prm.recon = in->recon;
  prm.riemann = in->riemann;
  prm.grav_form = in->grav_form;
  nyxo_stats st;
  std::memset(&st, 0, sizeof st);
  const int rc = nyxo_hydro_step(&prm, nx, ny, nz, ng, reinterpret_cast<const cdouble*>(Uin),
                                 reinterpret_cast<const cdouble*>(grav), dt, dx, a_old, a_new,
                                 reinterpret_cast<cdouble*>(Uout), &st);
  opc::stage = 0;
  if (stats8) {
    const int64_t* f = &st.nonfinite;
    for (int i = 0; i < 8; ++i) stats8[i] = f[i];
  }
  return rc;
}

int nyxo_opcount_dt(const void* prm_in, int nx, int ny, int nz, int ng, const double* state,
                    double a, double dx, double cfl, double* dt_out) {
  const struct {
    double gamma, eta, small_dens, small_pres, riemann_tol;
    int32_t riemann_maxiter, recon, riemann, grav_form;
  }* in = static_cast<const decltype(in)>(prm_in);
  nyxo_params prm;
  prm.gamma = in->gamma;
  prm.eta = in->eta;
  prm.small_dens = in->small_dens;
  prm.small_pres = in->small_pres;
  prm.riemann_tol = in->riemann_tol;
  prm.riemann_maxiter = in->riemann_maxiter;
  prm.recon = in->recon;
  prm.riemann = in->riemann;
  prm.grav_form = in->grav_form;
  cdouble dt;
  const int rc = nyxo_estimate_dt(&prm, nx, ny, nz, ng, reinterpret_cast<const cdouble*>(state),
                                  a, dx, cfl, &dt);
  opc::stage = 0;
  *dt_out = dt.v;
  return rc;
}

}  // extern "C"
