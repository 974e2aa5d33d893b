/*
 * mlp_oracle.c -- FP64 CPU reference of the learned Riemann-flux network:
 * input normalisation, forward pass, mean-squared loss and its gradient by
 * backpropagation.  TEST INFRASTRUCTURE ONLY (gradient oracle of the GPU
 * training kernels); shares no code with the HIP library.
 *
 * The network stands in for the two-shock Riemann solver of Sec. 3.2.  A
 * training sample is a face the solver itself resolved:
 *   raw[0..4]   left state  (rho, u_n, u_t1, u_t2, p)
 *   raw[5..9]   right state (rho, u_n, u_t1, u_t2, p)
 *   raw[10..14] solver result (p_star, u_star, rhostar_L, rhostar_R, and the
 *               density of the Godunov state)
 * Normalisation with c_K = sqrt(gamma p_K / rho_K), rbar = (rho_L + rho_R)/2,
 * cbar = (c_L + c_R)/2, ubar = (u_L + u_R)/2, Pbar = rbar cbar^2:
 *   x = (rho_L/rbar, (u_L-ubar)/cbar, v_L/cbar, w_L/cbar, p_L/Pbar,
 *        rho_R/rbar, (u_R-ubar)/cbar, v_R/cbar, w_R/cbar, p_R/Pbar)
 *   y = (ln(p_star/Pbar), (u_star-ubar)/cbar, ln(rhostar_L/rbar),
 *        ln(rhostar_R/rbar), ln(rho_g/rbar))
 * Network 10 -> 64 -> 64 -> 64 -> 5, ReLU on the hidden layers, linear
 * output.  Flat parameter vector (9349 values):
 *   W1[64][10], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[5][64], b4[5]
 * (W[o][i] multiplies input i into output o).
 * Loss L = (1/n) sum over in-domain samples of sum_outputs (yhat - y)^2
 * (a sample is in the training domain when its inputs and targets are finite
 * and at most 64 in magnitude; see nyxo_mlp_in_domain).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI 10
#define NH 64
#define NO 5
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH * NH)
#define OFF_W4 (OFF_B3 + NH)
#define OFF_B4 (OFF_W4 + NO * NH)
#define NPARAM (OFF_B4 + NO)

int nyxo_mlp_nparam(void) { return NPARAM; }

void nyxo_mlp_normalize(double gamma, const double* raw, long n, double* x, double* y) {
  for (long s = 0; s < n; ++s) {
    const double* r = raw + 15 * s;
    double rl = r[0], ul = r[1], vl = r[2], wl = r[3], pl = r[4];
    double rr = r[5], ur = r[6], vr = r[7], wr = r[8], pr = r[9];
    double cl = sqrt(gamma * pl / rl), cr = sqrt(gamma * pr / rr);
    double rbar = 0.5 * (rl + rr), cbar = 0.5 * (cl + cr), ubar = 0.5 * (ul + ur);
    double pbar = rbar * cbar * cbar;
    double* xs = x + NI * s;
    xs[0] = rl / rbar; xs[1] = (ul - ubar) / cbar; xs[2] = vl / cbar; xs[3] = wl / cbar;
    xs[4] = pl / pbar;
    xs[5] = rr / rbar; xs[6] = (ur - ubar) / cbar; xs[7] = vr / cbar; xs[8] = wr / cbar;
    xs[9] = pr / pbar;
    if (y) {
      double* ys = y + NO * s;
      ys[0] = log(r[10] / pbar);
      ys[1] = (r[11] - ubar) / cbar;
      ys[2] = log(r[12] / rbar);
      ys[3] = log(r[13] / rbar);
      ys[4] = log(r[14] / rbar);
    }
  }
}

/* dense layer: out[o] = b[o] + sum_i W[o][i] in[i] */
static void dense(const double* W, const double* b, int nin, int nout, const double* in,
                  double* out) {
  for (int o = 0; o < nout; ++o) {
    double acc = b[o];
    for (int i = 0; i < nin; ++i) acc += W[o * nin + i] * in[i];
    out[o] = acc;
  }
}

static void forward_one(const double* P, const double* x, double* z1, double* h1, double* z2,
                        double* h2, double* z3, double* h3, double* yhat) {
  dense(P + OFF_W1, P + OFF_B1, NI, NH, x, z1);
  for (int k = 0; k < NH; ++k) h1[k] = z1[k] > 0.0 ? z1[k] : 0.0;
  dense(P + OFF_W2, P + OFF_B2, NH, NH, h1, z2);
  for (int k = 0; k < NH; ++k) h2[k] = z2[k] > 0.0 ? z2[k] : 0.0;
  dense(P + OFF_W3, P + OFF_B3, NH, NH, h2, z3);
  for (int k = 0; k < NH; ++k) h3[k] = z3[k] > 0.0 ? z3[k] : 0.0;
  dense(P + OFF_W4, P + OFF_B4, NH, NO, h3, yhat);
}

void nyxo_mlp_forward(const double* P, const double* x, long n, double* yhat) {
  double z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH];
  for (long s = 0; s < n; ++s)
    forward_one(P, x + NI * s, z1, h1, z2, h2, z3, h3, yhat + NO * s);
}

/* a checksum of the ReLU activation pattern of the whole batch (for
 * finite-difference tests that must not cross a kink) */
uint64_t nyxo_mlp_relu_pattern(const double* P, const double* x, long n) {
  double z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], yh[NO];
  uint64_t hsh = 1469598103934665603ull;
  for (long s = 0; s < n; ++s) {
    forward_one(P, x + NI * s, z1, h1, z2, h2, z3, h3, yh);
    for (int k = 0; k < NH; ++k) {
      hsh = (hsh ^ (uint64_t)(z1[k] > 0.0)) * 1099511628211ull;
      hsh = (hsh ^ (uint64_t)(z2[k] > 0.0)) * 1099511628211ull;
      hsh = (hsh ^ (uint64_t)(z3[k] > 0.0)) * 1099511628211ull;
    }
  }
  return hsh;
}

/* loss and gradient over n samples; grad (NPARAM) is overwritten */
/* Training domain: a sample enters the loss only when its ten inputs and
 * five targets are finite and at most DOMAIN in magnitude (faces with floored
 * pressures or near-vacuum states normalise to huge values; the network is
 * not asked to fit them, and in a step they fall back to the two-shock
 * solver).  The loss stays normalised by the batch size n. */
#define DOMAIN 64.0
int nyxo_mlp_in_domain(const double* xs, const double* ys) {
  for (int k = 0; k < NI; ++k)
    if (!(fabs(xs[k]) <= DOMAIN)) return 0;
  for (int k = 0; k < NO; ++k)
    if (!(fabs(ys[k]) <= DOMAIN)) return 0;
  return 1;
}

double nyxo_mlp_loss_grad(const double* P, const double* x, const double* y, long n,
                          double* grad) {
  memset(grad, 0, sizeof(double) * NPARAM);
  double loss = 0.0;
  double z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], yh[NO];
  double d4[NO], d3[NH], d2[NH], d1[NH];
  for (long s = 0; s < n; ++s) {
    const double* xs = x + NI * s;
    const double* ys = y + NO * s;
    if (!nyxo_mlp_in_domain(xs, ys)) continue;
    forward_one(P, xs, z1, h1, z2, h2, z3, h3, yh);
    for (int o = 0; o < NO; ++o) {
      double e = yh[o] - ys[o];
      loss += e * e;
      d4[o] = 2.0 * e / (double)n;
    }
    /* output layer */
    for (int o = 0; o < NO; ++o) {
      grad[OFF_B4 + o] += d4[o];
      for (int i = 0; i < NH; ++i) grad[OFF_W4 + o * NH + i] += d4[o] * h3[i];
    }
    for (int i = 0; i < NH; ++i) {
      double acc = 0.0;
      for (int o = 0; o < NO; ++o) acc += P[OFF_W4 + o * NH + i] * d4[o];
      d3[i] = z3[i] > 0.0 ? acc : 0.0;
    }
    /* layer 3 */
    for (int o = 0; o < NH; ++o) {
      grad[OFF_B3 + o] += d3[o];
      for (int i = 0; i < NH; ++i) grad[OFF_W3 + o * NH + i] += d3[o] * h2[i];
    }
    for (int i = 0; i < NH; ++i) {
      double acc = 0.0;
      for (int o = 0; o < NH; ++o) acc += P[OFF_W3 + o * NH + i] * d3[o];
      d2[i] = z2[i] > 0.0 ? acc : 0.0;
    }
    /* layer 2 */
    for (int o = 0; o < NH; ++o) {
      grad[OFF_B2 + o] += d2[o];
      for (int i = 0; i < NH; ++i) grad[OFF_W2 + o * NH + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < NH; ++i) {
      double acc = 0.0;
      for (int o = 0; o < NH; ++o) acc += P[OFF_W2 + o * NH + i] * d2[o];
      d1[i] = z1[i] > 0.0 ? acc : 0.0;
    }
    /* layer 1 */
    for (int o = 0; o < NH; ++o) {
      grad[OFF_B1 + o] += d1[o];
      for (int i = 0; i < NI; ++i) grad[OFF_W1 + o * NI + i] += d1[o] * xs[i];
    }
  }
  return loss / (double)n;
}
