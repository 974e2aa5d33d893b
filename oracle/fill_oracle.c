/*
 * fill_oracle.c -- FP64 CPU reference of the ghost-cell fill of one AMR
 * level (Sec. 4.1 Mesh Hierarchy: each grid carries ghost cells that hold
 * data for the update of its valid cells; its regrid procedure: data in newly
 * refined regions are interpolated from the coarser level with limited
 * piecewise linear profiles whose values at the fine cell centres conserve
 * the coarse averages).  TEST INFRASTRUCTURE ONLY; shares no code with the
 * HIP library.
 *
 * A level is nbox boxes of one cell size in a periodic domain of dom[3]
 * cells.  Box b has n[3] valid cells, ng ghost cells and its valid cell
 * (0,0,0) at global index lo[3*b..]; its data are ncomp components in the
 * padded layout of the step (component-major, x fastest) at element offset
 * off[b] with component stride P_b (the padded cell count).
 *
 * Every ghost cell x of every box (global index, wrapped into the domain):
 *   1. if a box of the same level has x among its valid cells, its value is
 *      copied;
 *   2. otherwise the coarse level (refinement ratio 2, domain dom/2) must have
 *      the coarse cell X = floor(x / 2) among the valid cells of one of its
 *      boxes, whose ghost cells are already filled; the value is the
 *      limited linear profile of that coarse cell at the fine cell centre:
 *        s_d = MC-limited centred difference of U(X -/+ e_d) and U(X),
 *        alpha = the largest factor in [0, 1] that keeps all eight children
 *                U(X) + alpha sum_d (+/- s_d / 4) inside [min, max] of U
 *                over X and its six face neighbours,
 *        U_fine = U(X) + alpha sum_d o_d s_d, o_d = -1/4 for an even fine
 *                 index in d (the low child), +1/4 for an odd one;
 *      the eight children average to U(X) (conservation);
 *   3. no other case exists for properly nested levels; the function then
 *      returns -2.
 * Valid cells are never written.
 *
 * Subcycling (Sec. 4.2): when the fine level takes several steps per coarse
 * step, its ghost cells at an intermediate time take the coarse data
 * interpolated linearly in time, U_c = U_old + theta (U_new - U_old) for
 * every coarse value the profile reads (nyxo_fill_level_time; theta in
 * [0, 1] is the fine time's fraction of the coarse step).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "nyx_oracle.h"

typedef struct {
  int n[3], ng, lo[3];
  long off, P;
} Lbox;

static int wrap(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

static long padded(const Lbox* b, int i, int j, int k) { /* i, j, k box-local, may be ghosts */
  return ((long)(k + b->ng) * (b->n[1] + 2 * b->ng) + (j + b->ng)) * (b->n[0] + 2 * b->ng) +
         (i + b->ng);
}

/* box whose valid region holds the (wrapped) global cell g, or -1 */
static int owner(const Lbox* bx, int nbox, const int* g) {
  for (int b = 0; b < nbox; ++b) {
    int in = 1;
    for (int d = 0; d < 3; ++d) in = in && g[d] >= bx[b].lo[d] && g[d] < bx[b].lo[d] + bx[b].n[d];
    if (in) return b;
  }
  return -1;
}

static void load_boxes(Lbox* bx, int nbox, const int32_t* n3, int ng, const int32_t* lo3,
                       const int64_t* off) {
  for (int b = 0; b < nbox; ++b) {
    for (int d = 0; d < 3; ++d) {
      bx[b].n[d] = n3[3 * b + d];
      bx[b].lo[d] = lo3[3 * b + d];
    }
    bx[b].ng = ng;
    bx[b].off = (long)off[b];
    bx[b].P = (long)(bx[b].n[0] + 2 * ng) * (bx[b].n[1] + 2 * ng) * (bx[b].n[2] + 2 * ng);
  }
}

static double mc_slope(double um, double u0, double up) {
  double dp = up - u0, dm = u0 - um;
  double c = 0.5 * (dp + dm);
  if (dp * dm > 0.0) {
    double m = fabs(c);
    m = fmin(m, 2.0 * fabs(dp));
    m = fmin(m, 2.0 * fabs(dm));
    return c > 0.0 ? m : -m;
  }
  return 0.0;
}

/* coarse value at padded index i: the old data, or the old and new data
 * interpolated in time */
static double cval(const double* uo, const double* un, double theta, long i) {
  return un ? uo[i] + theta * (un[i] - uo[i]) : uo[i];
}

/* limited linear value of coarse cell (I, J, K) (local to coarse box cb) at
 * the fine child with parities par[3] (0 = low child), component c */
static double interp(const Lbox* cb, const double* cdata, const double* cnew, double theta,
                     int c, int I, int J, int K, const int* par) {
  const double* u = cdata + cb->off + (long)c * cb->P;
  const double* un = cnew ? cnew + cb->off + (long)c * cb->P : NULL;
  const double u0 = cval(u, un, theta, padded(cb, I, J, K));
  double s[3], lo = u0, hi = u0;
  for (int d = 0; d < 3; ++d) {
    int cm[3] = {I, J, K}, cp[3] = {I, J, K};
    cm[d] -= 1;
    cp[d] += 1;
    double um = cval(u, un, theta, padded(cb, cm[0], cm[1], cm[2]));
    double up = cval(u, un, theta, padded(cb, cp[0], cp[1], cp[2]));
    s[d] = mc_slope(um, u0, up);
    lo = fmin(lo, fmin(um, up));
    hi = fmax(hi, fmax(um, up));
  }
  /* the children's largest excursion is (|s_x| + |s_y| + |s_z|) / 4 on each side */
  double ext = 0.25 * ((fabs(s[0]) + fabs(s[1])) + fabs(s[2]));
  double alpha = 1.0;
  if (ext > 0.0) {
    if (u0 + ext > hi) alpha = fmin(alpha, (hi - u0) / ext);
    if (u0 - ext < lo) alpha = fmin(alpha, (u0 - lo) / ext);
  }
  double v = 0.0;
  for (int d = 0; d < 3; ++d) v = v + (par[d] ? 0.25 : -0.25) * s[d];
  return u0 + alpha * v;
}

/* Fill the ghost cells of every fine box.  Returns 0, -1 on bad arguments,
 * -2 when a ghost cell is neither covered by the level nor by the coarse
 * level's valid cells (ncoarse = 0: no coarse level). */
int nyxo_fill_level(int nbox, const int32_t* n3, const int32_t* lo3, const int64_t* off, int ng,
                    const int32_t* dom, int ncomp, double* data, int ncoarse,
                    const int32_t* cn3, const int32_t* clo3, const int64_t* coff, int cng,
                    const double* cdata, int64_t* n_copied, int64_t* n_interp) {
  return nyxo_fill_level_time(nbox, n3, lo3, off, ng, dom, ncomp, data, ncoarse, cn3, clo3, coff,
                              cng, cdata, NULL, 0.0, n_copied, n_interp);
}

int nyxo_fill_level_time(int nbox, const int32_t* n3, const int32_t* lo3, const int64_t* off,
                         int ng, const int32_t* dom, int ncomp, double* data, int ncoarse,
                         const int32_t* cn3, const int32_t* clo3, const int64_t* coff, int cng,
                         const double* cdata, const double* cdata_new, double theta,
                         int64_t* n_copied, int64_t* n_interp) {
  if (cdata_new && !(theta >= 0.0 && theta <= 1.0)) return -1;
  if (nbox < 1 || !n3 || !lo3 || !off || !dom || !data || ng < 1 || ncomp < 1) return -1;
  for (int d = 0; d < 3; ++d)
    if (dom[d] < 2 || (dom[d] & 1)) return -1;
  if (ncoarse > 0 && (!cn3 || !clo3 || !coff || !cdata || cng < 1)) return -1;
  Lbox* bx = (Lbox*)malloc(sizeof(Lbox) * (size_t)nbox);
  Lbox* cbx = ncoarse > 0 ? (Lbox*)malloc(sizeof(Lbox) * (size_t)ncoarse) : NULL;
  load_boxes(bx, nbox, n3, ng, lo3, off);
  if (ncoarse > 0) load_boxes(cbx, ncoarse, cn3, cng, clo3, coff);
  const int cdom[3] = {dom[0] / 2, dom[1] / 2, dom[2] / 2};
  long nc = 0, ni = 0;
  int rc = 0;
  for (int b = 0; b < nbox && rc == 0; ++b) {
    const Lbox* B = &bx[b];
    for (int k = -ng; k < B->n[2] + ng && rc == 0; ++k)
      for (int j = -ng; j < B->n[1] + ng && rc == 0; ++j)
        for (int i = -ng; i < B->n[0] + ng && rc == 0; ++i) {
          if (i >= 0 && i < B->n[0] && j >= 0 && j < B->n[1] && k >= 0 && k < B->n[2]) continue;
          const int loc[3] = {i, j, k};
          int g[3];
          for (int d = 0; d < 3; ++d) g[d] = wrap(B->lo[d] + loc[d], dom[d]);
          long dst = padded(B, i, j, k);
          int s = owner(bx, nbox, g);
          if (s >= 0) {
            const Lbox* S = &bx[s];
            long src = padded(S, g[0] - S->lo[0], g[1] - S->lo[1], g[2] - S->lo[2]);
            for (int c = 0; c < ncomp; ++c)
              data[B->off + (long)c * B->P + dst] = data[S->off + (long)c * S->P + src];
            nc++;
            continue;
          }
          int G[3], par[3];
          for (int d = 0; d < 3; ++d) {
            G[d] = wrap(g[d] / 2, cdom[d]);
            par[d] = g[d] & 1;
          }
          int cbi = ncoarse > 0 ? owner(cbx, ncoarse, G) : -1;
          if (cbi < 0) {
            rc = -2;
            break;
          }
          const Lbox* C = &cbx[cbi];
          for (int c = 0; c < ncomp; ++c)
            data[B->off + (long)c * B->P + dst] =
                interp(C, cdata, cdata_new, theta, c, G[0] - C->lo[0], G[1] - C->lo[1],
                       G[2] - C->lo[2], par);
          ni++;
        }
  }
  if (n_copied) *n_copied = nc;
  if (n_interp) *n_interp = ni;
  free(bx);
  free(cbx);
  return rc;
}
