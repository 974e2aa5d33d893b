/*
 * sync_oracle.c -- FP64 CPU reference of the synchronisation of two AMR
 * levels after the fine level has been advanced (Sec. 4.3 Multilevel
 * Algorithm, Steps 2 and 8): the coarse cells beside the fine level are
 * corrected by the difference between the fine and the coarse fluxes through
 * their shared faces, which keeps the sums over both levels conserved, and
 * each covered coarse cell takes the mean of its eight children.  TEST
 * INFRASTRUCTURE ONLY; shares no code with the HIP library.
 *
 * The coarse step moved conserved quantities through a coarse face with its
 * own flux over dt_c; the fine level moved them through the same face with
 * its fine fluxes over its substeps.  Reflux replaces the coarse transfer by
 * the fine one in the uncovered coarse cell next to the face:
 *   R = -dt_c F_c + sum_s (dt_f[s] / 4) (four fine faces' F summed),
 *   A += (+R for A's low face, -R for A's high face) / dx_c,
 * and average-down sets each covered coarse cell to the mean of its eight
 * children.  Sums run in the order written here.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int n[3], ng, lo[3];
  long off, P;
} Sbox;

static int wrapi(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

static long padded_idx(const Sbox* b, const int* l) { /* box-local valid/ghost indices */
  return ((long)(l[2] + b->ng) * (b->n[1] + 2 * b->ng) + (l[1] + b->ng)) * (b->n[0] + 2 * b->ng) +
         (l[0] + b->ng);
}

static void load(Sbox* bx, int nb, const int32_t* n3, const int32_t* lo3, const int64_t* off,
                 int ng) {
  for (int b = 0; b < nb; ++b) {
    for (int d = 0; d < 3; ++d) {
      bx[b].n[d] = n3[3 * b + d];
      bx[b].lo[d] = lo3[3 * b + d];
    }
    bx[b].ng = ng;
    bx[b].off = (long)off[b];
    bx[b].P = (long)(bx[b].n[0] + 2 * ng) * (bx[b].n[1] + 2 * ng) * (bx[b].n[2] + 2 * ng);
  }
}

static int contains(const Sbox* b, const int* g) {
  for (int d = 0; d < 3; ++d)
    if (g[d] < b->lo[d] || g[d] >= b->lo[d] + b->n[d]) return 0;
  return 1;
}

static int find_box(const Sbox* bx, int nb, const int* g) {
  for (int b = 0; b < nb; ++b)
    if (contains(&bx[b], g)) return b;
  return -1;
}

/* fine box holding the children of coarse cell C (global, wrapped), or -1 */
static int fine_owner(const Sbox* fb, int nf, const int* C) {
  const int ch[3] = {2 * C[0], 2 * C[1], 2 * C[2]};
  return find_box(fb, nf, ch);
}

/* offset of face (d, f[3]) (box-local; f[d] in [0, n_d]) and component c in
 * a box's face-flux block (layout of nyxo_hydro_step_faces) */
static long face_idx(const Sbox* b, int d, int c, const int* f) {
  long o = 0;
  for (int e = 0; e < d; ++e) {
    const long fe = (long)(b->n[0] + (e == 0)) * (b->n[1] + (e == 1)) * (b->n[2] + (e == 2));
    o += 6 * fe;
  }
  const int ex = b->n[0] + (d == 0), ey = b->n[1] + (d == 1), ez = b->n[2] + (d == 2);
  return o + (((long)c * ez + f[2]) * ey + f[1]) * ex + f[0];
}

int nyxo_reflux_average_down(int ncoarse, const int32_t* cn3, const int32_t* clo3,
                             const int64_t* coff, int cng, double cdx, double* cdata,
                             const double* cflux, const int64_t* cflux_off, double dt_c,
                             int nfine, const int32_t* fn3, const int32_t* flo3,
                             const int64_t* foff, int fng, const int32_t* dom,
                             const double* fdata, int nsub, const double* fflux,
                             const int64_t* fflux_off, int64_t fflux_sub_stride,
                             const double* dt_f, int ncomp, int64_t* n_faces,
                             int64_t* n_covered) {
  if (ncoarse < 1 || nfine < 1 || !cn3 || !clo3 || !coff || !cdata || !cflux || !cflux_off ||
      !fn3 || !flo3 || !foff || !dom || !fdata || nsub < 1 || !fflux || !fflux_off || !dt_f ||
      ncomp < 1 || ncomp > 6 || cng < 0 || fng < 0 || !(cdx > 0.0))
    return -1;
  for (int d = 0; d < 3; ++d)
    if (dom[d] < 2 || (dom[d] & 1)) return -1;
  Sbox* cb = (Sbox*)malloc(sizeof(Sbox) * (size_t)ncoarse);
  Sbox* fb = (Sbox*)malloc(sizeof(Sbox) * (size_t)nfine);
  load(cb, ncoarse, cn3, clo3, coff, cng);
  load(fb, nfine, fn3, flo3, foff, fng);
  int rc = 0;
  for (int b = 0; b < nfine; ++b)
    for (int d = 0; d < 3; ++d)
      if ((fb[b].lo[d] & 1) || (fb[b].n[d] & 1)) rc = -1;
  const int cdom[3] = {dom[0] / 2, dom[1] / 2, dom[2] / 2};
  long nface = 0, ncov = 0;

  /* reflux of every uncovered coarse cell next to a covered one */
  for (int c = 0; c < ncoarse && rc == 0; ++c) {
    const Sbox* B = &cb[c];
    int A[3];
    for (A[2] = 0; A[2] < B->n[2] && rc == 0; ++A[2])
      for (A[1] = 0; A[1] < B->n[1] && rc == 0; ++A[1])
        for (A[0] = 0; A[0] < B->n[0] && rc == 0; ++A[0]) {
          int Ag[3];
          for (int d = 0; d < 3; ++d) Ag[d] = B->lo[d] + A[d];
          if (fine_owner(fb, nfine, Ag) >= 0) continue; /* covered: averaged down */
          double delta[6] = {0, 0, 0, 0, 0, 0};
          int hit = 0;
          for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) { /* 0: low face of A, 1: high face */
              int Bg[3] = {Ag[0], Ag[1], Ag[2]};
              Bg[d] += side ? 1 : -1;
              for (int e = 0; e < 3; ++e) Bg[e] = wrapi(Bg[e], cdom[e]);
              const int f = fine_owner(fb, nfine, Bg);
              if (f < 0) continue;
              hit = 1;
              nface++;
              /* the coarse face in A's box */
              int cf[3] = {A[0], A[1], A[2]};
              cf[d] += side;
              /* the four fine faces: the children of B next to A */
              const Sbox* F = &fb[f];
              int ff[3];
              for (int e = 0; e < 3; ++e) ff[e] = 2 * Bg[e] - F->lo[e];
              if (!side) ff[d] += 2; /* B below A: the high faces of B's children */
              int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
              for (int v = 0; v < ncomp; ++v) {
                double r = 0.0;
                r = r + (-1.0 * dt_c) * cflux[cflux_off[c] + face_idx(B, d, v, cf)];
                for (int s = 0; s < nsub; ++s) {
                  const double* fl = fflux + (long)s * fflux_sub_stride + fflux_off[f];
                  double acc = 0.0;
                  for (int q = 0; q < 4; ++q) {
                    int g[3] = {ff[0], ff[1], ff[2]};
                    g[t1] += q & 1;
                    g[t2] += q >> 1;
                    const double x = fl[face_idx(F, d, v, g)];
                    acc = q == 0 ? x : acc + x;
                  }
                  r = r + (0.25 * dt_f[s]) * acc;
                }
                delta[v] = delta[v] + (side ? -r : r);
              }
            }
          if (!hit) continue;
          const long id = padded_idx(B, A);
          for (int v = 0; v < ncomp; ++v) {
            double* u = cdata + B->off + (long)v * B->P;
            u[id] = u[id] + delta[v] / cdx;
          }
        }
  }

  /* average-down of every covered coarse cell */
  for (int f = 0; f < nfine && rc == 0; ++f) {
    const Sbox* F = &fb[f];
    for (int k = 0; k < F->n[2] / 2 && rc == 0; ++k)
      for (int j = 0; j < F->n[1] / 2 && rc == 0; ++j)
        for (int i = 0; i < F->n[0] / 2 && rc == 0; ++i) {
          const int C[3] = {F->lo[0] / 2 + i, F->lo[1] / 2 + j, F->lo[2] / 2 + k};
          const int c = find_box(cb, ncoarse, C);
          if (c < 0) {
            rc = -2;
            break;
          }
          /* proper nesting: an uncovered face neighbour lies on the coarse level */
          for (int d = 0; d < 3 && rc == 0; ++d)
            for (int side = -1; side <= 1; side += 2) {
              int N[3] = {C[0], C[1], C[2]};
              N[d] = wrapi(N[d] + side, cdom[d]);
              if (fine_owner(fb, nfine, N) < 0 && find_box(cb, ncoarse, N) < 0) rc = -2;
            }
          if (rc) break;
          const Sbox* B = &cb[c];
          const int cl[3] = {C[0] - B->lo[0], C[1] - B->lo[1], C[2] - B->lo[2]};
          const long id = padded_idx(B, cl);
          for (int v = 0; v < ncomp; ++v) {
            const double* u = fdata + F->off + (long)v * F->P;
            double s = 0.0;
            for (int q = 0; q < 8; ++q) {
              const int l[3] = {2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2)};
              const double x = u[padded_idx(F, l)];
              s = q == 0 ? x : s + x;
            }
            cdata[B->off + (long)v * B->P + id] = 0.125 * s;
          }
          ncov++;
        }
  }
  if (n_faces) *n_faces = nface;
  if (n_covered) *n_covered = ncov;
  free(cb);
  free(fb);
  return rc;
}
