/*
 * nyx_oracle.h -- plain, slow FP64 CPU oracle of the comoving unsplit PPM
 * Godunov gas step (Almgren et al., "Nyx", Sec. 3.2 Gas Dynamics, Sec. 3.5
 * Computing the time step, Sec. 3.6 Single-Level Integration Algorithm,
 * Steps 2 and 6).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the HIP path
 * against an obviously correct implementation.  It shares no code, header,
 * table or constant with the HIP library and must never be linked into or
 * called from the product path.
 *
 * Layout of every 3-D field: a box of n = (nx, ny, nz) valid cells surrounded
 * by ng ghost cells on each side; component-major, x fastest:
 *   idx(c, k, j, i) = ((c*(nz+2ng) + k+ng)*(ny+2ng) + j+ng)*(nx+2ng) + i+ng
 * for i in [-ng, nx+ng), etc.  State components (Sec. 3.2):
 *   0: rho, 1..3: a*rho*U_{x,y,z}, 4: a^2*rho*E, 5: a^2*rho*e.
 * Gravity: 3 components g_{x,y,z} in the same padded layout.
 * All arrays are host memory owned by the caller.
 */
#ifndef NYX_ORACLE_H
#define NYX_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Scheme variants that Sec. 3.2 describes. */
#define NYXO_RECON_PPM 0        /* unsplit piecewise parabolic reconstruction */
#define NYXO_RECON_PLM 1        /* unsplit piecewise linear reconstruction */
#define NYXO_RIEMANN_TWOSHOCK 0 /* iterative two-shock solver (Colella & Glaz) */
#define NYXO_RIEMANN_LINEAR 1   /* linearised (acoustic) approximate solver */

typedef struct {
  double gamma;        /* gamma-law EOS exponent (Sec. 2.2: 5/3); any other value
                        * turns on the expansion term of the energy equations */
  double eta;          /* dual-energy threshold (Sec. 3.6, Step 6: 1e-4) */
  double small_dens;   /* density floor, primitives and edge states only */
  double small_pres;   /* pressure floor, primitives, edge states, Riemann */
  double riemann_tol;  /* relative stopping tolerance of the two-shock iteration */
  int32_t riemann_maxiter;
  int32_t recon;       /* NYXO_RECON_* */
  int32_t riemann;     /* NYXO_RIEMANN_* */
  int32_t grav_form;   /* energy gravity term (Sec. 3.2): 1 = (rho U).g at cell
                        * centres, 2 = the update of E is the update of the
                        * kinetic energy from the gravity momentum update */
} nyxo_params;

typedef struct {
  int64_t nonfinite;      /* valid output cells with a non-finite component */
  int64_t neg_dens;       /* valid output cells with rho <= 0 */
  int64_t neg_eint;       /* valid output cells with a^2 rho e <= 0 */
  int64_t floor_hits;     /* individual floor applications (O1, O4) */
  int64_t trans_reverts;  /* transverse corrections rejected (O7) */
  int64_t sync_E_from_e;  /* cells where E was rebuilt from e (Step 6) */
  int64_t riemann_iters;  /* total two-shock iterations */
  int64_t riemann_calls;  /* total Riemann solves */
} nyxo_stats;

/* Hydro CFL (Sec. 3.5): dt = cfl * a * dx / max_{cells,d}(|U_d| + c).
 * Returns 0, or -1 on bad arguments. */
int nyxo_estimate_dt(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                     const double* state, double a, double dx, double cfl,
                     double* dt_out);

/* One gas step (Sec. 3.6, Step 2 predictor with S_g^n and S_e, then the Step 6
 * gravity corrector with the same g and the dual-energy sync).  Input state is
 * scaled with a_old, output with a_new.  Only valid cells of state_out are
 * written.  Returns 0, or -1 on bad arguments / allocation failure. */
int nyxo_hydro_step(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                    const double* state_in, const double* grav, double dt,
                    double dx, double a_old, double a_new, double* state_out,
                    nyxo_stats* stats);

/* The same step; face_flux (or NULL) also receives the final comoving fluxes
 * F = (f_rho / a_h, f_m, a_h f_E, a_h f_e) of every face of the box (Sec. 3.2
 * flux vector), the values the update differences: for d = 0, 1, 2 in turn a
 * block of 6 components, each (nz + [d==2]) x (ny + [d==1]) x (nx + [d==0])
 * faces, x fastest; face index f along d is the low face of cell f. */
int nyxo_hydro_step_faces(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                          const double* state_in, const double* grav, double dt,
                          double dx, double a_old, double a_new, double* state_out,
                          nyxo_stats* stats, double* face_flux);

/* Synchronisation of two levels after the fine level's substeps (Sec. 4.3,
 * Steps 2 and 8): explicit reflux of the coarse cells next to the fine
 * level's boundary, then average-down of the covered coarse cells.
 * Coarse level: ncoarse boxes (cn3, clo3, coff, cng as in nyxo_fill_level),
 * cell size cdx, its step's face fluxes cflux (per box at cflux_off[b], the
 * layout of nyxo_hydro_step_faces) over dt_c.  Fine level (ratio 2, domain
 * dom, coarse domain dom/2): nfine boxes whose lo and n are even, data fdata
 * after its nsub substeps, whose face fluxes are fflux + s * fflux_sub_stride
 * (per box at fflux_off[b]) over dt_f[s].
 * A coarse cell is covered when its eight children lie in a fine box.  For
 * every valid coarse cell A that is not covered and each of its faces (x-,
 * x+, y-, y+, z-, z+ in that order) whose other side B is covered (periodic
 * images included):
 *   R = -dt_c F_c + sum_s (dt_f[s] / 4) (sum of the four fine faces' F)
 * with F_c the face's flux in A's own box; then A += (sum over its faces of
 * -/+ R) / cdx, the sign + when the face is A's low face.  Then every
 * covered coarse cell becomes the mean of its eight children.  ncomp
 * components.  Returns 0, -1 on bad arguments, -2 when a covered cell or an
 * uncovered neighbour of one lies in no coarse box. */
int nyxo_reflux_average_down(int ncoarse, const int32_t* cn3, const int32_t* clo3,
                             const int64_t* coff, int cng, double cdx, double* cdata,
                             const double* cflux, const int64_t* cflux_off, double dt_c,
                             int nfine, const int32_t* fn3, const int32_t* flo3,
                             const int64_t* foff, int fng, const int32_t* dom,
                             const double* fdata, int nsub, const double* fflux,
                             const int64_t* fflux_off, int64_t fflux_sub_stride,
                             const double* dt_f, int ncomp, int64_t* n_faces,
                             int64_t* n_covered);

/* ---- unit-level entry points used by the oracle's own pins ---- */

/* Two-shock Riemann solve on rotated primitive states (rho, u_n, u_t1, u_t2, p).
 * qg: Godunov state at xi = 0 in the same order.
 * star: {p*, u*, rho*_L, rho*_R}.  *iters: iterations taken. */
void nyxo_riemann(const nyxo_params* prm, const double* qL, const double* qR,
                  double* qg, double* star, int* iters);

/* PPM on a line of m cells: for j in [2, m-3], writes the flattened and
 * monotonized edge values qm[j] (at j-1/2) and qp[j] (at j+1/2); chi[j] is the
 * flattening coefficient of cell j.  Other entries are left untouched. */
void nyxo_ppm_line(int m, const double* q, const double* chi, double* qm,
                   double* qp);
/* O3 variant: PLM edge values (q_j -/+ chi s_j / 2, s_j the limited centred
 * slope) of cells 2..m-3 of a line, same layout as nyxo_ppm_line. */
void nyxo_plm_line(int m, const double* q, const double* chi, double* qm, double* qp);

/* Unflattened fourth-order interface value between cells j and j+1 from
 * q[j-1..j+2] with van Leer-limited slopes (q points at q[j-1]). */
double nyxo_ppm_interface(const double* q4);

/* Directional flattening coefficient chi_d on a line of m cells for
 * j in [3, m-4]; others untouched. */
/* The step's flattening coefficient chi (the minimum over the three
 * directions of chi_d, from the primitives of the state at scale factor a)
 * on the cells of [-1, n]^3: chi_out holds (nz+2)(ny+2)(nx+2) values, x
 * fastest.  Returns 0, or -1 on bad arguments / allocation failure. */
int nyxo_flattening(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                    const double* state, double a, double* chi_out);
void nyxo_flatten_line(const nyxo_params* prm, int m, const double* p,
                       const double* u, double* chi);

/* Characteristic tracing of one cell in direction d (0, 1, 2).
 * qc: cell primitives (rho, ux, uy, uz, p); cc: sound speed;
 * qmv, qpv: PPM edge values (5 each, already flattened/monotonized);
 * g: cell gravity (3); kh = dt/(a_h dx); hdt_a = (dt/2)/a_h;
 * hda_a = (da/2)/a_h; pexp = 1.5(gamma-1) da/a_h.
 * Outputs lab-frame edge states: lo = left-face state (R input of face j-1/2),
 * hi = right-face state (L input of face j+1/2).  Returns floors applied. */
int nyxo_trace_cell(const nyxo_params* prm, int d, const double* qc, double cc,
                    const double* qmv, const double* qpv, const double* g,
                    double kh, double hdt_a, double hda_a, double pexp,
                    double* lo, double* hi);

/* Ghost fill of one AMR level (fill_oracle.c; Sec. 4.1, ghost cells and regridding): ghost
 * cells covered by a valid cell of the level are copied; the others take the
 * limited linear profile of the coarse level (ratio 2) at the fine cell
 * centre.  n3/lo3: 3 ints per box (valid extents, global index of valid cell
 * (0,0,0)); off: element offset of each box's padded data (component stride
 * = its padded cell count); dom: periodic domain in fine cells (even).  The
 * coarse arrays follow the same conventions (ncoarse = 0: none; the coarse
 * ghosts must be filled).  Returns 0, -1 (bad arguments), or -2 (a ghost
 * cell covered by neither level); counts the copied and interpolated cells. */
int nyxo_fill_level(int nbox, const int32_t* n3, const int32_t* lo3, const int64_t* off, int ng,
                    const int32_t* dom, int ncomp, double* data, int ncoarse,
                    const int32_t* cn3, const int32_t* clo3, const int64_t* coff, int cng,
                    const double* cdata, int64_t* n_copied, int64_t* n_interp);

/* The same fill at an intermediate time of a subcycled fine level (Sec.
 * 4.2): every coarse value the interpolation reads is cdata + theta
 * (cdata_new - cdata), theta in [0, 1] (cdata_new = NULL: cdata alone). */
int nyxo_fill_level_time(int nbox, const int32_t* n3, const int32_t* lo3, const int64_t* off,
                         int ng, const int32_t* dom, int ncomp, double* data, int ncoarse,
                         const int32_t* cn3, const int32_t* clo3, const int64_t* coff, int cng,
                         const double* cdata, const double* cdata_new, double theta,
                         int64_t* n_copied, int64_t* n_interp);

#ifdef __cplusplus
}
#endif
#endif
