/*
 * CFNEB oracle: plain, slow, FP64 CPU reference of one cell-filter NEB band step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this code: it exists so that tests, the smoke check and the
 * CPU-baseline leg of the benchmark can check the HIP library against an
 * independent implementation written from the paper.  It shares no code,
 * header, table or constant with the HIP library.
 *
 * Paper: Jia, Shi, Sun, "Scalable cell filter nudged elastic band (CFNEB) for
 * large-scale transition-path calculations", arXiv:2510.16721.
 *
 * What each part follows (section / equation of the paper):
 *   - strain convention h' = h (I + eps), lattice vectors as rows:   Sec. II.B, Eq. (2)
 *   - per-atom energy decomposition U = sum_i U_i(r^{ij}):           Sec. II.B, Eq. (4)
 *   - pair force f^{ij} = dU_i/dr^{ij} - dU_j/dr^{ji}:                Sec. II.B, Eq. (5) as used
 *                                                                    in the derivation of Eq. (6)
 *   - virial V = -1/2 sum r^{ij} (x) f^{ij}:                          Sec. II.B, Eqs. (6)-(8)
 *   - deformation gradient D = h0^-1 h, R~ = R D^-1:                  Sec. II.C, Eqs. (10)-(11)
 *   - rotation-free filter B = D D^T, lattice force D^-T V D^-1:      Sec. II.C, Eqs. (15)-(17)
 *   - D-variant filter, coordinates D, lattice force D^-T V:          Sec. II.C, Eqs. (11)-(14)
 *   - applied anisotropic stress (a constant second Piola-Kirchhoff
 *     stress referred to h0; non-hydrostatic loading is named in
 *     Sec. I as the reason for finite-deformation NEB):              a reading, not in the paper
 *   - NEB force = perpendicular true force + spring:                  Sec. II.A, Eq. (1)
 *   - improved tangent / climbing image (cited by the paper,
 *     Henkelman & Jonsson 2000; Henkelman, Uberuaga & Jonsson 2000)   Sec. I / II.A
 *   - adaptive insertion / deletion of images after each iteration:   Sec. III
 *   - FIRE (Bitzek et al. 2006), the usual optimizer of the band:     Sec. II.C / III
 *   - energy profile, enthalpy against the normalized path
 *     coordinate, as the transitions are reported (Hermite
 *     interpolant with tangential-force slopes):                     Sec. III figures
 *
 * Parity pins: every function is pinned by a CPU test against finite
 * differences, brute force, closed forms or invariants (tests/test_oracle_*.py).
 * The path shape between images and the number of steps to converge depend on
 * readings of the paper (cell factor, the factor 1/2 on the B force, FIRE
 * parameters, the refine rule) and are "parity unpinned" beyond the fixed
 * points (saddle, barrier) that the tests pin.
 */
#ifndef CFNEB_ORACLE_H
#define CFNEB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LJ = 1, ORC_TERSOFF = 2 };

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ECELL = -4,
    ORC_ENEIGH = -5,
    ORC_ENONFINITE = -6,
    ORC_ERANGE = -8
};

/* Parameters of a band run.  Units: eV, Angstrom, GPa. */
typedef struct orc_params {
    int potential;           /* ORC_LJ or ORC_TERSOFF */
    /* Lennard-Jones, energy-shifted at the cutoff */
    double lj_eps, lj_sigma, lj_rc;
    int lj_shift;
    /* Tersoff form (bond order, lambda3 = 0) */
    double ts_A, ts_B, ts_lambda1, ts_lambda2, ts_beta, ts_n, ts_c, ts_d, ts_h, ts_R, ts_S;
    /* band */
    int n_images;            /* images including both fixed endpoints */
    int max_images, min_images;
    double k_spring;         /* eV / A^2 */
    int climb_after;         /* climbing image from this step index on; <0 never */
    int cell_filter;         /* 0: cell fixed; 1: D-variant; 2: rotation-free filter */
    double cell_factor;      /* c_f; <= 0 means |det h0|^(1/3) n^(1/6) */
    double b_force_scale;    /* multiplies the printed lattice force D^-T V D^-1 */
    double pressure_GPa;     /* hydrostatic pressure, enthalpy H = U + P Omega */
    /* FIRE */
    double fire_dt0, fire_dtmax, fire_maxstep;
    int fire_nmin;
    double fire_finc, fire_fdec, fire_astart, fire_fa;
    /* adaptive images */
    int refine_every;        /* 0 = off */
    int ins_num, ins_den, del_num, del_den;
    /* applied stress beyond the pressure: a constant second Piola-Kirchhoff stress S
       (Voigt xx yy zz yz xz xy, GPa, tensile positive) referred to h0; the enthalpy
       gains -Omega0 S : E with E = (D D^T - I)/2 and Omega0 = |det h0| */
    double stress_GPa[6];
} orc_params;

/* ---------------- 3x3 geometry (row-major, lattice vectors are rows) ---- */
double orc_det3(const double* A);
void   orc_inv3(const double* A, double* Ainv);
/* D = symmetric positive square root of sym(B).  Returns ORC_ECELL if sym(B) is
 * not positive definite. */
int    orc_symsqrt(const double* B, double* D);
/* Perpendicular widths of the cell (distance between opposite faces). */
void   orc_widths(const double* h, double* w);

/* ---------------- neighbour sets --------------------------------------- */
/* Every (j, n) with n in Z^3, (j, n) != (i, 0), and
 *   r = (R_j - R_i) + ((n0 h_0 + n1 h_1) + n2 h_2),   r.r < rc*rc
 * with each operation rounded separately.  Output per atom i: cnt[i] entries,
 * stored at ent[4*(off_i + e)] = (j, n0, n1, n2), sorted by (j, n0, n1, n2),
 * where off_i = sum_{i'<i} cnt[i'].  Returns the total number of entries, or a
 * negative code if it exceeds cap_total (cnt[] is still filled). */
int64_t orc_nlist_brute(int n, const double* R, const double* h, double rc,
                        int32_t* cnt, int32_t* ent, int64_t cap_total);
int64_t orc_nlist_cells(int n, const double* R, const double* h, double rc,
                        int32_t* cnt, int32_t* ent, int64_t cap_total);

/* ---------------- potential energy, forces, virial --------------------- */
/* E = sum_i u_i; F_i = -dE/dR_i; V_mn = -dE/deps_mn (m from r, n from f).
 * R, F are n x 3 row-major.  u may be NULL. */
int orc_eval(const orc_params* p, int n, const double* R, const double* h,
             double* E, double* u, double* F, double* V);

/* ---------------- one image through the rotation-free cell filter ------ */
/* X is (n+3) x 3: rows of R~ then rows of c_f B.  Outputs the enthalpy H, the
 * potential energy E, the generalized force Fg ((n+3) x 3), the raw virial V,
 * the Cartesian forces F (n x 3, may be NULL), positions R (may be NULL) and
 * cell h (may be NULL). */
int orc_cf_eval(const orc_params* p, int n, const double* h0, const double* X,
                double* H, double* E, double* Fg, double* V,
                double* F, double* R, double* h);

/* Build the generalized coordinates of an endpoint (Sec. II.C): X_A from
 * (R_A, h_A) with h0 = h_A, and X_B from (R_B, h_B) with fractional
 * displacements unwrapped against A. */
int orc_build_endpoints(const orc_params* p, int n, const double* RA, const double* hA,
                        const double* RB, const double* hB, double* XA, double* XB);

/* ---------------- band ---------------------------------------------------- */
typedef struct orc_band orc_band;

typedef struct orc_fire_state {
    double dt, alpha;
    int n_pos;       /* FIRE N_P counter */
    int fresh;       /* 1: skip the power test on the next step */
    int step;        /* steps taken (moves) */
    int ci;          /* climbing image chosen at the last evaluation, -1 if none */
} orc_fire_state;

orc_band* orc_band_create(const orc_params* p, int n, const int32_t* types,
                          const double* pos_init, const double* cell_init,
                          const double* pos_final, const double* cell_final, int* err);
int  orc_band_step(orc_band* b, int max_steps, double f_tol,
                   int* steps_done, double* fmax, int* converged);
int  orc_band_refine(orc_band* b, int* inserted_at, int* deleted_at);
int  orc_band_energies(const orc_band* b, double* H, int cap, int* n_images,
                       double* barrier, int* ci_index, double* path_coord);
int  orc_band_n_images(const orc_band* b);
/* State: X and v are n_images x (n+3) x 3 (v rows of the endpoints are zero). */
int  orc_band_get_state(const orc_band* b, double* X, double* v, int cap_images,
                        orc_fire_state* st, double* h0);
int  orc_band_set_state(orc_band* b, int n_images, const double* X, const double* v,
                        const orc_fire_state* st);
/* Data of image k from its last evaluation: E, H, V(9), raw force F (n x 3),
 * generalized force Fg ((n+3) x 3), NEB force Fneb ((n+3) x 3; zero for endpoints),
 * positions R (n x 3) and cell h (9).  Any output may be NULL. */
int  orc_band_image(const orc_band* b, int k, double* E, double* H, double* V,
                    double* F, double* Fg, double* Fneb, double* R, double* h);
void orc_band_destroy(orc_band* b);
/* Threads over which a band's images are evaluated (results do not depend on it). */
void orc_set_threads(int n);
int  orc_max_threads(void);

/* ---------------- energy profile (readout) ------------------------------ */
/* The transitions of Sec. III are shown as enthalpy against a normalized path
 * coordinate.  Path coordinate s_0 = 0, s_{k+1} = s_k + |X_{k+1} - X_k| and slopes
 * dH/ds = -Fg_k . tau_k / |tau_k| (improved tangent for moving images, one-sided
 * difference at the ends), all modulo a rigid translation of the first natoms rows.
 * X and Fg are M x dim row-major; s and slope receive M values. */
int  orc_profile(int M, int natoms, int dim, const double* X, const double* H, const double* Fg,
                 double* s, double* slope);
/* Cubic Hermite interpolant through (s_k, H_k) with slopes slope_k, at nq queries. */
int  orc_spline_eval(int M, const double* s, const double* H, const double* slope, int nq,
                     const double* sq, double* out);
/* Maximum of that interpolant over [s_0, s_{M-1}] and where it is reached. */
int  orc_spline_max(int M, const double* s, const double* H, const double* slope, double* Hmax,
                    double* s_at);
/* Band profile at the current coordinates (every image evaluated afresh): s, H,
 * slope (M values each), samples at xi_j = j / (n_samples - 1) of the normalized
 * coordinate s / s_{M-1} (n_samples = 0 or >= 2), the interpolant's maximum minus
 * H_0 and its normalized coordinate. */
int  orc_band_profile(orc_band* b, int n_samples, double* s, double* H, double* slope,
                      double* samples, double* barrier, double* xi_max);

/* Normalized path coordinate of a band (M x dim row-major, the first natoms rows
 * of 3 are atoms): xi_k = s_k / s_{M-1} with the arc length s of orc_profile
 * (translation-free differences).  orc_band_energies reports the same. */
int  orc_path_coord(int M, int natoms, int dim, const double* X, double* xi);

/* ---------------- pieces exposed for pinning ----------------------------- */
/* One band-global FIRE move (the band step's own routine) of the moving images
 * 1..M-2 of X (M x dim, rows of roww entries) driven by the NEB forces F (M x dim):
 * unless st->fresh, the power P = F.v decides between mixing v toward F (P > 0;
 * dt and alpha grow only after more than nmin such steps in a row) and a reset
 * (v = 0, alpha = astart, dt *= fdec, n_pos = 0); then v += dt F and X += dt v,
 * the step scaled so that no row moves farther than maxstep.  X, v, st in/out. */
int  orc_fire_step(int M, int dim, int roww, double* X, double* v, const double* F,
                   orc_fire_state* st, double dtmax, double maxstep, int nmin, double finc,
                   double fdec, double astart, double fa);
/* Improved tangent coefficients: tau = a tau+ + b tau-. */
void orc_tangent_coeffs(double Hm, double H0, double Hp, double* a, double* b);
/* Refine decision on a band of M images, each of dimension dim (row-major M x dim).
 * ci = current climbing image or -1.  Returns 0 and writes inserted_at / deleted_at
 * (-1 for none) and the spacings d2 (M-1 values, as doubles for reporting only). */
int  orc_refine_decide(int M, int dim, const double* X, int ci, int max_images, int min_images,
                       int ins_num, int ins_den, int del_num, int del_den,
                       int* inserted_at, int* deleted_at, double* d2_report);

/* Climbing-image NEB on the analytic surface V(x,y) = (1-x^2)^2 + kappa (y-x^2)^2.
 * xy: in/out M x 2 band (endpoints fixed).  Uses the same tangent, spring,
 * climbing-image and FIRE code as the atomistic band.  Returns steps taken. */
int  orc_neb2d(double kappa, int M, double* xy, double k_spring, int climb_after,
               double dt0, double dtmax, double maxstep, int max_steps, double f_tol,
               double* energies, int* ci, double* fmax);

/* Single-image relaxation with the cell filter (no NEB projection): FIRE on
 * generalized coordinates until fmax < f_tol.  R, h are in/out. */
int  orc_relax(const orc_params* p, int n, double* R, double* h, int max_steps,
               double f_tol, int* steps_done, double* fmax);

#ifdef __cplusplus
}
#endif
#endif
