/*
 * cfneb.h -- C ABI of the MI355X (gfx950) cell-filter nudged elastic band library.
 *
 * Method: Jia, Shi, Sun, "Scalable cell filter nudged elastic band (CFNEB) for
 * large-scale transition-path calculations", arXiv:2510.16721.
 *
 * The problem (Secs. I, II.A, III): two known endpoint configurations of the same
 * atoms are joined by a chain of images; the chain is relaxed toward the minimum-
 * energy path with the NEB force of Eq. (1) (true force perpendicular to the
 * tangent plus a spring along it, climbing image on the highest image); lattice
 * degrees of freedom move with the atoms through the rotation-free cell filter of
 * Sec. II.C (Eqs. (10)-(17)); images are inserted or removed after iterations
 * (Sec. III); the barrier is the highest image enthalpy minus the initial one.
 *
 * Conventions shared by every call:
 *   - Units: eV, Angstrom, GPa.  A cell is a 3x3 row-major matrix whose ROWS are
 *     the lattice vectors (Sec. II.B, Eq. (2)).  Positions are n x 3 row-major.
 *   - Ownership: the caller owns every host array (copied during the call) and the
 *     device workspace, whose size comes from cfneb_band_bytes.  The library never
 *     allocates or frees device memory; it owns the opaque handle until
 *     cfneb_destroy.  The HIP stream is the caller's; all device work of a band is
 *     ordered on it.
 *   - Errors: every call returns 0 (CFNEB_OK) or a negative CFNEB_E* code; text
 *     for the last failure of a band is in cfneb_last_error.  A step that fails
 *     leaves the band at its pre-step state.
 *   - Threading: one host thread per band handle at a time.
 *   - Environment: CFNEB_NO_GRAPH=1 launches every step kernel by kernel instead of
 *     through captured hipGraphs (same results); CFNEB_FORCE_GRID=persistent|tile
 *     fixes the force kernels' grid instead of choosing it by timing (same results);
 *     CFNEB_LJ_LANES=1|2|4|8, read when an LJ band is created, fixes the lanes that
 *     share an atom in its force kernel instead of the measured table (results equal
 *     to rounding: the lanes' partial forces are summed in a different order).
 */
#ifndef CFNEB_H
#define CFNEB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CFNEB_OK = 0,
    CFNEB_EINVAL = -1,      /* bad argument or parameter */
    CFNEB_ENOMEM = -2,      /* workspace smaller than cfneb_band_bytes */
    CFNEB_EHIP = -3,        /* a HIP runtime call failed */
    CFNEB_ECELL = -4,       /* cell not positive definite, or a neighbour shift beyond +-7 cells */
    CFNEB_ENEIGH = -5,      /* an atom has more neighbours than nbr_cap */
    CFNEB_ENONFINITE = -6,  /* energy, virial or force not finite */
    CFNEB_ECAPACITY = -7,   /* image capacity exceeded */
    CFNEB_ERANGE = -8       /* a squared spacing term outside [0, 2^40) */
};

enum { CFNEB_LJ = 1, CFNEB_TERSOFF_C = 2 };

/* Parameters of one band.  cfneb_params_default fills every field. */
typedef struct cfneb_params {
    int potential;          /* CFNEB_LJ or CFNEB_TERSOFF_C */
    int force_fp64;         /* 1: pair / three-body arithmetic in FP64; 0: FP32 with FP64 sums */
    /* shifted Lennard-Jones: 4 eps [(s/r)^12 - (s/r)^6] - (same at rc) */
    double lj_eps, lj_sigma, lj_rc;
    int lj_shift;
    /* Tersoff bond-order form, lambda3 = 0 (defaults: Tersoff 1988 carbon) */
    double ts_A, ts_B, ts_lambda1, ts_lambda2, ts_beta, ts_n, ts_c, ts_d, ts_h, ts_R, ts_S;
    /* band */
    int n_images;           /* images including both fixed endpoints, >= 3 */
    int max_images;         /* image capacity (adaptive insertion), <= 64 */
    int min_images;         /* deletion never goes below this */
    double k_spring;        /* eV / A^2 */
    int climb_after;        /* climbing image from this step on; < 0: never */
    int cell_filter;        /* 0: cell fixed; 1: D-variant, coordinates c_f D and force
                               D^-T V / c_f (Eq. (13)); 2: rotation-free filter, c_f B
                               and D^-T V D^-1 / c_f (Eq. (17)) */
    double cell_factor;     /* c_f, generalized cell coordinate c_f B;
                               <= 0: |det h0|^(1/3) n_atoms^(1/6) */
    double b_force_scale;   /* factor on the lattice force D^-T V D^-1 / c_f (default 1) */
    double pressure_GPa;    /* hydrostatic pressure; images carry H = U + P Omega */
    /* FIRE */
    double fire_dt0, fire_dtmax, fire_maxstep;
    int fire_nmin;
    double fire_finc, fire_fdec, fire_astart, fire_fa;
    /* adaptive images: every refine_every steps (0 = off); insert into the longest
       interval if ins_den (M-1) d_k^2 > ins_num sum d^2; otherwise delete the image
       whose longer neighbouring interval is shortest if
       del_den (M-1) max(d_{j-1}^2, d_j^2) < del_num sum d^2 */
    int refine_every;
    int ins_num, ins_den, del_num, del_den;
    int nbr_cap;            /* neighbour entries per atom */
    double nbr_skin;        /* candidate-list skin (A): pairs closer than rc + skin are kept
                               as candidates and re-tested exactly every step; the candidates
                               are rebuilt when atoms (relative to the affinely strained cell)
                               or the cell moved enough that a pair could have crossed it.
                               0: rebuild every step.  The neighbour set is the same. */
    double stress_GPa[6];   /* applied stress beyond the pressure, Voigt order xx yy zz yz xz
                               xy, tensile positive: a constant second Piola-Kirchhoff stress S
                               referred to the reference cell h0 (the non-hydrostatic loading
                               that Sec. I names as the reason for finite-deformation NEB).
                               Images carry H = U + P Omega - Omega0 S : E with
                               E = (D D^T - I) / 2 and Omega0 = |det h0|, and the lattice
                               forces of both filters follow from V_eff = V - P Omega I +
                               Omega0 D^T S D.  All zero: hydrostatic only. */
} cfneb_params;

/* Optimizer and band bookkeeping, for checkpoints and tests. */
typedef struct cfneb_fire_state {
    double dt, alpha;
    int n_pos;              /* FIRE count of consecutive P > 0 steps */
    int fresh;              /* 1: the next step skips the P = F.v test */
    int step;               /* steps taken (moves) */
    int ci;                 /* climbing image of the last evaluation, -1 if none */
    long long image_steps;  /* sum over the steps taken of the number of moving images
                               (read-only: cfneb_set_state ignores it) */
} cfneb_fire_state;

/* Phases of one band step, in launch order, for cfneb_step_profiled. */
enum {
    CFNEB_PH_GEOM = 0,      /* per-image D = symsqrt(B), h, h^-1, bin grid */
    CFNEB_PH_SKIN,          /* R = R~ D, displacement since the last candidate build */
    CFNEB_PH_BINS,          /* bin ids, counting sort, per-bin order (rebuilds only) */
    CFNEB_PH_NLIST,         /* candidate pairs within rc + skin (rebuilds only) */
    CFNEB_PH_FILTER,        /* exact neighbour test of the candidates, packed lists */
    CFNEB_PH_FORCE0,        /* LJ pair forces, or for Tersoff the exact test of the
                               candidates, bond orders, energy, virial and dU_i/dr^ij */
    CFNEB_PH_FORCE1,        /* Tersoff force gather (unused for LJ) */
    CFNEB_PH_FORCE2,        /* (empty: the Tersoff kernels are fused into two) */
    CFNEB_PH_REDUCE,        /* (empty in a step: the dots phase reduces E and V) */
    CFNEB_PH_DOTS,          /* per-image E, V, enthalpy, lattice force; band dots */
    CFNEB_PH_SCALARS,       /* tangents, climbing image, projection, FIRE proposal */
    CFNEB_PH_UPDATE,        /* NEB force rows, new velocities, row maxima */
    CFNEB_PH_FINALIZE,      /* fmax, convergence, step clamp, FIRE commit */
    CFNEB_PH_MOVE,          /* X += dr */
    CFNEB_PH_REFINE,        /* adaptive-image check */
    CFNEB_NPHASE
};

typedef struct cfneb_band cfneb_band;

/* Fill *out with the defaults for a potential (the short-range potentials of the
 * per-atom form of Sec. II.B, Eq. (4); the band, filter and optimizer settings of
 * Secs. II.A, II.C and III, where the paper leaves values open): LJ eps = sigma = 1,
 * rc = 2.5, shifted; Tersoff 1988 carbon (R = 1.8, S = 2.1); 7 images, k = 1,
 * climbing after 50 steps, rotation-free filter (Eq. (17)), c_f = 0 (that is,
 * |det h0|^(1/3) n_atoms^(1/6)); FIRE dt0 0.005 (LJ) / 0.05 (Tersoff), dtmax =
 * 10 dt0, maxstep 0.1, Nmin 5, finc 1.1, fdec 0.5, alpha 0.1, f_alpha 0.99; refine
 * off with thresholds 9/4 and 1/4; nbr_cap 128 (LJ) / 16; nbr_skin 0.3.
 * CFNEB_EINVAL for an unknown potential or NULL out. */
int cfneb_params_default(int potential, cfneb_params* out);

/* Device workspace bytes for a band of n_atoms atoms and up to max_images images
 * (max_images <= 0: p->max_images), the storage of the images, lists and scratch
 * that one band step of Secs. II and III needs.  This is also the band's HBM
 * footprint (what a request loop admits by).  CFNEB_EINVAL for bad parameters,
 * n_atoms outside [1, 2^20) or max_images outside [3, 64]. */
int cfneb_band_bytes(const cfneb_params* p, int64_t n_atoms, int max_images, size_t* bytes);

/* Build a band (Secs. II.C, III): h0 = cell_init is the reference cell of every
 * image; the initial image has D = I and R~ = pos_init; the final image has
 * B = D D^T with D = h0^-1 cell_final and R~ = pos_init + ds h0, where ds is the
 * fractional displacement wrapped to the nearest image; the n_images - 2 moving
 * images are linear in (R~, c_f B).  Every image is evaluated once.
 * pos_*: n_atoms x 3 host arrays; cell_*: 3x3 host arrays; types: ignored (one
 * species), may be NULL.  workspace: device pointer of workspace_bytes bytes,
 * 256-byte aligned.  hip_stream: a hipStream_t (NULL: the null stream).
 * Returns ENOMEM if workspace_bytes < cfneb_band_bytes(p, n_atoms, 0). */
int cfneb_create_band(const cfneb_params* p, int64_t n_atoms, const int32_t* types,
                      const double* pos_init, const double* cell_init,
                      const double* pos_final, const double* cell_final,
                      void* workspace, size_t workspace_bytes, void* hip_stream,
                      cfneb_band** out);

/* Up to max_steps band steps.  One step: per moving image the cell-filter
 * geometry, cell list, neighbour list, energy / forces / virial (Sec. II.B),
 * generalized forces (Eq. (17)); improved tangent, springs and climbing image
 * (Eq. (1)); fmax = largest row norm of the NEB force; if fmax < f_tol the band
 * is converged and is not moved; otherwise a band-global FIRE move.  Every
 * refine_every steps an image may be inserted or deleted (Sec. III).
 * Outputs (any may be NULL): steps taken, fmax of the last evaluation,
 * converged flag. */
int cfneb_step(cfneb_band* b, int max_steps, double f_tol, int* steps_done, double* fmax,
               int* converged);

/* The same steps as cfneb_step, launched one phase at a time with a HIP event
 * recorded on the band's stream around every phase.  phase_ms (nphase doubles,
 * nphase <= CFNEB_NPHASE, indexed by CFNEB_PH_*) receives the summed device time
 * of each phase over the steps run, in milliseconds; it is a measuring tool, not
 * the fast path (no graph, one event pair per phase and step). */
int cfneb_step_profiled(cfneb_band* b, int max_steps, double f_tol, int* steps_done, double* fmax,
                        int* converged, double* phase_ms, int nphase);

/* One adaptive-image decision now (Sec. III): squared spacings between
 * consecutive images summed exactly in fixed point, then at most one insertion
 * (midpoint of the longest interval) or deletion (never the climbing image),
 * followed by a FIRE velocity reset.  inserted_at / deleted_at: logical index of
 * the new or removed image, -1 for none. */
int cfneb_refine(cfneb_band* b, int* inserted_at, int* deleted_at);

/* Readout (Sec. III, which reports each transition as image enthalpies against a
 * normalized path coordinate, the barrier being the highest image minus the
 * initial state): H[k] for the n_images current images (cap >= n_images), the
 * barrier max_k H_k - H_0, the climbing image (-1 if none) and the path coordinate
 * xi_k = s_k / s_{M-1}, s_0 = 0, s_{k+1} = s_k + |X_{k+1} - X_k| with the atoms'
 * rigid translation removed from each difference (the arc length of cfneb_profile;
 * path_coord may be NULL).  H values are those of the last evaluation; a freshly
 * inserted image reports the mean of its neighbours until evaluated.  Launches two
 * small kernels on the band's stream and synchronises it.  Errors: CFNEB_EINVAL for
 * a NULL band or cap < n_images (H given). */
int cfneb_energies(const cfneb_band* b, double* H, int cap, int* n_images, double* barrier,
                   int* ci_index, double* path_coord);

/* Energy profile of the band at its current coordinates: the enthalpy against the
 * path coordinate, the form in which Sec. III reports its transitions, continued
 * between the images so that barriers can be read between them.  Every image is
 * evaluated afresh (also the endpoints and a band that has converged).  With
 * translation-free image differences and forces (atom-row means removed):
 *   s_0 = 0, s_{k+1} = s_k + |X_{k+1} - X_k|   arc length in generalized coordinates
 *   slope_k = dH/ds = -Fg_k . tau_k / |tau_k|   tau_k the improved tangent of the
 *                                               band for 0 < k < M-1, X_1 - X_0 at
 *                                               k = 0, X_{M-1} - X_{M-2} at M-1
 * and on each interval the cubic Hermite interpolant through (s_k, H_k) and
 * (s_{k+1}, H_{k+1}) with those slopes.
 * Outputs (host arrays; any pointer may be NULL): s, H, slope (M values each,
 * cap >= M when any is given); samples[j] = the interpolant at the normalized
 * coordinate xi_j = j / (n_samples - 1) of s / s_{M-1}, for n_samples = 0 (none) or
 * 2 .. CFNEB_PROFILE_MAX_SAMPLES; *barrier = its maximum minus H_0; *xi_max = the
 * normalized coordinate of that maximum.  Overwrites the images' stored energies
 * and forces with those of the current coordinates (what a following step computes
 * first anyway); not during a cfneb_batch_step call of a batch holding the band.
 * Errors: CFNEB_EINVAL for n_samples outside that range (or samples NULL with
 * n_samples > 0) or cap < M; the band's own error code if its last call failed or
 * the evaluation finds a non-finite energy, force or virial (outputs untouched).
 * Synchronises the band's stream before returning. */
#define CFNEB_PROFILE_MAX_SAMPLES 4096
int cfneb_profile(cfneb_band* b, int n_samples, double* s, double* H, double* slope, int cap, int* n_images,
                  double* samples, double* barrier, double* xi_max);

/* Cartesian positions (n_atoms x 3) and cell (3x3) of current image k, mapped back
 * from the filter's coordinates (Sec. II.C, Eqs. (10)-(11), (15)): h = h0 D and
 * R = R~ D with D = symsqrt(B) (rotation-free filter) or the stored D (D-variant).
 * Host outputs; CFNEB_EINVAL for k outside [0, n_images).  Synchronises the
 * band's stream. */
int cfneb_get_image(const cfneb_band* b, int k, double* pos, double* cell);

/* Relax one structure with the cell filter (Sec. II.C, which introduces the filter
 * for relaxing lattice and positions together; band endpoints are such minima).
 * FIRE, as in a band step, on the generalized coordinates (R~, c_f B) with the
 * input cell as reference h0, driven by the generalized force (F D^T, G / c_f)
 * without projection or springs, until the largest row norm is below f_tol or
 * max_steps moves were made.  Potential, pressure, applied stress (referred to the
 * input cell), cell filter, cell factor and FIRE fields of p apply; image, spring, climbing-image and refine fields are
 * ignored.  pos (n_atoms x 3) and cell (3x3) are host arrays, read, then
 * overwritten with the relaxed R = R~ D and h = h0 D; on error they are left as
 * they were.  workspace: >= cfneb_band_bytes(p, n_atoms, 3) device bytes,
 * 256-byte aligned, free again on return.  *converged = 1 if f_tol was reached. */
int cfneb_relax(const cfneb_params* p, int64_t n_atoms, const int32_t* types, double* pos, double* cell,
                int max_steps, double f_tol, void* workspace, size_t workspace_bytes, void* hip_stream,
                int* steps_done, double* fmax, int* converged);

/* cfneb_relax for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same relaxation and the same
 * kernels, with the band's device memory taken from a static array of
 * CFNEB_RELAX_SCRATCH_BYTES on each GPU (held until the process ends) instead of a
 * caller workspace, and no allocation of any kind (no device or pinned host memory,
 * no graph, stream or event).  Kernels are launched one by one on hip_stream; the call
 * synchronises it before returning.  Arguments and results as cfneb_relax.  Errors:
 * CFNEB_ENOMEM when cfneb_band_bytes(p, n_atoms, 3) exceeds
 * CFNEB_RELAX_SCRATCH_BYTES (about 13,500 atoms for LJ, 17,500 for FP32 Tersoff
 * carbon), CFNEB_EHIP if the array's address cannot be found; otherwise those of
 * cfneb_relax.  Every call on one GPU uses that GPU's array and clears it first; two
 * calls that overlap on one GPU (two host threads, or two streams) race and must not
 * be made. */
#define CFNEB_RELAX_SCRATCH_BYTES (64u << 20)
int cfneb_relax_noalloc(const cfneb_params* p, int64_t n_atoms, const int32_t* types, double* pos,
                        double* cell, int max_steps, double f_tol, void* hip_stream, int* steps_done,
                        double* fmax, int* converged);

/* Checkpoint: generalized coordinates X and velocities v of the n_images images,
 * each (n_atoms + 3) x 3 row-major (rows of R~, then rows of c_f B: the coordinates
 * of Sec. II.C, Eq. (15)), into host arrays of cap_images images; FIRE state.  X and
 * v may be NULL (then only n_images and st are written); CFNEB_EINVAL if
 * cap_images < n_images with X or v given. */
int cfneb_get_state(const cfneb_band* b, double* X, double* v, int cap_images, int* n_images,
                    cfneb_fire_state* st);

/* Restore a checkpoint (same layout as cfneb_get_state, Sec. II.C coordinates);
 * every image is evaluated again.  v may be NULL (zero velocities).  CFNEB_EINVAL
 * for n_images outside [3, max_images]; an evaluation error leaves the band failed
 * with that code. */
int cfneb_set_state(cfneb_band* b, int n_images, const double* X, const double* v,
                    const cfneb_fire_state* st);

/* Data of image k from its last evaluation (any output may be NULL): potential
 * energy E, enthalpy H, virial V (3x3, V_mn = -1/2 sum r^ij_m f^ij_n, Eq. (8)),
 * Cartesian force F (n x 3), generalized force Fg ((n+3) x 3, Eq. (17)), NEB force
 * Fneb ((n+3) x 3; filled only for moving images and only when the band was
 * created with record_neb_force set, else zero), positions R (n x 3), cell h (3x3). */
int cfneb_image_data(const cfneb_band* b, int k, double* E, double* H, double* V, double* F,
                     double* Fg, double* Fneb, double* R, double* h);

/* Keep the NEB force of Eq. (1) of every moving image in device memory at each
 * step so that cfneb_image_data can return it (costs one extra store per row).
 * on: 0 or 1. */
int cfneb_record_neb_force(cfneb_band* b, int on);

/* Neighbour set of image k from its last evaluation: cnt[i] entries per atom,
 * written as (j, n0, n1, n2) int32 quadruples into ent (cap quadruples), atom by
 * atom, each atom's entries in the (deterministic) order the device built them.
 * The entries of atom i are every (j, n) != (i, 0) with
 *     r = (R_j - R_i) + ((n0 h_0 + n1 h_1) + n2 h_2),  (r_x r_x + r_y r_y) + r_z r_z < rc^2
 * each operation rounded on its own in FP64.  *total is the number of entries
 * (may exceed cap; then ent holds the first cap).  A step keeps per-candidate data
 * only, so this call first re-runs the exact test of the current candidates on the
 * positions and cell of the last evaluation (one launch on the band's stream, then a
 * synchronisation); the set is the one the step's force kernels used. */
int cfneb_neighbours(const cfneb_band* b, int k, int32_t* cnt, int32_t* ent, int64_t cap,
                     int64_t* total);

/* Release the handle (the caller's workspace and stream are untouched; the band's
 * stream is synchronised first).  Not for a band attached to a batch. */
int cfneb_destroy(cfneb_band* b);

/* ---------------------------------------------------------------- batches
 * Many independent bands stepped together.  Every phase of the step (the same
 * computation as cfneb_step) is ONE persistent launch over the work items of all
 * live bands, whatever their atom and image counts; the step is captured once in a
 * hipGraph, and attaching or detaching a band only rewrites a device table.  Each
 * band's result does not depend on its batch-mates (no shared reductions).
 * Ownership: the caller owns the batch workspace (cfneb_batch_bytes) and every band
 * it attaches (cfneb_batch_attach), which must outlive its membership; a band made
 * with cfneb_batch_add belongs to the batch until removed.  While in a batch, a
 * band must not be stepped on its own. */
typedef struct cfneb_batch cfneb_batch;

/* Device bytes of a batch table for up to max_bands bands (<= 128): a descriptor
 * per band and the work plan of the persistent launches.  Bands keep their own
 * workspaces.  CFNEB_EINVAL for max_bands outside [1, 128]. */
int cfneb_batch_bytes(int max_bands, size_t* bytes);

/* A batch of up to max_bands independent bands, each relaxed by the band step of
 * Secs. II and III.  workspace: >= cfneb_batch_bytes device bytes, 256-byte
 * aligned, owned by the caller.  hip_stream: the stream every batch launch goes to
 * (NULL: null stream).  CFNEB_EINVAL / CFNEB_ENOMEM / CFNEB_EHIP on bad arguments, a
 * small workspace or a failing HIP call. */
int cfneb_batch_create(int max_bands, void* workspace, size_t workspace_bytes, void* hip_stream,
                       cfneb_batch** out);

/* Add a band (created with cfneb_create_band; it stays the caller's); *slot
 * receives its table index.  Synchronises the band's stream.  Returns
 * CFNEB_ECAPACITY when the table is full, CFNEB_EINVAL if the band is already in
 * the table. */
int cfneb_batch_attach(cfneb_batch* batch, cfneb_band* band, int* slot);

/* Remove the band in table slot `slot` (the band itself is untouched).  A band that
 * cfneb_batch_add made passes to the caller here (take its handle from
 * cfneb_batch_band first; destroy it with cfneb_destroy). */
int cfneb_batch_detach(cfneb_batch* batch, int slot);

/* Create a band (exactly as cfneb_create_band, Secs. II.C and III; the band's device
 * work goes to the batch's stream) and attach it in one call.  The band belongs to
 * the batch: cfneb_batch_remove or cfneb_batch_destroy destroys it.  The caller
 * still owns `workspace` (>= cfneb_band_bytes(p, n_atoms, 0) bytes, 256-byte
 * aligned), which must stay allocated until the band is removed.  *slot receives
 * the table index.  Errors: those of cfneb_create_band (nothing is attached), or
 * CFNEB_ECAPACITY when the table is full (nothing is created). */
int cfneb_batch_add(cfneb_batch* batch, const cfneb_params* p, int64_t n_atoms, const int32_t* types,
                    const double* pos_init, const double* cell_init, const double* pos_final,
                    const double* cell_final, void* workspace, size_t workspace_bytes, int* slot);

/* Detach the band in `slot` and, if cfneb_batch_add made it, destroy it (its
 * workspace is then free for the caller).  A band attached with cfneb_batch_attach
 * is only detached.  CFNEB_EINVAL for an empty slot. */
int cfneb_batch_remove(cfneb_batch* batch, int slot);

/* Handle of the band in `slot` (NULL for an empty slot), for the per-band calls
 * (cfneb_energies, cfneb_profile, cfneb_get_image, cfneb_get_state ...) between
 * batch steps.  A band the batch owns must not be destroyed through it. */
cfneb_band* cfneb_batch_band(cfneb_batch* batch, int slot);

/* Readout of the band in `slot` after batch steps: the outputs of cfneb_energies
 * (Sec. III: image enthalpies, barrier = highest image minus the initial state,
 * climbing image, normalized path coordinate).  CFNEB_EINVAL for an empty slot. */
int cfneb_batch_energies(cfneb_batch* batch, int slot, double* H, int cap, int* n_images, double* barrier,
                         int* ci_index, double* path_coord);

/* Up to max_steps steps of every attached band with the same f_tol; a band that
 * converges or fails stops moving while the others go on, and the call returns
 * early once no band is still relaxing.  Per table slot (arrays of max_bands
 * entries, any may be NULL): steps taken in this call, converged flag, error code
 * (0 or a CFNEB_E* code; the band is left at its pre-step state). */
int cfneb_batch_step(cfneb_batch* batch, int max_steps, double f_tol, int* steps_done,
                     uint8_t* converged, int* errors);

/* Release the batch: bands made by cfneb_batch_add are destroyed, attached bands
 * are left as they are (no longer in a table); the workspace stays the caller's. */
int cfneb_batch_destroy(cfneb_batch* batch);

/* Static text of a CFNEB_E* code. */
const char* cfneb_strerror(int code);
/* Text of the band's last failure ("" if none; "no band" for NULL); valid until
 * the band's next call. */
const char* cfneb_last_error(const cfneb_band* b);

#ifdef __cplusplus
}
#endif
#endif
