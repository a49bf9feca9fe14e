// Host runtime and C ABI of the CFNEB library: workspace layout, band creation,
// the captured step graph, checkpoints and readout.  All arithmetic of the band
// step runs in the kernels; the host only lays out memory, launches and copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cfneb_dev.h"
#include "lj_lanes_table.h"

using namespace cfneb;

namespace {

constexpr double kEvPerA3InGPa = 160.21766208;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    int N, ld, Mcap, ntA, ntR, ntR4, nbcap, cap, ccap, fp64, tersoff;
    size_t X, V, R, S, F, FN, binfo, bcount, bstart, bpos, nbr, ncnt, cand, ncand, Rref, skin, dvec, bo, bcid, P, crev, geom,
        scal, dotred, skmax,
        evpart, dotpart, maxpart, refpart, staging, state, table, live, plan, total;
};

bool make_layout(const cfneb_params* p, int64_t n_atoms, int max_images, Layout* L)
{
    if (n_atoms < 1 || n_atoms >= CFNEB_MAX_ATOMS) return false;
    if (max_images < 3 || max_images > CFNEB_MAX_IMAGES) return false;
    if (p->nbr_cap < 1 || p->nbr_cap > 1024) return false;
    L->N = int(n_atoms);
    L->ld = ((L->N + 3 + 63) / 64) * 64;
    L->Mcap = max_images;
    L->ntA = (L->N + CFNEB_TILE - 1) / CFNEB_TILE;
    L->ntR = (L->N + 3 + CFNEB_TILE - 1) / CFNEB_TILE;
    L->ntR4 = (L->N + 3 + CFNEB_TILE4 - 1) / CFNEB_TILE4;
    L->nbcap = L->N + 64;
    L->cap = p->nbr_cap;
    {
        // candidates within rc + skin: the neighbour capacity scaled by the volume ratio
        const double rc = p->potential == CFNEB_LJ ? p->lj_rc : p->ts_S;
        const double ratio = (rc + p->nbr_skin) / rc;
        L->ccap = int(std::ceil(1.25 * p->nbr_cap * ratio * ratio * ratio));
    }
    // the Tersoff reverse index (slot x N + atom) is 32-bit
    if (p->potential == CFNEB_TERSOFF_C && size_t(L->ccap) * size_t(L->N) > 0xFFFFFFFFull) return false;
    L->fp64 = p->force_fp64 ? 1 : 0;
    L->tersoff = (p->potential == CFNEB_TERSOFF_C) ? 1 : 0;
    const size_t M = size_t(L->Mcap), N = size_t(L->N), rows = 3 * size_t(L->ld);
    const size_t tsz = L->fp64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L->X = take(M * rows * 8);
    L->V = take(2 * M * rows * 8);
    L->R = take(M * size_t(L->ld) * 24);
    L->S = take(L->tersoff || L->fp64 ? 0 : M * size_t(L->ld) * 12);
    L->F = take(M * rows * tsz);
    L->FN = take(M * rows * 8);
    L->binfo = take(M * N * 16);
    L->bcount = take(M * (L->nbcap + 1) * 4);
    L->bstart = take(M * (L->nbcap + 1) * 4);
    L->bpos = take(M * N * sizeof(BinAtom));
    L->nbr = take(M * size_t(L->cap) * N * 4);
    L->ncnt = take(M * N * 4);
    L->cand = take(M * size_t(L->ccap) * N * 4);
    L->ncand = take(M * N * 4);
    L->Rref = take(M * rows * 4);
    L->skin = take(M * sizeof(SkinState));
    L->dvec = take(L->tersoff ? M * size_t(L->cap) * N * 4 * tsz : 0);
    L->bo = take(L->tersoff ? M * size_t(L->cap) * N * 2 * tsz : 0);
    L->bcid = take(L->tersoff ? M * size_t(L->cap) * N * 4 : 0);
    L->P = take(L->tersoff ? M * size_t(L->ccap) * N * 3 * tsz : 0);
    L->crev = take(L->tersoff ? M * size_t(L->ccap) * N * 4 : 0);
    L->geom = take(M * sizeof(ImageGeom));
    L->scal = take(M * sizeof(ImageScal));
    L->evpart = take(M * L->ntA * CFNEB_WAVES * 10 * 8);
    L->dotred = take(M * CFNEB_NDOT * 8);
    L->dotpart = take(M * L->ntR4 * CFNEB_WAVES * CFNEB_NDOT * 8);
    L->maxpart = take(M * L->ntR4 * 3 * 8);
    L->skmax = take(M * size_t((L->N + CFNEB_TILE4 - 1) / CFNEB_TILE4) * 2 * 8);
    L->refpart = take(M * L->ntR * 2 * 8);
    L->staging = take(std::max<size_t>(6 * N + 64, CFNEB_PROF_DOUBLES) * 8);
    L->state = take(sizeof(BandState));
    // the band's own one-entry table for the persistent kernels
    L->table = take(sizeof(BandDev));
    L->live = take(sizeof(int));
    L->plan = take((NKIND * 2 + 2) * sizeof(int));
    L->total = off;
    return true;
}

// Lanes sharing an atom in the LJ force kernel, a property of the band: from the
// table that tune_lanes.py measures (fastest lane count of a band stepped alone, by
// atoms x images), or CFNEB_LJ_LANES.
int lj_lanes_for(long long atoms, int images)
{
    const char* v = std::getenv("CFNEB_LJ_LANES");
    if (v) {
        const int k = std::atoi(v);
        if (k == 1 || k == 2 || k == 4 || k == 8) return k;
    }
    const long long work = atoms * images;
    for (const auto& e : kLjLanesTable)
        if (work <= e.max_atom_images) return e.lanes;
    return 1;
}

// Grids of a band table, bounded by the most items its bands can hold.
void size_grids(Launch& L, long long atom_tiles, long long row_tiles, long long bin_tiles, long long images,
                int bands, long long atom4_tiles, long long row4_tiles)
{
    L.g[KIND_ATOM4] = grid_for(atom4_tiles, CFNEB_GRID_TILES);
    L.g[KIND_ROW4] = grid_for(row4_tiles, CFNEB_GRID_TILES);
    L.g[KIND_ATOM] = grid_for(atom_tiles, CFNEB_GRID_TILES);
    L.g[KIND_ROW] = grid_for(row_tiles, CFNEB_GRID_TILES);
    L.g[KIND_BIN] = grid_for(bin_tiles, CFNEB_GRID_TILES);
    L.g[KIND_IMAGE] = grid_for(images, CFNEB_GRID_IMAGES);
    L.g[KIND_IVAL] = grid_for(row_tiles, CFNEB_GRID_TILES);
    L.g[KIND_SLOTROW] = grid_for(row_tiles, CFNEB_GRID_TILES);
    L.g[KIND_BAND] = grid_for(bands, CFNEB_GRID_BANDS);
    L.g_force_tile = grid_for(atom_tiles, CFNEB_GRID_FORCE);
    L.g_force = L.g_force_tile;
}

const char* err_text(int code)
{
    switch (code) {
    case CFNEB_OK: return "ok";
    case CFNEB_EINVAL: return "invalid argument";
    case CFNEB_ENOMEM: return "workspace too small";
    case CFNEB_EHIP: return "HIP runtime error";
    case CFNEB_ECELL: return "cell not positive definite or neighbour shift out of range";
    case CFNEB_ENEIGH: return "neighbour list capacity exceeded";
    case CFNEB_ENONFINITE: return "non-finite energy, virial or force";
    case CFNEB_ECAPACITY: return "image capacity exceeded";
    case CFNEB_ERANGE: return "spacing term out of range";
    default: return "unknown error";
    }
}

}  // namespace

struct cfneb_band {
    cfneb_params p;
    BandDev d;
    Layout L;
    Launch launch;  // the band as a table of one
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;  // a whole step
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_core = nullptr;  // a step without the refinement phase
    hipGraphExec_t exec_core = nullptr;
    BandState* host_state = nullptr;  // pinned
    bool use_graph = true;
    std::string last_error;
};

namespace {

int fail(cfneb_band* b, int code, const std::string& what)
{
    if (b) b->last_error = what + ": " + err_text(code);
    return code;
}

#define HIP_TRY(b, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((b), CFNEB_EHIP, std::string(#call) + " -> " + hipGetErrorString(e_)); \
    } while (0)

int read_state(cfneb_band* b)
{
    HIP_TRY(b, hipMemcpyAsync(b->host_state, b->d.st, sizeof(BandState), hipMemcpyDeviceToHost,
                              b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    return CFNEB_OK;
}

int write_state(cfneb_band* b)
{
    HIP_TRY(b, hipMemcpyAsync(b->d.st, b->host_state, sizeof(BandState), hipMemcpyHostToDevice,
                              b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    return CFNEB_OK;
}

int check_kernels(cfneb_band* b, const char* what)
{
    HIP_TRY(b, hipGetLastError());
    (void)what;
    return CFNEB_OK;
}

// Default c_f: |det h0|^(1/3) n^(1/6), the size-consistent Jacobian of the
// generalized solid-state NEB (cell strain and atomic displacement weigh alike in
// the band metric and have alike stiffness at every system size).
double default_cell_factor(const double* h0, int n)
{
    const double det = h0[0] * (h0[4] * h0[8] - h0[5] * h0[7]) - h0[1] * (h0[3] * h0[8] - h0[5] * h0[6]) +
                       h0[2] * (h0[3] * h0[7] - h0[4] * h0[6]);
    return std::cbrt(std::fabs(det)) * std::pow(double(n), 1.0 / 6.0);
}

void fill_dev(cfneb_band* b, void* ws, const double* h0, int relax)
{
    const cfneb_params* p = &b->p;
    const Layout& L = b->L;
    BandDev& d = b->d;
    std::memset(&d, 0, sizeof(d));
    d.N = L.N;
    d.ld = L.ld;
    d.Mcap = L.Mcap;
    d.ntA = L.ntA;
    d.ntR = L.ntR;
    d.ntR4 = L.ntR4;
    d.nbcap = L.nbcap;
    d.cap = L.cap;
    d.ccap = L.ccap;
    d.potential = p->potential;
    d.fp64 = L.fp64;
    if (p->potential == CFNEB_LJ) {
        d.rc = p->lj_rc;
    } else {
        d.rc = p->ts_S;
    }
    d.rc2 = d.rc * d.rc;
    d.skin = p->nbr_skin;
    d.rcl = d.rc + d.skin;
    d.rcl2 = d.rcl * d.rcl;
    d.lj_eps = p->lj_eps;
    d.lj_lanes = lj_lanes_for(L.N, p->n_images);
    d.lj_sig2 = p->lj_sigma * p->lj_sigma;
    if (p->lj_shift) {
        const double q = d.lj_sig2 / (p->lj_rc * p->lj_rc);
        const double q3 = q * q * q;
        d.lj_eshift = 4.0 * p->lj_eps * (q3 * q3 - q3);
    }
    d.ts_A = p->ts_A;
    d.ts_B = p->ts_B;
    d.ts_l1 = p->ts_lambda1;
    d.ts_l2 = p->ts_lambda2;
    d.ts_beta = p->ts_beta;
    d.ts_bn = std::pow(p->ts_beta, p->ts_n);
    d.ts_lnbeta = std::log(p->ts_beta);
    d.ts_n = p->ts_n;
    d.ts_c2 = p->ts_c * p->ts_c;
    d.ts_d2 = p->ts_d * p->ts_d;
    d.ts_c2d2 = d.ts_c2 / d.ts_d2;
    d.ts_h = p->ts_h;
    d.ts_R = p->ts_R;
    d.ts_S = p->ts_S;
    d.k_spring = p->k_spring;
    d.climb_after = p->climb_after;
    d.cell_filter = p->cell_filter;
    for (int q = 0; q < 9; ++q) d.h0[q] = h0[q];
    d.cf = p->cell_factor > 0.0 ? p->cell_factor : default_cell_factor(h0, L.N);
    d.relax = relax;
    d.bscale = p->b_force_scale;
    d.press = p->pressure_GPa / kEvPerA3InGPa;
    {
        // applied stress (Voigt xx yy zz yz xz xy) as a symmetric 3x3 in eV/A^3
        static const int voigt[9] = {0, 5, 4, 5, 1, 3, 4, 3, 2};
        d.stressed = 0;
        for (int q = 0; q < 9; ++q) {
            d.sapp[q] = p->stress_GPa[voigt[q]] / kEvPerA3InGPa;
            if (d.sapp[q] != 0.0) d.stressed = 1;
        }
        d.omega0 = std::fabs(h0[0] * (h0[4] * h0[8] - h0[5] * h0[7]) - h0[1] * (h0[3] * h0[8] - h0[5] * h0[6]) +
                             h0[2] * (h0[3] * h0[7] - h0[4] * h0[6]));
    }
    d.dt0 = p->fire_dt0;
    d.dtmax = p->fire_dtmax;
    d.maxstep = p->fire_maxstep;
    d.nmin = p->fire_nmin;
    d.finc = p->fire_finc;
    d.fdec = p->fire_fdec;
    d.astart = p->fire_astart;
    d.fa = p->fire_fa;
    d.refine_every = p->refine_every;
    d.ins_num = p->ins_num;
    d.ins_den = p->ins_den;
    d.del_num = p->del_num;
    d.del_den = p->del_den;
    d.max_images = p->max_images;
    d.min_images = p->min_images;
    char* base = static_cast<char*>(ws);
    d.X = reinterpret_cast<double*>(base + L.X);
    d.V = reinterpret_cast<double*>(base + L.V);
    d.R = reinterpret_cast<double*>(base + L.R);
    d.S = (L.tersoff || d.fp64) ? nullptr : reinterpret_cast<uint32_t*>(base + L.S);
    d.F = base + L.F;
    d.FN = reinterpret_cast<double*>(base + L.FN);
    d.binfo = reinterpret_cast<int4*>(base + L.binfo);
    d.bcount = reinterpret_cast<int*>(base + L.bcount);
    d.bstart = reinterpret_cast<int*>(base + L.bstart);
    d.bpos = reinterpret_cast<BinAtom*>(base + L.bpos);
    d.nbr = reinterpret_cast<uint32_t*>(base + L.nbr);
    d.ncnt = reinterpret_cast<int*>(base + L.ncnt);
    d.cand = reinterpret_cast<uint32_t*>(base + L.cand);
    d.ncand = reinterpret_cast<int*>(base + L.ncand);
    d.Rref = reinterpret_cast<float*>(base + L.Rref);
    d.skst = reinterpret_cast<SkinState*>(base + L.skin);
    d.dvec = L.tersoff ? base + L.dvec : nullptr;
    d.bo = L.tersoff ? base + L.bo : nullptr;
    d.bcid = L.tersoff ? base + L.bcid : nullptr;
    d.P = L.tersoff ? base + L.P : nullptr;
    d.crev = L.tersoff ? reinterpret_cast<uint32_t*>(base + L.crev) : nullptr;
    d.geom = reinterpret_cast<ImageGeom*>(base + L.geom);
    d.scal = reinterpret_cast<ImageScal*>(base + L.scal);
    d.evpart = reinterpret_cast<double*>(base + L.evpart);
    d.dotpart = reinterpret_cast<double*>(base + L.dotpart);
    d.dotred = reinterpret_cast<double*>(base + L.dotred);
    d.maxpart = reinterpret_cast<double*>(base + L.maxpart);
    d.skmax = reinterpret_cast<double*>(base + L.skmax);
    d.refpart = reinterpret_cast<uint64_t*>(base + L.refpart);
    d.staging = reinterpret_cast<double*>(base + L.staging);
    d.st = reinterpret_cast<BandState*>(base + L.state);
    Launch& ln = b->launch;
    ln.bd.bands = reinterpret_cast<const BandDev*>(base + L.table);
    ln.bd.live = reinterpret_cast<const int*>(base + L.live);
    ln.bd.plan = reinterpret_cast<int*>(base + L.plan);
    ln.bd.cap = 1;
    const long long M = L.Mcap;
    size_grids(ln, M * L.ntA, M * L.ntR, M * ((L.nbcap + CFNEB_TILE - 1) / CFNEB_TILE), M, 1,
               M * ((L.N + CFNEB_TILE4 - 1) / CFNEB_TILE4), M * L.ntR4);
    ln.variants = launch_variants(d);
}

int validate(const cfneb_params* p, int64_t n_atoms)
{
    if (!p) return CFNEB_EINVAL;
    if (p->potential != CFNEB_LJ && p->potential != CFNEB_TERSOFF_C) return CFNEB_EINVAL;
    if (n_atoms < 1 || n_atoms >= CFNEB_MAX_ATOMS) return CFNEB_EINVAL;
    if (p->n_images < 3 || p->max_images < p->n_images || p->max_images > CFNEB_MAX_IMAGES)
        return CFNEB_EINVAL;
    if (p->min_images < 3) return CFNEB_EINVAL;
    if (p->cell_filter < 0 || p->cell_filter > 2) return CFNEB_EINVAL;
    if (p->nbr_cap < 1 || p->nbr_cap > 1024) return CFNEB_EINVAL;
    if (!(p->nbr_skin >= 0.0) || !(p->nbr_skin <= 2.0)) return CFNEB_EINVAL;
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(p->stress_GPa[q])) return CFNEB_EINVAL;
    if (!(p->fire_dt0 > 0.0) || !(p->fire_maxstep > 0.0)) return CFNEB_EINVAL;
    if (p->refine_every < 0 || p->ins_num < 0 || p->ins_den < 1 || p->del_num < 0 || p->del_den < 1)
        return CFNEB_EINVAL;
    const double rc = p->potential == CFNEB_LJ ? p->lj_rc : p->ts_S;
    if (!(rc > 0.0)) return CFNEB_EINVAL;
    return CFNEB_OK;
}

int image_slot(const cfneb_band* b, int k)
{
    if (k < 0 || k >= b->host_state->M) return -1;
    return b->host_state->slot[k];
}

// SoA slab (3 x ld) -> row-major (rows x 3)
void soa_to_aos(const double* soa, int ld, int rows, double* aos)
{
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < 3; ++c) aos[3 * size_t(r) + c] = soa[size_t(c) * ld + r];
}

void aos_to_soa(const double* aos, int ld, int rows, double* soa)
{
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < 3; ++c) soa[size_t(c) * ld + r] = aos[3 * size_t(r) + c];
}

// Refinement runs on the steps that finish with step % refine_every == 0 (the band's
// step counter advances by one on every step that moves it, and a band that does not
// move refines nothing), so the host knows which launches can need it.
bool refine_due(const cfneb_params& p, long long step_after)
{
    return p.refine_every > 0 && step_after % p.refine_every == 0;
}

int launch_step_direct(cfneb_band* b, bool with_refine)
{
    if (with_refine)
        launch_step(b->launch, b->stream);
    else
        launch_step_core(b->launch, b->stream);
    return check_kernels(b, "step");
}

// Launch-shape tuning of the force kernels, before the step graphs are captured.
// Both grids give bit-identical results (each item is computed the same way
// whichever block takes it), so the faster is kept.  The table's moving images are
// re-evaluated from their current positions and candidate lists (what the last
// evaluation computed, so the stored forces do not change), with the candidate
// rebuild flags held back as on most steps; three repetitions of both force phases
// per grid, timed with HIP events on the table's stream.
int tune_force_grid(Launch& L, hipStream_t s)
{
    const unsigned cand[2] = {L.g[KIND_ATOM], L.g_force_tile};
    // CFNEB_FORCE_GRID=persistent|tile fixes the choice (tests, reproducible timing)
    const char* fixed = std::getenv("CFNEB_FORCE_GRID");
    if (fixed && (std::strcmp(fixed, "persistent") == 0 || std::strcmp(fixed, "tile") == 0)) {
        L.g_force = cand[fixed[0] == 'p' ? 0 : 1];
        return CFNEB_OK;
    }
    if (cand[0] == cand[1]) {
        L.g_force = cand[0];
        return CFNEB_OK;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CFNEB_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CFNEB_EHIP;
    }
    int rc = CFNEB_OK;
    float best = 0.0f;
    unsigned pick = L.g_force_tile;
    launch_plan(L, 0, 1, s);
    launch_skin_hold(L, 1, s);
    for (int c = 0; c < 2 && rc == CFNEB_OK; ++c) {
        L.g_force = cand[c];
        launch_force_stage(L, 0, 0, s);  // warm-up
        launch_force_stage(L, 0, 1, s);
        if (hipEventRecord(e0, s) != hipSuccess) rc = CFNEB_EHIP;
        for (int r = 0; r < 3; ++r) {
            launch_force_stage(L, 0, 0, s);
            launch_force_stage(L, 0, 1, s);
        }
        float ms = 0.0f;
        if (rc != CFNEB_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
            rc = CFNEB_EHIP;
        else if (c == 0 || ms < best) {
            best = ms;
            pick = cand[c];
        }
    }
    launch_skin_hold(L, 0, s);
    L.g_force = pick;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int capture_band_graphs(cfneb_band* b)
{
    if (tune_force_grid(b->launch, b->stream) != CFNEB_OK) return fail(b, CFNEB_EHIP, "tuning");
    HIP_TRY(b, hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeRelaxed));
    launch_step(b->launch, b->capture_stream);
    HIP_TRY(b, hipStreamEndCapture(b->capture_stream, &b->graph));
    HIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    HIP_TRY(b, hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeRelaxed));
    launch_step_core(b->launch, b->capture_stream);
    HIP_TRY(b, hipStreamEndCapture(b->capture_stream, &b->graph_core));
    HIP_TRY(b, hipGraphInstantiate(&b->exec_core, b->graph_core, nullptr, nullptr, 0));
    return CFNEB_OK;
}

void drop_band_graphs(cfneb_band* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec_core) (void)hipGraphExecDestroy(b->exec_core);
    if (b->graph_core) (void)hipGraphDestroy(b->graph_core);
    b->exec = b->exec_core = nullptr;
    b->graph = b->graph_core = nullptr;
}

// Both step graphs, or neither (a failed capture leaves none behind).
int ensure_graph(cfneb_band* b)
{
    if ((b->exec && b->exec_core) || !b->use_graph) return CFNEB_OK;
    drop_band_graphs(b);
    const int rc = capture_band_graphs(b);
    if (rc != CFNEB_OK) drop_band_graphs(b);
    return rc;
}

}  // namespace

extern "C" {

int cfneb_params_default(int potential, cfneb_params* out)
{
    if (!out || (potential != CFNEB_LJ && potential != CFNEB_TERSOFF_C)) return CFNEB_EINVAL;
    std::memset(out, 0, sizeof(*out));
    cfneb_params& p = *out;
    p.potential = potential;
    p.force_fp64 = 0;
    p.lj_eps = 1.0;
    p.lj_sigma = 1.0;
    p.lj_rc = 2.5;
    p.lj_shift = 1;
    p.ts_A = 1393.6;
    p.ts_B = 346.74;
    p.ts_lambda1 = 3.4879;
    p.ts_lambda2 = 2.2119;
    p.ts_beta = 1.5724e-7;
    p.ts_n = 0.72751;
    p.ts_c = 38049.0;
    p.ts_d = 4.3484;
    p.ts_h = -0.57058;
    p.ts_R = 1.8;
    p.ts_S = 2.1;
    p.n_images = 7;
    p.max_images = 7;
    p.min_images = 3;
    p.k_spring = 1.0;
    p.climb_after = 50;
    p.cell_filter = 2;
    p.cell_factor = 0.0;
    p.b_force_scale = 1.0;
    p.pressure_GPa = 0.0;
    p.fire_dt0 = potential == CFNEB_LJ ? 0.005 : 0.05;
    p.fire_dtmax = 10.0 * p.fire_dt0;
    p.fire_maxstep = 0.1;
    p.fire_nmin = 5;
    p.fire_finc = 1.1;
    p.fire_fdec = 0.5;
    p.fire_astart = 0.1;
    p.fire_fa = 0.99;
    p.refine_every = 0;
    p.ins_num = 9;
    p.ins_den = 4;
    p.del_num = 1;
    p.del_den = 4;
    p.nbr_cap = potential == CFNEB_LJ ? 128 : 16;
    p.nbr_skin = 0.3;
    for (int q = 0; q < 6; ++q) p.stress_GPa[q] = 0.0;
    return CFNEB_OK;
}

int cfneb_band_bytes(const cfneb_params* p, int64_t n_atoms, int max_images, size_t* bytes)
{
    if (!bytes) return CFNEB_EINVAL;
    const int rc = validate(p, n_atoms);
    if (rc != CFNEB_OK) return rc;
    Layout L;
    if (!make_layout(p, n_atoms, max_images > 0 ? max_images : p->max_images, &L)) return CFNEB_EINVAL;
    *bytes = L.total;
    return CFNEB_OK;
}

}  // extern "C"

namespace {

// Device set-up of a band whose handle, host state and layout are in place: clear
// the workspace, upload the endpoints, build and evaluate every image.  A fill kernel
// clears the workspace when zero_kernel is set (no memset node if a caller captures).
int init_band(cfneb_band* b, const double* pos_init, const double* cell_init, const double* pos_final,
              const double* cell_final, void* workspace, int zero_kernel)
{
    const size_t N = size_t(b->L.N);
    if (zero_kernel)
        launch_fill_zero(workspace, b->L.total, b->stream);
    else
        HIP_TRY(b, hipMemsetAsync(workspace, 0, b->L.total, b->stream));
    // upload the endpoints to the staging area: RA | RB | hA | hB
    double* stg = b->d.staging;
    HIP_TRY(b, hipMemcpyAsync(stg, pos_init, 3 * N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(b, hipMemcpyAsync(stg + 3 * N, pos_final, 3 * N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(b, hipMemcpyAsync(stg + 6 * N, cell_init, 9 * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(b, hipMemcpyAsync(stg + 6 * N + 9, cell_final, 9 * sizeof(double), hipMemcpyHostToDevice, b->stream));
    static const int one = 1;
    HIP_TRY(b, hipMemcpyAsync(const_cast<BandDev*>(b->launch.bd.bands), &b->d, sizeof(BandDev),
                              hipMemcpyHostToDevice, b->stream));
    HIP_TRY(b, hipMemcpyAsync(const_cast<int*>(b->launch.bd.live), &one, sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
    launch_init_endpoints(b->d, b->stream);
    launch_init_images(b->d, b->p.n_images, b->stream);
    launch_init_state(b->d, b->p.n_images, b->stream);
    launch_evaluate(b->launch, 1, b->stream);
    int rc = check_kernels(b, "create");
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    if (b->host_state->err != 0) return b->host_state->err;
    return CFNEB_OK;
}

int create_impl(const cfneb_params* p, int64_t n_atoms, const double* pos_init, const double* cell_init,
                const double* pos_final, const double* cell_final, void* workspace,
                size_t workspace_bytes, void* hip_stream, int relax, cfneb_band** out)
{
    if (!out || !pos_init || !cell_init || !pos_final || !cell_final || !workspace) return CFNEB_EINVAL;
    *out = nullptr;
    int rc = validate(p, n_atoms);
    if (rc != CFNEB_OK) return rc;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return CFNEB_EINVAL;
    auto* b = new (std::nothrow) cfneb_band();
    if (!b) return CFNEB_ENOMEM;
    b->p = *p;
    if (!make_layout(p, n_atoms, p->max_images, &b->L)) {
        delete b;
        return CFNEB_EINVAL;
    }
    if (workspace_bytes < b->L.total) {
        delete b;
        return CFNEB_ENOMEM;
    }
    const char* ng = std::getenv("CFNEB_NO_GRAPH");
    b->use_graph = !(ng && ng[0] == '1');
    b->stream = static_cast<hipStream_t>(hip_stream);
    fill_dev(b, workspace, cell_init, relax);
    auto bail = [&](int code) {
        cfneb_destroy(b);
        return code;
    };
    if (hipHostMalloc(reinterpret_cast<void**>(&b->host_state), sizeof(BandState), hipHostMallocDefault) !=
        hipSuccess)
        return bail(CFNEB_EHIP);
    if (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(CFNEB_EHIP);
    rc = init_band(b, pos_init, cell_init, pos_final, cell_final, workspace, 0);
    if (rc != CFNEB_OK) return bail(rc);
    *out = b;
    return CFNEB_OK;
}

// One moving image between two fixed copies of itself, no projection, no climbing
// image, no refinement: FIRE on (R~, c_f B) down the generalized force.
cfneb_params relax_params(const cfneb_params* p)
{
    cfneb_params q = *p;
    q.n_images = 3;
    q.max_images = 3;
    q.min_images = 3;
    q.climb_after = -1;
    q.refine_every = 0;
    return q;
}

}  // namespace

extern "C" {

int cfneb_create_band(const cfneb_params* p, int64_t n_atoms, const int32_t* types,
                      const double* pos_init, const double* cell_init, const double* pos_final,
                      const double* cell_final, void* workspace, size_t workspace_bytes,
                      void* hip_stream, cfneb_band** out)
{
    (void)types;
    return create_impl(p, n_atoms, pos_init, cell_init, pos_final, cell_final, workspace, workspace_bytes,
                       hip_stream, 0, out);
}

int cfneb_relax(const cfneb_params* p, int64_t n_atoms, const int32_t* types, double* pos, double* cell,
                int max_steps, double f_tol, void* workspace, size_t workspace_bytes, void* hip_stream,
                int* steps_done, double* fmax, int* converged)
{
    (void)types;
    if (!p || !pos || !cell || max_steps < 0) return CFNEB_EINVAL;
    const cfneb_params q = relax_params(p);
    cfneb_band* b = nullptr;
    int rc = create_impl(&q, n_atoms, pos, cell, pos, cell, workspace, workspace_bytes, hip_stream, 1, &b);
    if (rc != CFNEB_OK) return rc;
    int conv = 0;
    rc = cfneb_step(b, max_steps, f_tol, steps_done, fmax, &conv);
    if (rc == CFNEB_OK) rc = cfneb_get_image(b, 1, pos, cell);
    if (converged) *converged = conv;
    cfneb_destroy(b);
    return rc;
}

}  // extern "C"

// ------------------------------------------------- relaxation without allocation
// Device memory of cfneb_relax_noalloc: one array per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy: the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[CFNEB_RELAX_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array (looked up on the first call on that
// device, with it current); nullptr on failure.
void* scratch_of_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int cfneb_relax_noalloc(const cfneb_params* p, int64_t n_atoms, const int32_t* types, double* pos, double* cell,
                        int max_steps, double f_tol, void* hip_stream, int* steps_done, double* fmax,
                        int* converged)
{
    (void)types;
    if (!p || !pos || !cell || max_steps < 0) return CFNEB_EINVAL;
    const cfneb_params q = relax_params(p);
    int rc = validate(&q, n_atoms);
    if (rc != CFNEB_OK) return rc;
    // the band lives on this stack frame: handle, pageable host state, no graphs, no
    // capture stream, kernels launched one by one
    cfneb_band b;
    b.p = q;
    if (!make_layout(&q, n_atoms, q.max_images, &b.L)) return CFNEB_EINVAL;
    if (b.L.total > size_t(CFNEB_RELAX_SCRATCH_BYTES)) return CFNEB_ENOMEM;
    void* ws = scratch_of_current_device();
    if (!ws) return CFNEB_EHIP;
    BandState host_state;
    b.host_state = &host_state;
    b.use_graph = false;
    b.stream = static_cast<hipStream_t>(hip_stream);
    fill_dev(&b, ws, cell, 1);
    rc = init_band(&b, pos, cell, pos, cell, ws, 1);
    int conv = 0;
    if (rc == CFNEB_OK) rc = cfneb_step(&b, max_steps, f_tol, steps_done, fmax, &conv);
    if (rc == CFNEB_OK) rc = cfneb_get_image(&b, 1, pos, cell);
    if (converged) *converged = conv;
    (void)hipStreamSynchronize(b.stream);
    b.host_state = nullptr;  // nothing of this band is freed: it owns nothing
    return rc;
}

int cfneb_step(cfneb_band* b, int max_steps, double f_tol, int* steps_done, double* fmax,
               int* converged)
{
    if (!b || max_steps < 0) return CFNEB_EINVAL;
    launch_begin_call(b->launch, f_tol, -1, b->stream);
    int rc = ensure_graph(b);
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    long long next = b->host_state->step + 1;  // step count after the next launch moves the band
    const int check_every = 16;
    for (int s = 0; s < max_steps; ++s, ++next) {
        const bool with_refine = refine_due(b->p, next);
        if (b->exec) {
            HIP_TRY(b, hipGraphLaunch(with_refine ? b->exec : b->exec_core, b->stream));
        } else {
            rc = launch_step_direct(b, with_refine);
            if (rc != CFNEB_OK) return rc;
        }
        if ((s + 1) % check_every == 0 && s + 1 < max_steps) {
            rc = read_state(b);
            if (rc != CFNEB_OK) return rc;
            if (b->host_state->done || b->host_state->err) break;
            next = b->host_state->step;  // the loop's ++next makes it the next launch's
        }
    }
    launch_flush_move(b->launch, b->stream);  // the last step's move
    rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const BandState& st = *b->host_state;
    if (steps_done) *steps_done = st.steps_call;
    if (fmax) *fmax = st.fmax;
    if (converged) *converged = st.done;
    if (st.err != 0) return fail(b, st.err, "cfneb_step");
    return CFNEB_OK;
}

int cfneb_step_profiled(cfneb_band* b, int max_steps, double f_tol, int* steps_done, double* fmax,
                        int* converged, double* phase_ms, int nphase)
{
    if (!b || max_steps < 0 || nphase < 0 || nphase > CFNEB_NPHASE || (nphase > 0 && !phase_ms))
        return CFNEB_EINVAL;
    launch_begin_call(b->launch, f_tol, -1, b->stream);
    const int NP = CFNEB_NPHASE;
    // one event before every phase and one after the last, for every step
    std::vector<hipEvent_t> ev(size_t(max_steps) * (NP + 1), nullptr);
    int rc = CFNEB_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            rc = fail(b, CFNEB_EHIP, "hipEventCreate");
            break;
        }
    const Launch& d = b->launch;
    hipStream_t s = b->stream;
    if (rc == CFNEB_OK) rc = read_state(b);
    const long long step0 = rc == CFNEB_OK ? b->host_state->step : 0;
    for (int st = 0; st < max_steps && rc == CFNEB_OK; ++st) {
        hipEvent_t* e = ev.data() + size_t(st) * (NP + 1);
        const bool with_refine = refine_due(b->p, step0 + st + 1);
        for (int ph = 0; ph < NP; ++ph) {
            (void)hipEventRecord(e[ph], s);
            switch (ph) {
            case CFNEB_PH_GEOM:
                launch_geom(d, 0, s);  // also writes the plan
                break;
            case CFNEB_PH_SKIN: launch_skin(d, 0, s); break;
            case CFNEB_PH_BINS: launch_bins(d, 0, s); break;
            case CFNEB_PH_NLIST: launch_list(d, 0, s); break;
            case CFNEB_PH_FILTER: launch_filter(d, 0, s); break;
            case CFNEB_PH_FORCE0: launch_force_stage(d, 0, 0, s); break;
            case CFNEB_PH_FORCE1: launch_force_stage(d, 0, 1, s); break;
            case CFNEB_PH_FORCE2: launch_force_stage(d, 0, 2, s); break;
            case CFNEB_PH_REDUCE: break;  // inside the band dots pass
            case CFNEB_PH_DOTS: launch_dots(d, s); break;
            case CFNEB_PH_SCALARS: launch_scalars(d, s); break;
            case CFNEB_PH_UPDATE: launch_update(d, s); break;
            case CFNEB_PH_FINALIZE: launch_finalize(d, s); break;
            case CFNEB_PH_MOVE: break;  // applied by the next step's geometry and skin passes
            case CFNEB_PH_REFINE:
                if (with_refine) {
                    launch_flush_move(d, s);
                    launch_refine(d, 0, s);
                }
                break;
            default: break;
            }
        }
        (void)hipEventRecord(e[NP], s);
        rc = check_kernels(b, "step_profiled");
    }
    launch_flush_move(d, s);  // the last step's move
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc == CFNEB_OK) {
        for (int ph = 0; ph < nphase; ++ph) phase_ms[ph] = 0.0;
        for (int st = 0; st < max_steps; ++st) {
            hipEvent_t* e = ev.data() + size_t(st) * (NP + 1);
            for (int ph = 0; ph < nphase; ++ph) {
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, e[ph], e[ph + 1]) == hipSuccess) phase_ms[ph] += ms;
            }
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != CFNEB_OK) return rc;
    const BandState& st = *b->host_state;
    if (steps_done) *steps_done = st.steps_call;
    if (fmax) *fmax = st.fmax;
    if (converged) *converged = st.done;
    if (st.err != 0) return fail(b, st.err, "cfneb_step_profiled");
    return CFNEB_OK;
}

int cfneb_refine(cfneb_band* b, int* inserted_at, int* deleted_at)
{
    if (!b) return CFNEB_EINVAL;
    launch_begin_call(b->launch, 0.0, -1, b->stream);
    launch_plan(b->launch, 0, 1, b->stream);
    launch_refine(b->launch, 1, b->stream);
    int rc = check_kernels(b, "refine");
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    if (inserted_at) *inserted_at = b->host_state->ins;
    if (deleted_at) *deleted_at = b->host_state->del;
    if (b->host_state->err != 0) return fail(b, b->host_state->err, "cfneb_refine");
    return CFNEB_OK;
}

int cfneb_energies(const cfneb_band* cb, double* H, int cap, int* n_images, double* barrier,
                   int* ci_index, double* path_coord)
{
    auto* b = const_cast<cfneb_band*>(cb);
    if (!b) return CFNEB_EINVAL;
    launch_plan(b->launch, 0, 1, b->stream);
    launch_readout(b->launch, b->stream);
    int rc = check_kernels(b, "readout");
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const BandState& st = *b->host_state;
    if (n_images) *n_images = st.M;
    if (H && cap < st.M) return fail(b, CFNEB_EINVAL, "cfneb_energies: cap");
    for (int k = 0; k < st.M; ++k) {
        if (H) H[k] = st.Hlog[k];
        if (path_coord) path_coord[k] = st.xi[k];
    }
    if (barrier) *barrier = st.barrier;
    if (ci_index) *ci_index = st.ci;
    return CFNEB_OK;
}

int cfneb_profile(cfneb_band* b, int n_samples, double* s, double* H, double* slope, int cap, int* n_images,
                  double* samples, double* barrier, double* xi_max)
{
    if (!b) return CFNEB_EINVAL;
    if (n_samples < 0 || n_samples == 1 || n_samples > CFNEB_PROFILE_SAMPLES || (n_samples > 0 && !samples))
        return fail(b, CFNEB_EINVAL, "cfneb_profile: n_samples");
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    BandState& st = *b->host_state;
    if (st.err != 0) return fail(b, st.err, "cfneb_profile");
    if ((s || H || slope) && cap < st.M) return fail(b, CFNEB_EINVAL, "cfneb_profile: cap");
    if (st.done) {
        // the evaluation kernels skip a band that converged in its last call; the flag
        // only describes that call and is cleared by the next one anyway
        st.done = 0;
        rc = write_state(b);
        if (rc != CFNEB_OK) return rc;
    }
    launch_evaluate(b->launch, 1, b->stream);
    launch_profile(b->launch, n_samples, b->stream);
    rc = check_kernels(b, "profile");
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    if (st.err != 0) return fail(b, st.err, "cfneb_profile");
    const int M = st.M;
    std::vector<double> out(size_t(CFNEB_PROF_SAMP) + size_t(n_samples));
    HIP_TRY(b, hipMemcpyAsync(out.data(), b->d.staging, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    if (n_images) *n_images = M;
    for (int k = 0; k < M; ++k) {
        if (s) s[k] = out[CFNEB_PROF_S + k];
        if (H) H[k] = out[CFNEB_PROF_H + k];
        if (slope) slope[k] = out[CFNEB_PROF_SLOPE + k];
    }
    for (int j = 0; j < n_samples; ++j) samples[j] = out[CFNEB_PROF_SAMP + j];
    if (barrier) *barrier = out[CFNEB_PROF_OUT];
    if (xi_max) *xi_max = out[CFNEB_PROF_OUT + 1];
    return CFNEB_OK;
}

int cfneb_get_image(const cfneb_band* cb, int k, double* pos, double* cell)
{
    auto* b = const_cast<cfneb_band*>(cb);
    if (!b) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    if (image_slot(b, k) < 0) return CFNEB_EINVAL;
    launch_image_positions(b->d, k, b->stream);
    rc = check_kernels(b, "get_image");
    if (rc != CFNEB_OK) return rc;
    const size_t N = size_t(b->L.N);
    if (pos)
        HIP_TRY(b, hipMemcpyAsync(pos, b->d.staging, 3 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (cell)
        HIP_TRY(b, hipMemcpyAsync(cell, b->d.staging + 3 * N, 9 * sizeof(double), hipMemcpyDeviceToHost,
                                  b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    return CFNEB_OK;
}

int cfneb_get_state(const cfneb_band* cb, double* X, double* v, int cap_images, int* n_images,
                    cfneb_fire_state* fs)
{
    auto* b = const_cast<cfneb_band*>(cb);
    if (!b) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const BandState st = *b->host_state;
    if (n_images) *n_images = st.M;
    if ((X || v) && cap_images < st.M) return fail(b, CFNEB_EINVAL, "cfneb_get_state: cap");
    const int rows = b->L.N + 3, ld = b->L.ld;
    std::vector<double> slab(3 * size_t(ld));
    for (int k = 0; k < st.M; ++k) {
        const int slot = st.slot[k];
        if (X) {
            HIP_TRY(b, hipMemcpy(slab.data(), b->d.X + size_t(slot) * 3 * ld, slab.size() * 8,
                                 hipMemcpyDeviceToHost));
            soa_to_aos(slab.data(), ld, rows, X + size_t(k) * 3 * rows);
        }
        if (v) {
            const double* src = b->d.V + (size_t(st.vcur) * b->L.Mcap + slot) * 3 * ld;
            HIP_TRY(b, hipMemcpy(slab.data(), src, slab.size() * 8, hipMemcpyDeviceToHost));
            soa_to_aos(slab.data(), ld, rows, v + size_t(k) * 3 * rows);
        }
    }
    if (fs) {
        fs->dt = st.dt;
        fs->alpha = st.alpha;
        fs->n_pos = st.n_pos;
        fs->fresh = st.fresh;
        fs->step = st.step;
        fs->ci = st.ci;
        fs->image_steps = st.image_steps;
    }
    return CFNEB_OK;
}

int cfneb_set_state(cfneb_band* b, int n_images, const double* X, const double* v,
                    const cfneb_fire_state* fs)
{
    if (!b || !X || !fs || n_images < 3 || n_images > b->L.Mcap) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const int rows = b->L.N + 3, ld = b->L.ld;
    std::vector<double> slab(3 * size_t(ld), 0.0);
    for (int k = 0; k < n_images; ++k) {
        aos_to_soa(X + size_t(k) * 3 * rows, ld, rows, slab.data());
        HIP_TRY(b, hipMemcpy(b->d.X + size_t(k) * 3 * ld, slab.data(), slab.size() * 8, hipMemcpyHostToDevice));
        std::fill(slab.begin(), slab.end(), 0.0);
        if (v && k > 0 && k < n_images - 1) aos_to_soa(v + size_t(k) * 3 * rows, ld, rows, slab.data());
        HIP_TRY(b, hipMemcpy(b->d.V + size_t(k) * 3 * ld, slab.data(), slab.size() * 8, hipMemcpyHostToDevice));
        std::fill(slab.begin(), slab.end(), 0.0);
    }
    // new positions: every candidate list is rebuilt at the evaluation below
    HIP_TRY(b, hipMemset(b->d.skst, 0, size_t(b->L.Mcap) * sizeof(SkinState)));
    BandState& st = *b->host_state;
    st.M = n_images;
    for (int k = 0; k < CFNEB_MAX_IMAGES; ++k) st.slot[k] = k < b->L.Mcap ? k : 0;
    st.vcur = 0;
    st.dt = fs->dt;
    st.alpha = fs->alpha;
    st.n_pos = fs->n_pos;
    st.fresh = fs->fresh;
    st.step = fs->step;
    st.ci = fs->ci;
    st.done = 0;
    st.err = 0;
    st.refine_due = 0;
    rc = write_state(b);
    if (rc != CFNEB_OK) return rc;
    launch_evaluate(b->launch, 1, b->stream);
    rc = check_kernels(b, "set_state");
    if (rc == CFNEB_OK) rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    if (b->host_state->err != 0) return fail(b, b->host_state->err, "cfneb_set_state");
    return CFNEB_OK;
}

int cfneb_image_data(const cfneb_band* cb, int k, double* E, double* H, double* V, double* F,
                     double* Fg, double* Fneb, double* R, double* h)
{
    auto* b = const_cast<cfneb_band*>(cb);
    if (!b) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const int slot = image_slot(b, k);
    if (slot < 0) return CFNEB_EINVAL;
    const int N = b->L.N, ld = b->L.ld;
    ImageScal sc;
    ImageGeom g;
    HIP_TRY(b, hipMemcpy(&sc, b->d.scal + slot, sizeof(sc), hipMemcpyDeviceToHost));
    HIP_TRY(b, hipMemcpy(&g, b->d.geom + slot, sizeof(g), hipMemcpyDeviceToHost));
    if (E) *E = sc.E;
    if (H) *H = sc.H;
    if (V) std::memcpy(V, sc.V, 9 * sizeof(double));
    if (h) std::memcpy(h, g.h, 9 * sizeof(double));
    std::vector<double> slab(3 * size_t(ld));
    if (F || Fg) {
        std::vector<double> fa(3 * size_t(N));
        if (b->L.fp64) {
            HIP_TRY(b, hipMemcpy(slab.data(), static_cast<double*>(b->d.F) + size_t(slot) * 3 * ld, slab.size() * 8,
                                 hipMemcpyDeviceToHost));
        } else {
            std::vector<float> sf(3 * size_t(ld));
            HIP_TRY(b, hipMemcpy(sf.data(), static_cast<float*>(b->d.F) + size_t(slot) * 3 * ld, sf.size() * 4,
                                 hipMemcpyDeviceToHost));
            for (size_t q = 0; q < sf.size(); ++q) slab[q] = double(sf[q]);
        }
        soa_to_aos(slab.data(), ld, N, fa.data());
        if (F) std::memcpy(F, fa.data(), fa.size() * sizeof(double));
        if (Fg) {
            // generalized force rows as the band kernels form them: F D^T, then the
            // lattice force rows
            for (int i = 0; i < N; ++i)
                for (int c = 0; c < 3; ++c)
                    Fg[3 * size_t(i) + c] = fa[3 * size_t(i)] * g.D[3 * c] + fa[3 * size_t(i) + 1] * g.D[3 * c + 1] +
                                            fa[3 * size_t(i) + 2] * g.D[3 * c + 2];
            std::memcpy(Fg + 3 * size_t(N), sc.Fcell, 9 * sizeof(double));
        }
    }
    if (Fneb) {
        HIP_TRY(b, hipMemcpy(slab.data(), b->d.FN + size_t(slot) * 3 * ld, slab.size() * 8, hipMemcpyDeviceToHost));
        soa_to_aos(slab.data(), ld, N + 3, Fneb);
    }
    if (R) {
        // packed (x, y, z) records: the first N are the caller's layout
        HIP_TRY(b, hipMemcpy(R, b->d.R + size_t(slot) * 3 * ld, 3 * size_t(N) * 8, hipMemcpyDeviceToHost));
    }
    return CFNEB_OK;
}

int cfneb_record_neb_force(cfneb_band* b, int on)
{
    if (!b) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    b->host_state->record_fneb = on ? 1 : 0;
    return write_state(b);
}

int cfneb_neighbours(const cfneb_band* cb, int k, int32_t* cnt, int32_t* ent, int64_t cap, int64_t* total)
{
    auto* b = const_cast<cfneb_band*>(cb);
    if (!b || !cnt) return CFNEB_EINVAL;
    int rc = read_state(b);
    if (rc != CFNEB_OK) return rc;
    const int slot = image_slot(b, k);
    if (slot < 0) return CFNEB_EINVAL;
    const size_t N = size_t(b->L.N), C = size_t(b->L.cap);
    launch_neighbour_lists(b->launch, b->stream);
    HIP_TRY(b, hipGetLastError());
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    std::vector<uint32_t> nb(C * N);
    HIP_TRY(b, hipMemcpy(cnt, b->d.ncnt + size_t(slot) * N, N * 4, hipMemcpyDeviceToHost));
    HIP_TRY(b, hipMemcpy(nb.data(), b->d.nbr + size_t(slot) * C * N, nb.size() * 4, hipMemcpyDeviceToHost));
    int64_t t = 0;
    for (size_t i = 0; i < N; ++i) {
        const int c = cnt[i] < int(C) ? cnt[i] : int(C);
        for (int e = 0; e < c; ++e, ++t) {
            if (t >= cap || !ent) continue;
            const uint32_t v = nb[size_t(e) * N + i];
            ent[4 * t + 0] = int32_t(v & 0xFFFFFu);
            ent[4 * t + 1] = int32_t((v >> 20) & 0xFu) - 8;
            ent[4 * t + 2] = int32_t((v >> 24) & 0xFu) - 8;
            ent[4 * t + 3] = int32_t((v >> 28) & 0xFu) - 8;
        }
    }
    if (total) *total = t;
    return CFNEB_OK;
}

int cfneb_destroy(cfneb_band* b)
{
    if (!b) return CFNEB_EINVAL;
    if (b->stream || b->host_state) (void)hipStreamSynchronize(b->stream);
    drop_band_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->host_state) (void)hipHostFree(b->host_state);
    delete b;
    return CFNEB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
// A batch is a table of bands stepped together: every phase of the step is one
// persistent launch over the items of all live bands (sizes may differ), captured
// once in a graph; attaching or detaching a band rewrites the device table only.
struct cfneb_batch {
    int cap = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    Launch launch;
    BandDev* table = nullptr;
    int* live = nullptr;
    int* plan = nullptr;
    int* summary = nullptr;
    int* host_summary = nullptr;  // pinned, per table entry: done, err, steps this call, step
    std::vector<cfneb_band*> bands;
    std::vector<char> owned;  // 1: the band was made by cfneb_batch_add and is the batch's
    unsigned graph_variants = 0;
    hipGraph_t graph = nullptr;  // a whole step
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_core = nullptr;  // a step without the refinement phase
    hipGraphExec_t exec_core = nullptr;
    bool use_graph = true;
};

namespace {

struct BatchLayout {
    size_t table, live, plan, summary, total;
};

BatchLayout batch_layout(int cap)
{
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.table = take(size_t(cap) * sizeof(BandDev));
    L.live = take(size_t(cap) * sizeof(int));
    L.plan = take((size_t(NKIND) * (cap + 1) + 2) * sizeof(int));
    L.summary = take(size_t(cap) * 4 * sizeof(int));
    L.total = off;
    return L;
}

void drop_graph(cfneb_batch* B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->exec_core) (void)hipGraphExecDestroy(B->exec_core);
    if (B->graph_core) (void)hipGraphDestroy(B->graph_core);
    B->exec = B->exec_core = nullptr;
    B->graph = B->graph_core = nullptr;
}

int capture_batch_graphs(cfneb_batch* B)
{
    if (tune_force_grid(B->launch, B->stream) != CFNEB_OK) return CFNEB_EHIP;
    if (hipStreamBeginCapture(B->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return CFNEB_EHIP;
    launch_step(B->launch, B->capture_stream);
    if (hipStreamEndCapture(B->capture_stream, &B->graph) != hipSuccess ||
        hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess)
        return CFNEB_EHIP;
    if (hipStreamBeginCapture(B->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return CFNEB_EHIP;
    launch_step_core(B->launch, B->capture_stream);
    if (hipStreamEndCapture(B->capture_stream, &B->graph_core) != hipSuccess ||
        hipGraphInstantiate(&B->exec_core, B->graph_core, nullptr, nullptr, 0) != hipSuccess)
        return CFNEB_EHIP;
    return CFNEB_OK;
}

// Whether the step after `ahead` more launches can refine any band of the table:
// summary field 3 of a band is its step count at the last summary.
bool batch_refine_due(const cfneb_batch* B, int ahead)
{
    for (int q = 0; q < B->cap; ++q) {
        const cfneb_band* bb = B->bands[q];
        if (!bb) continue;
        const int* o = B->host_summary + 4 * q;
        if (o[0] || o[1]) continue;  // stopped: nothing to refine
        if (refine_due(bb->p, (long long)o[3] + ahead + 1)) return true;
    }
    return false;
}

int read_summary(cfneb_batch* B)
{
    launch_summary(B->launch, B->summary, B->stream);
    if (hipMemcpyAsync(B->host_summary, B->summary, size_t(B->cap) * 4 * sizeof(int), hipMemcpyDeviceToHost,
                       B->stream) != hipSuccess)
        return CFNEB_EHIP;
    if (hipStreamSynchronize(B->stream) != hipSuccess) return CFNEB_EHIP;
    return CFNEB_OK;
}

}  // namespace

extern "C" {

int cfneb_batch_bytes(int max_bands, size_t* bytes)
{
    if (!bytes || max_bands < 1 || max_bands > CFNEB_MAX_BANDS) return CFNEB_EINVAL;
    *bytes = batch_layout(max_bands).total;
    return CFNEB_OK;
}

int cfneb_batch_create(int max_bands, void* workspace, size_t workspace_bytes, void* hip_stream,
                       cfneb_batch** out)
{
    if (!out || !workspace || max_bands < 1 || max_bands > CFNEB_MAX_BANDS) return CFNEB_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return CFNEB_EINVAL;
    const BatchLayout BL = batch_layout(max_bands);
    if (workspace_bytes < BL.total) return CFNEB_ENOMEM;
    auto* B = new (std::nothrow) cfneb_batch();
    if (!B) return CFNEB_ENOMEM;
    B->cap = max_bands;
    B->stream = static_cast<hipStream_t>(hip_stream);
    char* base = static_cast<char*>(workspace);
    B->table = reinterpret_cast<BandDev*>(base + BL.table);
    B->live = reinterpret_cast<int*>(base + BL.live);
    B->plan = reinterpret_cast<int*>(base + BL.plan);
    B->summary = reinterpret_cast<int*>(base + BL.summary);
    B->bands.assign(max_bands, nullptr);
    B->owned.assign(max_bands, 0);
    B->launch.bd.bands = B->table;
    B->launch.bd.live = B->live;
    B->launch.bd.plan = B->plan;
    B->launch.bd.cap = max_bands;
    // any band may join later: size the persistent grids for the whole chip
    size_grids(B->launch, 1LL << 40, 1LL << 40, 1LL << 40, 1LL << 40, max_bands, 1LL << 40, 1LL << 40);
    B->launch.variants = 0;
    const char* ng = std::getenv("CFNEB_NO_GRAPH");
    B->use_graph = !(ng && ng[0] == '1');
    if (hipHostMalloc(reinterpret_cast<void**>(&B->host_summary), size_t(max_bands) * 4 * sizeof(int),
                      hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&B->capture_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMemsetAsync(workspace, 0, BL.total, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess) {
        cfneb_batch_destroy(B);
        return CFNEB_EHIP;
    }
    *out = B;
    return CFNEB_OK;
}

int cfneb_batch_attach(cfneb_batch* B, cfneb_band* band, int* slot)
{
    if (!B || !band) return CFNEB_EINVAL;
    int s = -1;
    for (int q = 0; q < B->cap; ++q) {
        if (B->bands[q] == band) return CFNEB_EINVAL;
        if (s < 0 && !B->bands[q]) s = q;
    }
    if (s < 0) return CFNEB_ECAPACITY;
    static const int one = 1;
    if (hipStreamSynchronize(band->stream) != hipSuccess ||
        hipMemcpyAsync(B->table + s, &band->d, sizeof(BandDev), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipMemcpyAsync(B->live + s, &one, sizeof(int), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess)
        return CFNEB_EHIP;
    B->bands[s] = band;
    unsigned v = 0;
    for (auto* bb : B->bands)
        if (bb) v |= launch_variants(bb->d);
    B->launch.variants = v;
    if (slot) *slot = s;
    return CFNEB_OK;
}

int cfneb_batch_detach(cfneb_batch* B, int slot)
{
    if (!B || slot < 0 || slot >= B->cap || !B->bands[slot]) return CFNEB_EINVAL;
    static const int zero = 0;
    if (hipMemcpyAsync(B->live + slot, &zero, sizeof(int), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess)
        return CFNEB_EHIP;
    B->bands[slot] = nullptr;
    B->owned[slot] = 0;  // a band of cfneb_batch_add detached here passes to the caller
    unsigned v = 0;
    for (auto* bb : B->bands)
        if (bb) v |= launch_variants(bb->d);
    B->launch.variants = v;
    return CFNEB_OK;
}

int cfneb_batch_add(cfneb_batch* B, const cfneb_params* p, int64_t n_atoms, const int32_t* types,
                    const double* pos_init, const double* cell_init, const double* pos_final,
                    const double* cell_final, void* workspace, size_t workspace_bytes, int* slot)
{
    if (!B) return CFNEB_EINVAL;
    int free_slot = -1;
    for (int q = 0; q < B->cap && free_slot < 0; ++q)
        if (!B->bands[q]) free_slot = q;
    if (free_slot < 0) return CFNEB_ECAPACITY;
    cfneb_band* band = nullptr;
    int rc = cfneb_create_band(p, n_atoms, types, pos_init, cell_init, pos_final, cell_final, workspace,
                               workspace_bytes, B->stream, &band);
    if (rc != CFNEB_OK) return rc;
    int s = -1;
    rc = cfneb_batch_attach(B, band, &s);
    if (rc != CFNEB_OK) {
        cfneb_destroy(band);
        return rc;
    }
    B->owned[s] = 1;
    if (slot) *slot = s;
    return CFNEB_OK;
}

int cfneb_batch_remove(cfneb_batch* B, int slot)
{
    if (!B || slot < 0 || slot >= B->cap || !B->bands[slot]) return CFNEB_EINVAL;
    cfneb_band* band = B->bands[slot];
    const bool own = B->owned[slot] != 0;
    const int rc = cfneb_batch_detach(B, slot);
    if (rc != CFNEB_OK) return rc;
    B->owned[slot] = 0;
    if (own) cfneb_destroy(band);
    return CFNEB_OK;
}

cfneb_band* cfneb_batch_band(cfneb_batch* B, int slot)
{
    if (!B || slot < 0 || slot >= B->cap) return nullptr;
    return B->bands[slot];
}

int cfneb_batch_energies(cfneb_batch* B, int slot, double* H, int cap, int* n_images, double* barrier,
                         int* ci_index, double* path_coord)
{
    if (!B || slot < 0 || slot >= B->cap || !B->bands[slot]) return CFNEB_EINVAL;
    return cfneb_energies(B->bands[slot], H, cap, n_images, barrier, ci_index, path_coord);
}

int cfneb_batch_step(cfneb_batch* B, int max_steps, double f_tol, int* steps_done, uint8_t* converged,
                     int* errors)
{
    if (!B || max_steps < 0) return CFNEB_EINVAL;
    launch_begin_call(B->launch, f_tol, -1, B->stream);
    if (B->use_graph && (!B->exec || !B->exec_core || B->graph_variants != B->launch.variants)) {
        drop_graph(B);
        const int crc = capture_batch_graphs(B);
        if (crc != CFNEB_OK) {
            drop_graph(B);
            return crc;
        }
        B->graph_variants = B->launch.variants;
    }
    const int check_every = 16;
    int rc = read_summary(B);
    if (rc != CFNEB_OK) return rc;
    int ahead = 0;  // launches since the last summary
    for (int s = 0; s < max_steps; ++s, ++ahead) {
        const bool with_refine = batch_refine_due(B, ahead);
        if (B->exec) {
            if (hipGraphLaunch(with_refine ? B->exec : B->exec_core, B->stream) != hipSuccess) return CFNEB_EHIP;
        } else {
            if (with_refine)
                launch_step(B->launch, B->stream);
            else
                launch_step_core(B->launch, B->stream);
            if (hipGetLastError() != hipSuccess) return CFNEB_EHIP;
        }
        if ((s + 1) % check_every == 0 && s + 1 < max_steps) {
            rc = read_summary(B);
            if (rc != CFNEB_OK) return rc;
            ahead = -1;  // the loop's ++ahead makes it 0 for the next launch
            bool active = false;
            for (int q = 0; q < B->cap; ++q)
                if (B->bands[q] && !B->host_summary[4 * q] && !B->host_summary[4 * q + 1]) active = true;
            if (!active) break;
        }
    }
    launch_flush_move(B->launch, B->stream);  // the last step's moves
    rc = read_summary(B);
    if (rc != CFNEB_OK) return rc;
    for (int q = 0; q < B->cap; ++q) {
        const int* o = B->host_summary + 4 * q;
        if (steps_done) steps_done[q] = B->bands[q] ? o[2] : 0;
        if (converged) converged[q] = B->bands[q] ? uint8_t(o[0] != 0) : 0;
        if (errors) errors[q] = B->bands[q] ? o[1] : 0;
    }
    return CFNEB_OK;
}

int cfneb_batch_destroy(cfneb_batch* B)
{
    if (!B) return CFNEB_EINVAL;
    (void)hipStreamSynchronize(B->stream);
    for (int q = 0; q < B->cap; ++q)
        if (B->bands[q] && B->owned[q]) {
            cfneb_destroy(B->bands[q]);
            B->bands[q] = nullptr;
        }
    drop_graph(B);
    if (B->capture_stream) (void)hipStreamDestroy(B->capture_stream);
    if (B->host_summary) (void)hipHostFree(B->host_summary);
    delete B;
    return CFNEB_OK;
}

const char* cfneb_strerror(int code) { return err_text(code); }

const char* cfneb_last_error(const cfneb_band* b) { return b ? b->last_error.c_str() : "no band"; }

}  // extern "C"
