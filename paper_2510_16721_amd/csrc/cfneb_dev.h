// Device-side layout and helpers of the CFNEB library (gfx950).
//
// HBM layout of one band (all inside the caller's workspace, 256-B aligned):
//   X      [slot][3][ld]  FP64  generalized coordinates: rows 0..N-1 = R~ (SoA),
//                               rows N..N+2 = the three rows of c_f B
//   V      [2][slot][3][ld] FP64 FIRE velocities, ping-pong (vcur selects)
//   R      [slot][ld]     32 B  Cartesian positions R = R~ D of the last evaluation
//   S      [slot][ld]     16 B  FP32 LJ bands: fractional coordinates of R in the
//                               image's cell, wrapped to [0, 1), as 32-bit fixed point
//   F      [slot][3][ld]  T     Cartesian forces (T = float, or double for FP64 bands)
//   FN     [slot][3][ld]  FP64  NEB force (only when recording is on)
//   binfo  [slot][N]      int4  (bin, rank in bin, packed lattice image) per atom
//   bins   [slot][...]    int   counts, starts; bpos: atoms in bin order (R, packed id)
//   nbr    [slot][cap][N] u32   packed neighbour entries, entry-major (readouts only)
//   cand   [slot][ccap][N] u32  candidates within rc + skin (atom index and shifts)
//   ncnt   [slot][N]      int   neighbour count (may exceed cap: overflow)
//   dvec   [slot][cap][N] T4    Tersoff: bond vector and length (bonds past the fourth)
//   bo     [slot][cap][N] T2    Tersoff: b_ij and db/dzeta (same)
//   P      [slot][ccap][N] T4   Tersoff: dU_i/dr^ij per candidate (zero if not a bond)
//   geom / scal [slot]          per-image 3x3 geometry and reduced scalars
//   partial buffers             fixed-order block partials of every reduction
//   state                       band scalars (FIRE, slot table, flags)
// A "slot" is a physical image buffer; the slot table maps logical image k to a slot,
// so inserting or deleting an image rewrites the table, not the data.
#ifndef CFNEB_DEV_H
#define CFNEB_DEV_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "cfneb.h"

#define CFNEB_MAX_IMAGES 64
#define CFNEB_TILE 256           // threads per block of every streaming kernel
#define CFNEB_TILE4 1024         // rows (atoms) of a streaming item with 4 per thread
#define CFNEB_WAVES 4            // waves per block of CFNEB_TILE threads
#define CFNEB_NDOT 22            // band-dot partial sums per moving image and row tile
#define CFNEB_NPROF 14           // energy-profile partial sums per image and row tile
#define CFNEB_PROFILE_SAMPLES CFNEB_PROFILE_MAX_SAMPLES
// Energy-profile readout area at the start of the staging buffer (doubles): arc
// lengths s, enthalpies H and slopes dH/ds of the images, then barrier, normalized
// coordinate of the maximum and H_max, then the samples.
#define CFNEB_PROF_S 0
#define CFNEB_PROF_H CFNEB_MAX_IMAGES
#define CFNEB_PROF_SLOPE (2 * CFNEB_MAX_IMAGES)
#define CFNEB_PROF_OUT (3 * CFNEB_MAX_IMAGES)
#define CFNEB_PROF_SAMP (3 * CFNEB_MAX_IMAGES + 8)
#define CFNEB_PROF_DOUBLES (CFNEB_PROF_SAMP + CFNEB_PROFILE_SAMPLES)
#define CFNEB_MAX_SHIFT 7        // packed shifts are 4-bit offset-binary
#define CFNEB_J_BITS 20
#define CFNEB_MAX_ATOMS (1 << CFNEB_J_BITS)

namespace cfneb {

// One atom in bin order: unwrapped position and (id, lattice image) packed as
// id | (n0 + 512) << 20 | (n1 + 512) << 30 | (n2 + 512) << 40.
struct alignas(32) BinAtom {
    double x, y, z;
    long long info;
};

struct ImageGeom {
    double D[9], Dinv[9], h[9], hinv[9];
    double omega;
    double w[3];
    int nb[3];
    int reach[3];
    int sub;  // bins per rcl along each axis (2 for dense systems)
    int nbins;
    int err;
    // strain since the last candidate build: h = h_ref (I + E), and |E|_F
    double E[9];
    double enorm;
    // Fixed-point separations (FP32 LJ bands): wrap = 1 when every candidate's
    // fractional separation stays within half a cell on each axis, so the wrapped
    // 32-bit difference of two fixed-point coordinates is the separation itself; an
    // FP32 r^2 from it below r2lo is inside rc, at or above r2hi outside, and between
    // the two the exact FP64 test decides.
    int wrap;
    float r2lo, r2hi;
};

// Candidate lists of one image slot (Verlet skin).  The candidates are every pair
// closer than rc + skin at the build; a pair closer than rc now was a candidate if
// 2 max_i |R_i - R_i,ref (I + E)| + (rc + skin) |E| < skin.
struct SkinState {
    double href[9], hrefinv[9];
    int valid;                 // a candidate list exists for this slot
    int rebuild;               // this step rebuilds it
    int held;                  // rebuild, set aside while the force grid is tuned
};

struct ImageScal {
    double E, H;
    double V[9];
    double Fcell[9];  // generalized force on the three cell rows
};

struct BandState {
    int M;                         // current number of images
    int slot[CFNEB_MAX_IMAGES];    // logical image -> physical slot
    int vcur;                      // current velocity buffer
    int step;                      // moves taken in total
    long long image_steps;         // sum over moves of the number of moving images
    int steps_call;                // moves taken in the current cfneb_step call
    int done;                      // converged in the current call
    int err;                       // first error code of the current call (0 = none)
    int ci;                        // climbing image of the last evaluation, -1 none
    int fresh, n_pos;
    double dt, alpha;
    double f_tol;
    double fmax;                   // fmax of the last evaluation
    int record_fneb;
    // proposal of the current step (committed by the finalize kernel)
    double cplus[CFNEB_MAX_IMAGES], cminus[CFNEB_MAX_IMAGES];
    // atom-row means of tau+, tau- and the generalized force (rigid translation)
    double tmean[CFNEB_MAX_IMAGES][9];
    double cv, cf, dt_new, alpha_new;
    int n_pos_new;
    int move;
    double scale;
    // refine
    int refine_due;                // 1: refine kernels act at the end of this step
    int ins, del;                  // last refine decision (logical index, -1 none)
    int changed;
    int new_slot, ins_a, ins_b;    // slots of an insertion
    double d2[CFNEB_MAX_IMAGES];   // squared spacings (reporting)
    // readout
    double barrier;
    double xi[CFNEB_MAX_IMAGES];
    double Hlog[CFNEB_MAX_IMAGES];
};

// Everything a kernel needs, passed by value.
struct BandDev {
    int N, ld, Mcap, ntA, ntR, ntR4, nbcap, cap, ccap;
    int potential, fp64;
    double rc, rc2;
    double skin, rcl, rcl2;  // candidate skin, list cutoff rc + skin and its square
    double lj_eps, lj_sig2, lj_eshift;
    int lj_lanes;  // lanes sharing an atom in the LJ force kernel (1, 2, 4 or 8)
    double ts_A, ts_B, ts_l1, ts_l2, ts_beta, ts_bn, ts_lnbeta, ts_n, ts_c2, ts_d2, ts_c2d2, ts_h, ts_R, ts_S;
    double k_spring;
    int climb_after, cell_filter;
    int relax;  // no tangent projection or springs: F_NEB = generalized force
    double cf, bscale, press;
    int stressed;          // an applied stress beyond the pressure is set
    double sapp[9];        // applied second Piola-Kirchhoff stress (eV/A^3), referred to h0
    double omega0;         // |det h0|
    double dt0, dtmax, maxstep;
    int nmin;
    double finc, fdec, astart, fa;
    int refine_every, ins_num, ins_den, del_num, del_den, max_images, min_images;
    double h0[9];
    // device pointers
    double* X;
    double* V;
    double* R;
    uint32_t* S;        // FP32 LJ bands, else null: three words per atom
    void* F;
    double* FN;
    int4* binfo;
    int* bcount;
    int* bstart;
    struct BinAtom* bpos;
    uint32_t* nbr;
    int* ncnt;
    uint32_t* cand;     // [slot][ccap][N] candidate entries, packed like nbr
    int* ncand;         // [slot][N]
    float* Rref;        // [slot][3][ld] positions at the candidate build, rounded to FP32
    SkinState* skst;    // [slot]
    // Tersoff bond scratch: bond vectors, bond orders and candidate slots of bonds
    // past the fourth ([slot][cap][N]); the per-candidate derivatives P
    // ([slot][ccap][N], zero for candidates that are not bonds) and, per candidate,
    // the index in P of its reverse (i, -n) in j's list: q N + j for j's slot q.
    void* dvec;
    void* bo;
    void* bcid;
    void* P;
    uint32_t* crev;
    ImageGeom* geom;
    ImageScal* scal;
    double* evpart;     // [slot][ntA][4][10]: energy and virial sums of each wave of a tile
    double* dotpart;    // [k][CFNEB_NDOT][ntR4][4]: one partial per wave of each 1024-row item
    double* dotred;     // [k][CFNEB_NDOT] reduced band dots
    double* maxpart;    // [k][3][ntR4]
    double* skmax;      // [slot][1024-atom tile][2] max |R_i - R_i,ref (I + E)|^2 and max |R_i,ref|^2 of the tile
    uint64_t* refpart;  // [k][ntR][2]
    double* staging;    // endpoint upload and readout area
    BandState* st;
};

// ---------------------------------------------------------------- helpers
// Global-memory views of device pointers.  A pointer read out of a struct is generic
// to the compiler, which then emits flat accesses (counted against the LDS/scalar
// counter as well, so waits are coarser and loads cannot go through the scalar
// cache); accesses through these views compile to global (or scalar) loads.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ inline gmem<T>* gp(T* p)
{
    return (gmem<T>*)p;
}
// Constant-memory views, for data that no block writes while the kernel runs (the
// band table, the work plan, a band's state in the kernels that only read it):
// uniform reads through them become scalar loads through the scalar cache, which
// the compiler cannot otherwise prove safe once the kernel has stored anything.
template <typename T>
using cmem = __attribute__((address_space(4))) T;
template <typename T>
__device__ inline const cmem<T>* cp(const T* p)
{
    return (const cmem<T>*)p;
}
// Values that are the same for every lane (band fields, the potential's parameters):
// marking them uniform lets the compiler keep them in scalar registers, and a pointer
// so marked serves as the scalar base of a load with a 32-bit lane offset.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline unsigned long long uni(unsigned long long v)
{
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(v & 0xffffffffull)));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(v >> 32)));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ inline double uni(double v)
{
    return __longlong_as_double((long long)uni((unsigned long long)__double_as_longlong(v)));
}
template <typename T>
__device__ inline T* uni(T* p)
{
    return reinterpret_cast<T*>(uni((unsigned long long)reinterpret_cast<uintptr_t>(p)));
}

// HIP's vector structs cannot be copied through such a view; these move them as
// native 4-vectors.
template <typename T>
using nvec4 = T __attribute__((ext_vector_type(4)));
template <typename V>
__device__ inline V load4(const gmem<const V>* p, size_t i)
{
    using E = decltype(V().x);
    const nvec4<E> v = reinterpret_cast<const gmem<const nvec4<E>>*>(p)[i];
    V o;
    o.x = v.x;
    o.y = v.y;
    o.z = v.z;
    o.w = v.w;
    return o;
}
// packed FP64 position record (x, y, z)
struct R3 {
    double x, y, z;
};
// a packed position record (w = 0)
__device__ inline double4 load4(const gmem<const R3>* p, size_t i)
{
    const gmem<const double>* q = reinterpret_cast<const gmem<const double>*>(p + i);
    return make_double4(q[0], q[1], q[2], 0.0);
}
__device__ inline void store3(gmem<R3>* p, size_t i, double x, double y, double z)
{
    gmem<double>* q = reinterpret_cast<gmem<double>*>(p + i);
    q[0] = x;
    q[1] = y;
    q[2] = z;
}
template <typename V>
__device__ inline void store4(gmem<V>* p, size_t i, const V& o)
{
    using E = decltype(V().x);
    nvec4<E> v;
    v.x = o.x;
    v.y = o.y;
    v.z = o.z;
    v.w = o.w;
    reinterpret_cast<gmem<nvec4<E>>*>(p)[i] = v;
}

__host__ __device__ inline size_t slot_rows(const BandDev& b) { return size_t(3) * b.ld; }

__device__ inline double* Xs(const BandDev& b, int slot) { return b.X + size_t(slot) * slot_rows(b); }
__device__ inline double* Vs(const BandDev& b, int buf, int slot)
{
    return b.V + (size_t(buf) * b.Mcap + slot) * slot_rows(b);
}
// Cartesian positions R = R~ D, one packed 24-byte record (x, y, z) per atom, so a
// neighbour's position is one contiguous gather.
__device__ inline R3* Rs(const BandDev& b, int slot) { return reinterpret_cast<R3*>(b.R) + size_t(slot) * b.ld; }
__device__ inline uint32_t* Ss(const BandDev& b, int slot) { return b.S + size_t(slot) * b.ld * 3; }

__device__ inline uint32_t pack_nbr(int j, int n0, int n1, int n2)
{
    return uint32_t(j) | (uint32_t(n0 + 8) << 20) | (uint32_t(n1 + 8) << 24) | (uint32_t(n2 + 8) << 28);
}
__device__ inline int nbr_j(uint32_t e) { return int(e & 0xFFFFFu); }
__device__ inline int nbr_n(uint32_t e, int k) { return int((e >> (20 + 4 * k)) & 0xFu) - 8; }

// Exact squared distance of entry (j, n); every operation rounded separately.
__device__ inline double exact_r2(const double* ri, double xj, double yj, double zj, const double* h,
                                  int n0, int n1, int n2, double* d)
{
#pragma clang fp contract(off)
    const double rj[3] = {xj, yj, zj};
    for (int c = 0; c < 3; ++c) {
        const double sh = (double(n0) * h[c] + double(n1) * h[3 + c]) + double(n2) * h[6 + c];
        d[c] = (rj[c] - ri[c]) + sh;
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

// Logical image range of a per-image launch: all images, or the moving ones.
__device__ inline bool image_active(const BandState* st, int k, int all_images)
{
    const int M = st->M;
    return all_images ? (k < M) : (k >= 1 && k < M - 1);
}

__device__ inline bool band_stopped(const BandState* st) { return st->done != 0 || st->err != 0; }
__device__ inline bool band_stopped(const cmem<BandState>* st) { return (st->done | st->err) != 0; }

// ---------------------------------------------------------------- work plan
// Every kernel of a step is persistent: a fixed grid walks a work plan of items
// over all bands of a batch (a single band is a batch of one).  The plan kernel,
// launched first, counts each band's items of every kind from the band's live
// image count and flags and stores exclusive prefix offsets; a block maps its
// linear item L to (band, tile, image) by binary search over the offsets.  Bands
// of any size share one launch per phase, and the grid (captured once in a graph)
// does not depend on how many bands or images are live.
//
// XCD awareness: workgroups go to the 8 XCDs round-robin by linear id and each XCD
// has its own L2.  Block W serves items (W % 8) * chunk + W / 8 + n * (G / 8),
// chunk = ceil(total / 8), so every XCD walks one contiguous run of items (tiles of
// one image of one band at a time) and the XCDs get equal shares.
#define CFNEB_XCDS 8
#define CFNEB_MAX_BANDS 128

enum ItemKind {
    KIND_ATOM = 0,  // 256-atom tiles x images
    KIND_ROW,       // 256-row tiles (N + 3 rows) x images
    KIND_BIN,       // 256-bin tiles x images
    KIND_IMAGE,     // one item per image
    KIND_IVAL,      // 256-row tiles x intervals between consecutive images
    KIND_SLOTROW,   // 256-row tiles x every image slot of the capacity
    KIND_BAND,      // one item per band
    KIND_ATOM4,     // 1024-atom tiles x images (4 atoms per thread)
    KIND_ROW4,      // 1024-row tiles x images (4 rows per thread)
    NKIND
};

struct BatchDev {
    const BandDev* bands;  // [cap] band table
    const int* live;       // [cap] 1 where the table holds a band
    int* plan;             // [NKIND][cap + 1] exclusive prefix offsets
    int cap;
};

// Set by the skin decision when any image of any band rebuilds its candidates this
// step (cleared by the plan kernel); the rebuild kernels return at once without it.
__device__ inline int* rebuild_flag(const BatchDev& bd) { return bd.plan + NKIND * (bd.cap + 1); }
// Set by the finalize kernel when any band's step is due for the adaptive-image check
// (cleared by the plan kernel); the step-end refine kernels return at once without it.
__device__ inline int* refine_flag(const BatchDev& bd) { return bd.plan + NKIND * (bd.cap + 1) + 1; }

// A band's table entry copied out of the constant view: the fields a kernel uses
// become scalar loads (the copy itself is taken apart into registers).
__device__ inline BandDev band_ro(const BatchDev& bd, int i) { return *(const BandDev*)(cp(bd.bands) + i); }

struct Item {
    int band, tile, image;
};

__device__ inline int kind_tiles(const BandDev& b, int kind)
{
    switch (kind) {
    case KIND_ATOM: return b.ntA;
    case KIND_ATOM4: return (b.N + CFNEB_TILE4 - 1) / CFNEB_TILE4;
    case KIND_ROW4: return b.ntR4;
    case KIND_BIN: return (b.nbcap + CFNEB_TILE - 1) / CFNEB_TILE;
    case KIND_ROW:
    case KIND_IVAL:
    case KIND_SLOTROW: return b.ntR;
    default: return 1;
    }
}

// Items of one band: images of a step (the moving ones) or of an evaluation of every
// image; first image index of the walk.
__device__ inline void kind_span(const BandDev& b, int kind, int M, int all_images, int& count, int& first)
{
    const int nimg = all_images ? M : M - 2;
    first = all_images ? 0 : 1;
    switch (kind) {
    case KIND_IVAL:
        count = kind_tiles(b, kind) * (M - 1);
        first = 0;
        break;
    case KIND_SLOTROW:
        count = kind_tiles(b, kind) * b.Mcap;
        first = 0;
        break;
    case KIND_BAND:
        count = 1;
        first = 0;
        break;
    default: count = kind_tiles(b, kind) * (nimg > 0 ? nimg : 0); break;
    }
}

// Persistent, XCD-ordered walk over the items of one kind.  RO: the kernel writes
// no band's image count, so the plan, band table and counts are read as constants.
template <bool RO>
struct ItemLoopT {
    const BatchDev* bd;
    int kind, total, chunk, xcd, j, per, n, first_mode;
    __device__ ItemLoopT(const BatchDev& b, int k, int all_images)
        : bd(&b), kind(k), n(0), first_mode(all_images)
    {
        total = RO ? cp(b.plan)[k * (b.cap + 1) + b.cap] : b.plan[k * (b.cap + 1) + b.cap];
        per = int(gridDim.x) / CFNEB_XCDS;
        xcd = int(blockIdx.x) % CFNEB_XCDS;
        j = int(blockIdx.x) / CFNEB_XCDS;
        chunk = (total + CFNEB_XCDS - 1) / CFNEB_XCDS;
    }
    __device__ bool next(Item& it)
    {
        const int idx = j + n * per;
        ++n;
        if (idx >= chunk) return false;
        const int L = xcd * chunk + idx;
        if (L >= total) return false;
        const int* off = bd->plan + kind * (bd->cap + 1);
        int lo = 0, hi = bd->cap;  // off[lo] <= L < off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if ((RO ? cp(off)[mid] : off[mid]) <= L)
                lo = mid;
            else
                hi = mid;
        }
        int count, first, nt;
        if constexpr (RO) {
            const BandDev b = band_ro(*bd, lo);
            kind_span(b, kind, cp(b.st)->M, first_mode, count, first);
            nt = kind_tiles(b, kind);
        } else {
            const BandDev& b = bd->bands[lo];
            kind_span(b, kind, b.st->M, first_mode, count, first);
            nt = kind_tiles(b, kind);
        }
        const int local = L - (RO ? cp(off)[lo] : off[lo]);
        it.band = lo;
        if (kind == KIND_ROW4) {
            // tile-major: the same rows of consecutive images are neighbouring items,
            // so the neighbour images' X read by the band passes come from L2; last
            // tile first, since the tile with the cell rows is the slowest item
            const int nimg = count / nt;
            it.tile = nt - 1 - local / nimg;
            it.image = first + local % nimg;
        } else {
            it.tile = local % nt;
            it.image = first + local / nt;
        }
        return true;
    }
};
using ItemLoop = ItemLoopT<false>;
using ItemLoopRO = ItemLoopT<true>;

// The work plan of a table, written by one block of CFNEB_MAX_BANDS threads: each
// thread counts one band's items of every kind, then the exclusive prefix offsets go
// to the plan; the step's device flags are cleared.
__device__ inline void plan_block(const BatchDev& bd, int all_images, int ignore_stop)
{
    __shared__ int cnt[NKIND][CFNEB_MAX_BANDS];
    const int t = threadIdx.x;
    if (t == 0) {
        *rebuild_flag(bd) = 0;
        *refine_flag(bd) = 0;
    }
    if (t < bd.cap) {
        int c[NKIND];
        for (int q = 0; q < NKIND; ++q) c[q] = 0;
        if (bd.live[t]) {
            const BandDev& b = bd.bands[t];
            const BandState* st = b.st;
            if (ignore_stop || !band_stopped(st)) {
                const int M = st->M;
                for (int q = 0; q < NKIND; ++q) {
                    int first;
                    kind_span(b, q, M, all_images, c[q], first);
                }
            }
        }
        for (int q = 0; q < NKIND; ++q) cnt[q][t] = c[q];
    }
    __syncthreads();
    if (t < NKIND) {
        int* off = bd.plan + t * (bd.cap + 1);
        int run = 0;
        for (int bi = 0; bi < bd.cap; ++bi) {
            off[bi] = run;
            run += cnt[t][bi];
        }
        off[bd.cap] = run;
    }
}

// Grid sizes of the persistent launches (multiples of 8).
#define CFNEB_GRID_TILES 2048
#define CFNEB_GRID_IMAGES 512
#define CFNEB_GRID_BANDS CFNEB_MAX_BANDS
#define CFNEB_GRID_FORCE 16384

__host__ __device__ inline unsigned grid_for(long long max_items, unsigned cap)
{
    long long g = (max_items + CFNEB_XCDS - 1) / CFNEB_XCDS * CFNEB_XCDS;
    if (g < CFNEB_XCDS) g = CFNEB_XCDS;
    return unsigned(g < cap ? g : cap);
}

// Kernel variants by potential and force precision; a launch serves the bands of
// the variants it is instantiated for and skips the others.
enum { VARIANT_LJ32 = 0, VARIANT_LJ64, VARIANT_TS32, VARIANT_TS64, NVARIANT };

__host__ __device__ inline int band_variant(const BandDev& b)
{
    return (b.potential == CFNEB_TERSOFF_C ? 2 : 0) + (b.fp64 ? 1 : 0);
}

// Bits 8..11 of a launch's variant set: the LJ lane counts 1, 2, 4, 8 present (each
// band keeps its own count, alone and in a batch, so its sums never depend on its
// batch-mates).
__host__ __device__ inline unsigned lanes_bit(const BandDev& b)
{
    if (b.potential != CFNEB_LJ) return 0u;
    const int k = b.lj_lanes;
    return 1u << (8 + (k >= 8 ? 3 : k >= 4 ? 2 : k >= 2 ? 1 : 0));
}
__host__ __device__ inline unsigned launch_variants(const BandDev& b) { return (1u << band_variant(b)) | lanes_bit(b); }

// Launch geometry of one batch: the grid of each kind, bounded by the most items
// the table can ever hold, and the variants present.
struct Launch {
    BatchDev bd;
    unsigned g[NKIND];
    // grid of the force kernels (LJ pair kernel, the two Tersoff kernels): the
    // persistent grid g[KIND_ATOM] or one block per atom tile of the largest item
    // count (g_force_tile), where the hardware hands the last tiles to whichever
    // slots free first; chosen by timing before the step graphs are captured
    unsigned g_force, g_force_tile;
    unsigned variants;
};

__device__ inline void set_error(BandState* st, int code)
{
    atomicCAS(&st->err, 0, code);
}

// Lane exchanges of the transposed wave reduction.  A step halves the n values each
// lane holds: the lane whose bit m is set keeps the upper half, its partner (bit m
// clear) the lower half, and each adds the partner's copy of the half it keeps.  Any
// partner that differs in bit m and agrees in the bits above it gives the same
// result, so the row-internal steps take the DPP mirror patterns.
// Steps of 32 and 16 lanes: v_permlane32_swap / v_permlane16_swap exchange the
// upper lanes of the first operand with the lower lanes of the second, so with the
// lower half of the values as the first operand and the upper half as the second,
// the two results always add up to the kept half plus the partner's copy of it.
template <bool S32>
__device__ inline void swap_pair(double a, double b, double& p, double& q)
{
    const unsigned long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    const auto lo = S32 ? __builtin_amdgcn_permlane32_swap(unsigned(x), unsigned(y), false, false)
                        : __builtin_amdgcn_permlane16_swap(unsigned(x), unsigned(y), false, false);
    const auto hi = S32 ? __builtin_amdgcn_permlane32_swap(unsigned(x >> 32), unsigned(y >> 32), false, false)
                        : __builtin_amdgcn_permlane16_swap(unsigned(x >> 32), unsigned(y >> 32), false, false);
    p = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    q = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
template <bool S32>
__device__ inline double swap_add(double a, double b)
{
    double p, q;
    swap_pair<S32>(a, b, p, q);
    return p + q;
}
template <int CTRL>
__device__ inline double dpp_f64(double x)
{
    const unsigned long long v = __double_as_longlong(x);
    const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(v)), CTRL, 0xF, 0xF, true));
    const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(v >> 32)), CTRL, 0xF, 0xF, true));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Sum and maximum over a wave, the same value in every lane: partners 32 and 16
// lanes apart through the lane swaps, then lane ^ 15, ^ 7, ^ 2 and ^ 1 within a row
// (DPP); each step pairs lanes by an xor mask, so partners hold identical results.
// These exchanges and the transposed ones below read every lane: all 64 lanes of the
// wave must take part (no caller sits inside a lane-dependent branch).
__device__ inline double wave_sum(double v)
{
    v = swap_add<true>(v, v);
    v = swap_add<false>(v, v);
    v += dpp_f64<0x140>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0xB1>(v);
    return v;
}
__device__ inline double wave_max(double v)
{
    double p, q;
    swap_pair<true>(v, v, p, q);
    v = fmax(p, q);
    swap_pair<false>(v, v, p, q);
    v = fmax(p, q);
    v = fmax(v, dpp_f64<0x140>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0xB1>(v));
    return v;
}

// Block sum of NV doubles in a fixed order (waves in index order); the result is
// valid in thread 0.  lds must hold (blockDim.x / 64) * NV doubles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[wid * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = lds[q];
            for (int w = 1; w < nw; ++w) s += lds[w * NV + q];
            v[q] = s;
        }
    __syncthreads();
}

template <int N, bool S32>
__device__ inline void wave_swap_step(double* u)
{
    constexpr int half = N > 1 ? N / 2 : 1;
#pragma unroll
    for (int i = 0; i < half; ++i) u[i] = swap_add<S32>(u[i], N > 1 ? u[half + i] : u[i]);
}
template <int N, int M, int CTRL>
__device__ inline void wave_dpp_step(double* u, int lane)
{
    if constexpr (N > 1) {
        constexpr int half = N / 2;
        const bool up = (lane & M) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = up ? u[i] : u[half + i];
            const double keep = up ? u[half + i] : u[i];
            u[i] = keep + dpp_f64<CTRL>(send);
        }
    } else {
        u[0] += dpp_f64<CTRL>(u[0]);
    }
}
// Block sum of NV doubles by a transposed wave reduction: at each halving step a lane
// keeps half of its values and trades the other half with its partner, so a wave
// makes P - 1 + 6 - log2 P exchanges instead of 6 NV (P = NV rounded up to a power of
// two, at most 64), through lane swaps and DPP moves rather than LDS permutes.  Fixed
// order; the result is valid in thread 0.  lds must hold (blockDim.x / 64) * NV
// doubles.
constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }
template <int NV>
constexpr int wave_sum_logp()
{
    constexpr int P = pow2_at_least(NV);
    return P <= 1 ? 0 : P <= 2 ? 1 : P <= 4 ? 2 : P <= 8 ? 3 : P <= 16 ? 4 : P <= 32 ? 5 : 6;
}
// The wave stage of block_sum_t: returns the lane's sum, which is the wave's total of
// value (lane >> (6 - LOGP)) & (P - 1) on lanes whose low 6 - LOGP bits are zero.
template <int NV>
__device__ inline double wave_sum_t(const double (&v)[NV])
{
    constexpr int P = pow2_at_least(NV);
    static_assert(P <= 64, "at most 64 values");
    const int lane = threadIdx.x & 63;
    double u[P];
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = i < NV ? v[i] : 0.0;
    // lanes 32 apart, then 16 apart: one swap trades the halves both ways
    wave_swap_step<P, true>(u);
    wave_swap_step<(P > 1 ? P / 2 : 1), false>(u);
    // within a row of 16: partners by mirror images and quad permutations (DPP)
    wave_dpp_step<(P > 4 ? P / 4 : 1), 8, 0x140>(u, lane);   // row_mirror: lane ^ 15
    wave_dpp_step<(P > 8 ? P / 8 : 1), 4, 0x141>(u, lane);   // row_half_mirror: lane ^ 7
    wave_dpp_step<(P > 16 ? P / 16 : 1), 2, 0x4E>(u, lane);  // quad_perm [2,3,0,1]: lane ^ 2
    wave_dpp_step<(P > 32 ? P / 32 : 1), 1, 0xB1>(u, lane);  // quad_perm [1,0,3,2]: lane ^ 1
    return u[0];
}
template <int NV>
__device__ inline void block_sum_t(double (&v)[NV], double* lds)
{
    constexpr int P = pow2_at_least(NV);
    constexpr int LOGP = wave_sum_logp<NV>();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
    const double ws = wave_sum_t<NV>(v);
    // the lane's sum is value (lane >> (6 - LOGP)) of the wave
    const int idx = (lane >> (6 - LOGP)) & (P - 1);
    if ((lane & ((64 >> LOGP) - 1)) == 0 && idx < NV) lds[wid * NV + idx] = ws;
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = lds[q];
            for (int w = 1; w < nw; ++w) s += lds[w * NV + q];
            v[q] = s;
        }
    __syncthreads();
}

template <int NV>
__device__ inline void block_max(double (&v)[NV], double* lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_max(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[wid * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = lds[q];
            for (int w = 1; w < nw; ++w) s = fmax(s, lds[w * NV + q]);
            v[q] = s;
        }
    __syncthreads();
}

// 3x3 helpers (row-major)
__host__ __device__ inline double det3(const double* a)
{
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6])
         + a[2] * (a[3] * a[7] - a[4] * a[6]);
}
__host__ __device__ inline void inv3(const double* a, double* o)
{
    const double id = 1.0 / det3(a);
    o[0] = (a[4] * a[8] - a[5] * a[7]) * id;
    o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = (a[5] * a[6] - a[3] * a[8]) * id;
    o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = (a[3] * a[7] - a[4] * a[6]) * id;
    o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}
__host__ __device__ inline void mm3(const double* a, const double* b, double* c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// Tersoff force gather of atoms i0 + q * stride (q < Q, those below N): F_i =
// sum_c (P_c - P_rev(c)) over i's candidates c in increasing order, four at a time, P_c
// from i's own slot and P_rev(c) from the reverse candidate (i, -n) of j's list; both
// vanish unless the pair is a bond.  All loads of one round (slots, reverse slots,
// own P of every atom), then every reverse P, are in flight together.
template <typename T>
using vec4_of = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
// dU_i/dr^ij of a Tersoff candidate slot: three packed components (12 bytes in FP32,
// one dwordx3 access)
template <typename T>
struct P3 {
    T x, y, z;
};
template <typename T>
__device__ inline P3<T> load3(const gmem<const P3<T>>* p, size_t i)
{
    const gmem<const T>* q = reinterpret_cast<const gmem<const T>*>(p + i);
    return P3<T>{q[0], q[1], q[2]};
}
template <typename T>
__device__ inline void store3(gmem<P3<T>>* p, size_t i, T x, T y, T z)
{
    gmem<T>* q = reinterpret_cast<gmem<T>*>(p + i);
    q[0] = x;
    q[1] = y;
    q[2] = z;
}

template <typename T, int Q>
__device__ inline void tersoff_gather(const BandDev& b, int slot, int i0, int stride, T (&f)[Q][3])
{
    const size_t N = b.N;
    const gmem<const uint32_t>* __restrict__ crev = gp<const uint32_t>(b.crev + size_t(slot) * b.ccap * N);
    const gmem<const P3<T>>* __restrict__ Pb =
        gp<const P3<T>>(reinterpret_cast<const P3<T>*>(b.P) + size_t(slot) * b.ccap * N);
    const gmem<const int>* __restrict__ ncand = gp<const int>(b.ncand + size_t(slot) * N);
    constexpr int U = 4;
    int nc[Q], ii[Q], nmax = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = i0 + q * stride;
        ii[q] = i < b.N ? i : b.N - 1;
        nc[q] = i < b.N ? ncand[ii[q]] : 0;
        f[q][0] = f[q][1] = f[q][2] = T(0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) nmax = max(nmax, nc[q]);
    for (int c0 = 0; c0 < nmax; c0 += U) {
        uint32_t rv[Q][U];
        P3<T> pe[Q][U], pr[Q][U];
        // past an atom's last candidate the loads repeat it (always in bounds, no
        // branch between the loads) and its sum below stops
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t o = size_t(max(min(c0 + u, nc[q] - 1), 0)) * N + ii[q];
                rv[q][u] = crev[o];
                pe[q][u] = load3(Pb, o);
            }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads of the round ahead of their uses
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) pr[q][u] = load3(Pb, rv[q][u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (c0 + u >= nc[q]) break;
                f[q][0] += pe[q][u].x;
                f[q][1] += pe[q][u].y;
                f[q][2] += pe[q][u].z;
                f[q][0] -= pr[q][u].x;
                f[q][1] -= pr[q][u].y;
                f[q][2] -= pr[q][u].z;
            }
    }
}

// Energy and virial partials of one 256-atom tile: each wave stores its own ten sums
// (transposed wave reduction, no block barrier).  Every wave of the tile stores, so
// no partial of an earlier evaluation survives.
__device__ inline void store_ev_partials(const BandDev& b, int slot, int tile, const double (&v)[10])
{
    const double s = wave_sum_t<10>(v);
    constexpr int LOGP = wave_sum_logp<10>();
    const int lane = int(threadIdx.x) & 63, idx = lane >> (6 - LOGP);
    if ((lane & ((64 >> LOGP) - 1)) == 0 && idx < 10)
        b.evpart[((size_t(slot) * b.ntA + tile) * CFNEB_WAVES + (int(threadIdx.x) >> 6)) * 10 + idx] = s;
}

// ---------------------------------------------------------------- launchers
// Defined in the kernel translation units, called by the host runtime.
// One band, direct launches (construction and readout helpers):
// Per-image reduction of the energy and virial tile partials in a fixed order, then
// the enthalpy and the lattice force G = D^-T (V - P Omega I) D^-1 / c_f
// (Eqs. (16)-(17)); thread 0 writes the image's scalars.
__device__ inline void image_reduce_item(const BandDev& b, BandState* st, int slot, double* lds)
{
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double* part = b.evpart + size_t(slot) * b.ntA * CFNEB_WAVES * 10;
    for (int t = threadIdx.x; t < b.ntA * CFNEB_WAVES; t += CFNEB_TILE)
        for (int q = 0; q < 10; ++q) acc[q] += part[size_t(t) * 10 + q];
    block_sum<10>(acc, lds);
    if (threadIdx.x != 0) return;
    const ImageGeom& g = b.geom[slot];
    ImageScal& s = b.scal[slot];
    s.E = acc[0];
    s.H = acc[0] + b.press * g.omega;
    bool finite = isfinite(s.H);
    double Veff[9];
    for (int q = 0; q < 9; ++q) {
        s.V[q] = acc[1 + q];
        Veff[q] = acc[1 + q];
        finite = finite && isfinite(Veff[q]);
    }
    for (int q = 0; q < 3; ++q) Veff[4 * q] -= b.press * g.omega;
    if (b.stressed) {
        // H gains -Omega0 S : E with E = (D D^T - I) / 2, whose virtual work in the
        // strain D^-1 dD is that of the extra virial Omega0 D^T S D
        double SD[9], W[9];
        mm3(b.sapp, g.D, SD);
        double work = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double e = 0.0, w = 0.0;
                for (int q = 0; q < 3; ++q) {
                    e += g.D[3 * r + q] * g.D[3 * c + q];
                    w += g.D[3 * q + r] * SD[3 * q + c];
                }
                if (r == c) e -= 1.0;
                work += b.sapp[3 * r + c] * (0.5 * e);
                W[3 * r + c] = w;
            }
        s.H -= b.omega0 * work;
        for (int q = 0; q < 9; ++q) Veff[q] += b.omega0 * W[q];
        finite = finite && isfinite(s.H);
    }
    double DinvT[9], T1[9], G[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) DinvT[3 * r + c] = g.Dinv[3 * c + r];
    mm3(DinvT, Veff, T1);
    if (b.cell_filter == 1) {
        // D-variant (Eq. (13)): the conjugate of D is D^-T V_eff, all nine entries
        for (int q = 0; q < 9; ++q) s.Fcell[q] = T1[q] / b.cf;
    } else {
        mm3(T1, g.Dinv, G);
        const double sc = (b.cell_filter == 2) ? b.bscale / b.cf : 0.0;
        // the force conjugate to the symmetric B is the symmetric part of G (the FP32
        // virial is symmetric only to rounding; an antisymmetric rest would move the
        // cell rows along a direction the energy does not see)
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) s.Fcell[3 * r + c] = sc * (0.5 * (G[3 * r + c] + G[3 * c + r]));
    }
    if (!finite) set_error(st, CFNEB_ENONFINITE);
}


// Zero a workspace of `bytes` bytes (a multiple of 256 at a 256-byte aligned address).
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t s);
void launch_init_endpoints(const BandDev& b, hipStream_t s);
void launch_init_images(const BandDev& b, int M, hipStream_t s);
void launch_init_state(const BandDev& b, int M, hipStream_t s);
void launch_image_positions(const BandDev& b, int k, hipStream_t s);
// Persistent launches over every live band of a table:
void launch_plan(const Launch& L, int all_images, int ignore_stop, hipStream_t s);
// Set aside (hold = 1) or restore (hold = 0) the per-slot rebuild flags of every live
// band, so that force kernels re-run outside a step do the work of a step without a
// candidate rebuild.
void launch_skin_hold(const Launch& L, int hold, hipStream_t s);
void launch_profile(const Launch& L, int n_samples, hipStream_t s);
void launch_begin_call(const Launch& L, double f_tol, int only, hipStream_t s);
void launch_geom(const Launch& L, int all_images, hipStream_t s);
void launch_skin(const Launch& L, int all_images, hipStream_t s);
void launch_bins(const Launch& L, int all_images, hipStream_t s);
void launch_list(const Launch& L, int all_images, hipStream_t s);
void launch_filter(const Launch& L, int all_images, hipStream_t s);
void launch_neighbour_lists(const Launch& L, hipStream_t s);
void launch_force_stage(const Launch& L, int all_images, int stage, hipStream_t s);
void launch_tersoff_stage(const Launch& L, int all_images, int stage, hipStream_t s);
void launch_image_reduce(const Launch& L, int all_images, hipStream_t s);
void launch_dots(const Launch& L, hipStream_t s);
void launch_scalars(const Launch& L, hipStream_t s);
void launch_update(const Launch& L, hipStream_t s);
void launch_finalize(const Launch& L, hipStream_t s);
void launch_flush_move(const Launch& L, hipStream_t s);

// The pending move of one row of a moving image: X += scale (dt v'), v' in the
// committed velocity buffer (the same rounding as a separate move pass).
__device__ inline bool move_pending(const BandState* st, int all_images)
{
    return all_images == 0 && st->move != 0 && st->err == 0;
}
__device__ inline bool move_pending(const cmem<BandState>* st, int all_images)
{
    return all_images == 0 && (st->move != 0) & (st->err == 0);
}
void launch_refine(const Launch& L, int forced, hipStream_t s);
void launch_readout(const Launch& L, hipStream_t s);
void launch_evaluate(const Launch& L, int all_images, hipStream_t s);
// One band step: launch_step_core (evaluation, projection, FIRE, move) then the
// refinement phase; a step on which no band can be due for refinement may launch the
// core alone (refinement then has nothing to do).
void launch_step_core(const Launch& L, hipStream_t s);
void launch_step(const Launch& L, hipStream_t s);
void launch_summary(const Launch& L, int* out, hipStream_t s);

}  // namespace cfneb

#endif
