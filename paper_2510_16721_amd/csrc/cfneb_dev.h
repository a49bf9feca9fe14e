// Device-side layout and helpers of the CFNEB library (gfx950).
//
// HBM layout of one band (all inside the caller's workspace, 256-B aligned):
//   X      [slot][3][ld]  FP64  generalized coordinates: rows 0..N-1 = R~ (SoA),
//                               rows N..N+2 = the three rows of c_f B
//   V      [2][slot][3][ld] FP64 FIRE velocities, ping-pong (vcur selects)
//   R      [slot][3][ld]  FP64  Cartesian positions R = R~ D of the last evaluation
//   F      [slot][3][ld]  T     Cartesian forces (T = float, or double for FP64 bands)
//   FN     [slot][3][ld]  FP64  NEB force (only when recording is on)
//   binfo  [slot][N]      int4  (bin, rank in bin, packed lattice image) per atom
//   bins   [slot][...]    int   counts, starts; bpos: atoms in bin order (R, packed id)
//   nbr    [slot][cap][N] u32   packed neighbour entries, entry-major (coalesced)
//   ncnt   [slot][N]      int   neighbour count (may exceed cap: overflow)
//   dvec   [slot][cap][N] T4    Tersoff: bond vector and length
//   bo     [slot][cap][N] T2    Tersoff: b_ij and db/dzeta
//   P      [slot][cap][N] T4    Tersoff: dU_i/dr^ij per bond
//   geom / scal [slot]          per-image 3x3 geometry and reduced scalars
//   partial buffers             fixed-order block partials of every reduction
//   state                       band scalars (FIRE, slot table, flags)
// A "slot" is a physical image buffer; the slot table maps logical image k to a slot,
// so inserting or deleting an image rewrites the table, not the data.
#ifndef CFNEB_DEV_H
#define CFNEB_DEV_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cfneb.h"

#define CFNEB_MAX_IMAGES 64
#define CFNEB_TILE 256           // threads per block of every streaming kernel
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
    int nbins;
    int err;
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
    int N, ld, Mcap, ntA, ntR, nbcap, cap;
    int potential, fp64;
    double rc, rc2;
    double lj_eps, lj_sig2, lj_eshift;
    double ts_A, ts_B, ts_l1, ts_l2, ts_bn, ts_n, ts_c2, ts_d2, ts_c2d2, ts_h, ts_R, ts_S;
    double k_spring;
    int climb_after, cell_filter;
    double cf, bscale, press;
    double dt0, dtmax, maxstep;
    int nmin;
    double finc, fdec, astart, fa;
    int refine_every, ins_num, ins_den, del_num, del_den, max_images, min_images;
    double h0[9];
    // device pointers
    double* X;
    double* V;
    double* R;
    void* F;
    double* FN;
    int4* binfo;
    int* bcount;
    int* bstart;
    struct BinAtom* bpos;
    uint32_t* nbr;
    int* ncnt;
    void* dvec;
    void* bo;
    void* P;
    ImageGeom* geom;
    ImageScal* scal;
    double* evpart;     // [slot][ntA][10]
    double* dotpart;    // [k][ntR][10]
    double* maxpart;    // [k][ntR][2]
    uint64_t* refpart;  // [k][ntR][2]
    double* staging;    // endpoint upload and readout area
    BandState* st;
};

// ---------------------------------------------------------------- helpers
__host__ __device__ inline size_t slot_rows(const BandDev& b) { return size_t(3) * b.ld; }

__device__ inline double* Xs(const BandDev& b, int slot) { return b.X + size_t(slot) * slot_rows(b); }
__device__ inline double* Vs(const BandDev& b, int buf, int slot)
{
    return b.V + (size_t(buf) * b.Mcap + slot) * slot_rows(b);
}
__device__ inline double* Rs(const BandDev& b, int slot) { return b.R + size_t(slot) * slot_rows(b); }

__device__ inline uint32_t pack_nbr(int j, int n0, int n1, int n2)
{
    return uint32_t(j) | (uint32_t(n0 + 8) << 20) | (uint32_t(n1 + 8) << 24) | (uint32_t(n2 + 8) << 28);
}
__device__ inline int nbr_j(uint32_t e) { return int(e & 0xFFFFFu); }
__device__ inline int nbr_n(uint32_t e, int k) { return int((e >> (20 + 4 * k)) & 0xFu) - 8; }

// Logical image range of a per-image launch: all images, or the moving ones.
__device__ inline bool image_active(const BandState* st, int k, int all_images)
{
    const int M = st->M;
    return all_images ? (k < M) : (k >= 1 && k < M - 1);
}

__device__ inline bool band_stopped(const BandState* st) { return st->done != 0 || st->err != 0; }

// XCD-aware work mapping.  Workgroups of a launch go to the 8 XCDs round-robin by
// linear id, and each XCD has its own L2.  A launch over (tile, image) items uses a
// 1-D grid of cfneb_grid(ntiles, Mcap) blocks; block W serves item
//     L = (W % 8) * chunk + W / 8,   chunk = ceil(nact * ntiles / 8),
// over the nact images active now (first = first active image), so every XCD walks
// one contiguous run of tiles of one image at a time and all 8 XCDs get equal work
// whatever the current image count.  Blocks past the work exit at once.
#define CFNEB_XCDS 8
struct WorkItem {
    int tile, image;
    bool valid;
};

__device__ inline WorkItem xcd_item(int ntiles, int first, int nact)
{
    WorkItem w;
    const int W = int(blockIdx.x);
    const int chunk = (nact * ntiles + CFNEB_XCDS - 1) / CFNEB_XCDS;
    const int idx = W / CFNEB_XCDS;
    const int L = (W % CFNEB_XCDS) * chunk + idx;
    w.valid = nact > 0 && idx < chunk && L < nact * ntiles;
    w.tile = w.valid ? L % ntiles : 0;
    w.image = w.valid ? first + L / ntiles : 0;
    return w;
}

// (tile, image) item of a per-atom or per-row launch over the images of a step
// (moving images) or of an evaluation of every image.
__device__ inline WorkItem image_item(const BandState* st, int ntiles, int all_images)
{
    const int M = st->M;
    return all_images ? xcd_item(ntiles, 0, M) : xcd_item(ntiles, 1, M - 2);
}

__host__ __device__ inline unsigned cfneb_grid(int ntiles, int nimages)
{
    const long long t = (long long)ntiles * nimages;
    return unsigned((t + CFNEB_XCDS - 1) / CFNEB_XCDS * CFNEB_XCDS);
}

__device__ inline void set_error(BandState* st, int code)
{
    atomicCAS(&st->err, 0, code);
}

// 64-lane wavefront sum with a fixed butterfly order (deterministic).
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
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

// ---------------------------------------------------------------- launchers
// Defined in the kernel translation units, called by the host runtime.
void launch_init_endpoints(const BandDev& b, hipStream_t s);
void launch_init_images(const BandDev& b, int M, hipStream_t s);
void launch_init_state(const BandDev& b, int M, hipStream_t s);
void launch_begin_call(const BandDev& b, double f_tol, hipStream_t s);
void launch_geom(const BandDev& b, int all_images, hipStream_t s);
void launch_nlist(const BandDev& b, int all_images, hipStream_t s);
void launch_forces(const BandDev& b, int all_images, hipStream_t s);
void launch_bins(const BandDev& b, int all_images, hipStream_t s);
void launch_list(const BandDev& b, int all_images, hipStream_t s);
void launch_force_stage(const BandDev& b, int all_images, int stage, hipStream_t s);
void launch_image_reduce(const BandDev& b, int all_images, hipStream_t s);
void launch_tersoff_stage(const BandDev& b, int all_images, int stage, hipStream_t s);
void launch_dots(const BandDev& b, hipStream_t s);
void launch_scalars(const BandDev& b, hipStream_t s);
void launch_update(const BandDev& b, hipStream_t s);
void launch_finalize(const BandDev& b, hipStream_t s);
void launch_move(const BandDev& b, hipStream_t s);
void launch_evaluate(const BandDev& b, int all_images, hipStream_t s);
void launch_band_update(const BandDev& b, hipStream_t s);
void launch_refine(const BandDev& b, int forced, hipStream_t s);
void launch_readout(const BandDev& b, hipStream_t s);
void launch_image_positions(const BandDev& b, int k, hipStream_t s);
void launch_set_state_fixup(const BandDev& b, int M, hipStream_t s);

}  // namespace cfneb

#endif
