// Work plan of a band table and the order of the kernels of one step.
//
// A table holds up to CFNEB_MAX_BANDS bands (a single band is a table of one).  The
// plan is written first in every step (by block 0 of the geometry kernel, or by the
// plan kernel for calls outside a step): each thread counts one band's items of every
// kind (per-atom tiles, per-row tiles, per-image, ...) from its live image count and
// flags, and the exclusive prefix offsets go to the plan array that every persistent
// kernel of the step walks.  A converged or failed band contributes no items, so a
// batch keeps running the bands that are still relaxing.
#include "cfneb_dev.h"

namespace cfneb {

__global__ void __launch_bounds__(CFNEB_MAX_BANDS) k_plan(BatchDev bd, int all_images, int ignore_stop)
{
    plan_block(bd, all_images, ignore_stop);
}

// Zero `bytes` bytes (a multiple of 16, 16-byte aligned) with vector stores: clears a
// workspace without a memset.
__global__ void k_fill_zero(uint4* p, size_t n16)
{
    const uint4 z = {0u, 0u, 0u, 0u};
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += size_t(gridDim.x) * blockDim.x)
        p[i] = z;
}

void launch_fill_zero(void* ptr, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_zero<<<unsigned(blocks), 256, 0, s>>>(static_cast<uint4*>(ptr), n16);
}

// Per-band status for the host: done, err, steps of the call, M (4 ints per band).
__global__ void k_summary(BatchDev bd, int* out)
{
    const int t = threadIdx.x;
    if (t >= bd.cap) return;
    int* o = out + 4 * t;
    if (!bd.live[t]) {
        o[0] = o[1] = o[2] = o[3] = 0;
        return;
    }
    const BandState* st = bd.bands[t].st;
    o[0] = st->done;
    o[1] = st->err;
    o[2] = st->steps_call;
    o[3] = st->step;
}

void launch_plan(const Launch& L, int all_images, int ignore_stop, hipStream_t s)
{
    k_plan<<<1, CFNEB_MAX_BANDS, 0, s>>>(L.bd, all_images, ignore_stop);
}

void launch_summary(const Launch& L, int* out, hipStream_t s)
{
    k_summary<<<1, CFNEB_MAX_BANDS, 0, s>>>(L.bd, out);
}

// Energies, forces, virials and generalized forces of the moving images (or of every
// image): geometry, cell lists, neighbour lists, potential, per-image reduction.  In
// a step (moving images only) the per-image reduction runs inside the band dots pass.
void launch_evaluate(const Launch& L, int all_images, hipStream_t s)
{
    launch_geom(L, all_images, s);  // also writes the plan
    launch_skin(L, all_images, s);
    launch_bins(L, all_images, s);
    launch_list(L, all_images, s);
    launch_filter(L, all_images, s);
    launch_force_stage(L, all_images, 0, s);
    launch_force_stage(L, all_images, 1, s);
    if (all_images) launch_image_reduce(L, all_images, s);
}

// One band step of every live band.
// (the previous step's move is applied by the geometry and skin passes; this step's
// is left pending)
void launch_step_core(const Launch& L, hipStream_t s)
{
    launch_evaluate(L, 0, s);
    launch_dots(L, s);
    launch_scalars(L, s);
    launch_update(L, s);
    launch_finalize(L, s);
}

// a refinement needs the moved band
void launch_step(const Launch& L, hipStream_t s)
{
    launch_step_core(L, s);
    launch_flush_move(L, s);
    launch_refine(L, 0, s);
}

}  // namespace cfneb
