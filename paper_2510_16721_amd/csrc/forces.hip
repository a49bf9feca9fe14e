// Energies, forces and virials of every image (Sec. II.B).
//
// Each atom's energy U_i is a function of the bond vectors r^ij to its neighbours
// (Eq. (4)).  With P_ij = dU_i/dr^ij the force is F_i = sum_j (P_ij - P_ji) (the
// pair force of Eq. (5) in the index order of the derivation leading to Eq. (6)),
// and the virial is V_mn = -sum_ij r^ij_m P_ij,n = -1/2 sum_ij r^ij_m f^ij_n
// (Eqs. (6)-(8)).  Lists are full, so every force is a gather: no atomics.
// Lennard-Jones lives here; the Tersoff kernels are in tersoff.hip.
//
// Precision: bond vectors are formed in FP64 from FP64 positions, then the pair and
// three-body arithmetic runs in T (float, or double for FP64 bands); per-atom
// energy and virial terms are summed in FP64, then per block and per image in a
// fixed order.
#include <type_traits>

#include "cfneb_dev.h"

namespace cfneb {

// ------------------------------------------------------------ Lennard-Jones
// U_i = 1/2 sum_j phi(r_ij), phi = 4 eps [(s/r)^12 - (s/r)^6] - phi(rc)
template <typename T>
__device__ void lj_item(const BandDev& b, BandState* st, int slot, int tile, double* lds)
{
    const int i = tile * CFNEB_TILE + threadIdx.x;
    const size_t N = b.N;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // u, then V row-major
    if (i < b.N) {
        const gmem<const double4>* __restrict__ R = gp<const double4>(Rs(b, slot));
        const ImageGeom& g = b.geom[slot];
        double h[9];
        for (int q = 0; q < 9; ++q) h[q] = g.h[q];
        const double4 ri = load4(R, i);
        const double ri0 = ri.x, ri1 = ri.y, ri2 = ri.z;
        const gmem<const uint32_t>* __restrict__ nbr = gp<const uint32_t>(b.nbr + size_t(slot) * b.cap * N);
        const int cnt = min(gp<const int>(b.ncnt)[size_t(slot) * N + i], b.cap);
        const T eps4 = T(4.0 * b.lj_eps), eps24 = T(24.0 * b.lj_eps), sig2 = T(b.lj_sig2),
                esh = T(b.lj_eshift);
        T fx = 0, fy = 0, fz = 0;
        // four neighbours at a time: their entries, then their positions, are in flight
        // together (past the last neighbour the loads repeat it; the sums stop there)
        constexpr int U = 4;
        for (int e0 = 0; e0 < cnt; e0 += U) {
            uint32_t ents[U];
            double4 rjs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) ents[u] = nbr[size_t(min(e0 + u, cnt - 1)) * N + i];
#pragma unroll
            for (int u = 0; u < U; ++u) rjs[u] = load4(R, nbr_j(ents[u]));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u >= cnt) break;
                const uint32_t ent = ents[u];
                const int n0 = nbr_n(ent, 0), n1 = nbr_n(ent, 1), n2 = nbr_n(ent, 2);
                const double4 rj = rjs[u];
                const double d0 = (rj.x - ri0) + ((n0 * h[0] + n1 * h[3]) + n2 * h[6]);
                const double d1 = (rj.y - ri1) + ((n0 * h[1] + n1 * h[4]) + n2 * h[7]);
                const double d2 = (rj.z - ri2) + ((n0 * h[2] + n1 * h[5]) + n2 * h[8]);
                const T dx = T(d0), dy = T(d1), dz = T(d2);
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T ir2 = T(1) / r2;
                T s6 = sig2 * ir2;
                s6 = s6 * s6 * s6;
                const T phi = eps4 * (s6 * s6 - s6) - esh;
                const T fr = eps24 * (s6 - T(2) * s6 * s6) * ir2;  // phi'(r) / r
                fx += fr * dx;
                fy += fr * dy;
                fz += fr * dz;
                acc[0] += double(T(0.5) * phi);
                const T hf = T(-0.5) * fr;
                const T wx = hf * dx, wy = hf * dy, wz = hf * dz;
                acc[1] += double(wx * dx);
                acc[2] += double(wx * dy);
                acc[3] += double(wx * dz);
                acc[4] += double(wy * dx);
                acc[5] += double(wy * dy);
                acc[6] += double(wy * dz);
                acc[7] += double(wz * dx);
                acc[8] += double(wz * dy);
                acc[9] += double(wz * dz);
            }
        }
        gmem<T>* F = gp(reinterpret_cast<T*>(b.F) + size_t(slot) * slot_rows(b));
        F[i] = fx;
        F[b.ld + i] = fy;
        F[2 * size_t(b.ld) + i] = fz;
        if (!isfinite(double(fx) + double(fy) + double(fz))) set_error(st, CFNEB_ENONFINITE);
    }
    block_sum_t<10>(acc, lds);
    if (threadIdx.x == 0) {
        double* out = b.evpart + (size_t(slot) * b.ntA + tile) * 10;
        for (int q = 0; q < 10; ++q) out[q] = acc[q];
    }
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_lj(BatchDev bd, int all_images, int variant)
{
    __shared__ double lds[4 * 10];
    ItemLoop loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (band_variant(b) != variant || band_stopped(st)) continue;  // uniform over the block
        lj_item<T>(b, st, st->slot[it.image], it.tile, lds);
    }
}

// ------------------------------------------------------------ per-image reduction
// (image_reduce_item: the step reduces its moving images inside the band dots pass)
__global__ void __launch_bounds__(CFNEB_TILE) k_image_reduce(BatchDev bd, int all_images)
{
    __shared__ double lds[4 * 10];
    ItemLoop loop(bd, KIND_IMAGE, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (band_stopped(st)) continue;  // uniform over the block
        image_reduce_item(b, st, st->slot[it.image], lds);
    }
}

// stage 0: LJ, or Tersoff bond orders and dU_i/dr^ij; 1: Tersoff gather
void launch_force_stage(const Launch& L, int all_images, int stage, hipStream_t s)
{
    const unsigned g = L.g_force;
    if (stage == 0) {
        if (L.variants & (1u << VARIANT_LJ32)) k_lj<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_LJ32);
        if (L.variants & (1u << VARIANT_LJ64)) k_lj<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_LJ64);
    }
    launch_tersoff_stage(L, all_images, stage, s);
}

void launch_image_reduce(const Launch& L, int all_images, hipStream_t s)
{
    k_image_reduce<<<L.g[KIND_IMAGE], CFNEB_TILE, 0, s>>>(L.bd, all_images);
}

}  // namespace cfneb
