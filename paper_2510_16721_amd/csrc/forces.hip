// Energies, forces and virials of every image (Sec. II.B).
//
// Each atom's energy U_i is a function of the bond vectors r^ij to its neighbours
// (Eq. (4)).  With P_ij = dU_i/dr^ij the force is F_i = sum_j (P_ij - P_ji) (the
// pair force of Eq. (5) in the index order of the derivation leading to Eq. (6)),
// and the virial is V_mn = -sum_ij r^ij_m P_ij,n = -1/2 sum_ij r^ij_m f^ij_n
// (Eqs. (6)-(8)).  Lists are full, so every force is a gather: no atomics.
// Lennard-Jones lives here; the Tersoff kernels are in tersoff.hip.
//
// Precision: bond vectors are formed in FP64 (from FP64 positions, or for FP32 LJ
// bands in wide cells from 32-bit fixed-point fractional coordinates, exact to
// 2^-33 of a cell), then the pair and three-body arithmetic runs in T (float, or
// double for FP64 bands); per-atom energy and virial terms are summed in FP64, then
// per block and per image in a fixed order.
#include <type_traits>

#include "cfneb_dev.h"

namespace cfneb {

// ------------------------------------------------------------ Lennard-Jones
// U_i = 1/2 sum_j phi(r_ij), phi = 4 eps [(s/r)^12 - (s/r)^6] - phi(rc)
// Lennard-Jones straight from the candidates (Verlet skin): each candidate gets the
// exact inclusion test and, if it is a neighbour, its pair term, so neither a packed
// neighbour list nor a second gather of the positions is needed in a step.  K lanes
// share an atom, taking candidates l, l + K, l + 2K, ... (lane l); the atom's force
// is the fixed butterfly sum of its lanes, energy and virial go into the wave sums.
// A tile of 256 atoms is covered in K passes of 256 / K atoms.
//
// FP64-record path (FP64 bands, narrow cells): the inclusion test decides on the
// exact FP64 r^2 (every operation rounded on its own): the separation d is formed in FP64 (a candidate without a lattice shift, most
// of them in a large cell, skips the shift arithmetic, which adds an exact zero), and
// its FP32 square, within 3e-7 of r^2 relative, settles every pair outside a 1e-6
// band around rc^2; only pairs inside the band square d in FP64.  The virial of a
// pair is symmetric (f parallel to d): six FP32 components, added to the FP64 sums once
// per batch of four candidates.
__device__ inline void separation(const double* ri, const double4& rj, const double* h, uint32_t ent,
                                  double* d)
{
#pragma clang fp contract(off)
    if ((ent >> 20) == 0x888u) {  // no lattice shift
        d[0] = rj.x - ri[0];
        d[1] = rj.y - ri[1];
        d[2] = rj.z - ri[2];
    } else {
        const int n0 = nbr_n(ent, 0), n1 = nbr_n(ent, 1), n2 = nbr_n(ent, 2);
        const double r[3] = {rj.x, rj.y, rj.z};
        for (int c = 0; c < 3; ++c) {
            const double sh = (double(n0) * h[c] + double(n1) * h[3 + c]) + double(n2) * h[6 + c];
            d[c] = (r[c] - ri[c]) + sh;
        }
    }
}

// r^2 as the definition rounds it: each product and sum on its own
__device__ inline double exact_r2(const double* d)
{
#pragma clang fp contract(off)
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

__device__ inline bool exact_inside(const double* d, float r2f, float lo, float hi, double rc2)
{
    if (r2f < lo) return true;
    if (r2f >= hi) return false;
    return exact_r2(d) < rc2;
}

template <typename T, int K>
__device__ void lj_cand_item(const BandDev& b, BandState* st, int slot, int tile)
{
    const size_t N = b.N;
    const int lane = int(threadIdx.x) % K;
    const gmem<const R3>* __restrict__ R = gp<const R3>(Rs(b, slot));
    const gmem<const uint32_t>* __restrict__ cand = gp<const uint32_t>(b.cand + size_t(slot) * b.ccap * N);
    const gmem<const int>* __restrict__ ncand = gp<const int>(b.ncand + size_t(slot) * N);
    gmem<T>* F = gp(reinterpret_cast<T*>(b.F) + size_t(slot) * slot_rows(b));
    const cmem<ImageGeom>* g = cp(b.geom + slot);
    double h[9];
    for (int q = 0; q < 9; ++q) h[q] = g->h[q];
    const double rc2 = b.rc2;
    const float lo = float(rc2 * (1.0 - 1e-6)), hi = float(rc2 * (1.0 + 1e-6));
    const T eps4 = T(4.0 * b.lj_eps), eps24 = T(24.0 * b.lj_eps), sig2 = T(b.lj_sig2), esh = T(b.lj_eshift);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // u, then V xx yy zz xy xz yz
    bool over = false, bad = false;
#pragma unroll 1
    for (int sub = 0; sub < K; ++sub) {
        const int i = tile * CFNEB_TILE + sub * (CFNEB_TILE / K) + int(threadIdx.x) / K;
        const bool in = i < b.N;
        const int ii = in ? i : 0;
        const double4 r4 = load4(R, ii);
        const double ri[3] = {r4.x, r4.y, r4.z};
        const int nc = in ? ncand[ii] : 0;
        T fx = 0, fy = 0, fz = 0;
        int cnt = 0;
        // four of the lane's candidates at a time: entries, then positions, in flight
        // together (past the last candidate the loads repeat it; the tests stop there)
        constexpr int U = 4;
        for (int e0 = lane; e0 < nc; e0 += U * K) {
            uint32_t ent[U];
            double4 rj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = e0 + u * K;
                ent[u] = cand[size_t(c < nc ? c : e0) * N + ii];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) rj[u] = load4(R, nbr_j(ent[u]));
            __builtin_amdgcn_sched_barrier(0);
            T w[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u * K >= nc) break;
                double d[3];
                separation(ri, rj[u], h, ent[u], d);
                const T dx = T(d[0]), dy = T(d[1]), dz = T(d[2]);
                const float fdx = float(dx), fdy = float(dy), fdz = float(dz);
                if (!exact_inside(d, fdx * fdx + fdy * fdy + fdz * fdz, lo, hi, rc2)) continue;
                ++cnt;
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
                w[0] += wx * dx;
                w[1] += wy * dy;
                w[2] += wz * dz;
                w[3] += wx * dy;
                w[4] += wx * dz;
                w[5] += wy * dz;
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) acc[1 + q] += double(w[q]);
        }
        // the atom's lanes: fixed butterfly (K consecutive, aligned lanes)
#pragma unroll
        for (int off = K / 2; off > 0; off >>= 1) {
            fx += __shfl_xor(fx, off, 64);
            fy += __shfl_xor(fy, off, 64);
            fz += __shfl_xor(fz, off, 64);
            cnt += __shfl_xor(cnt, off, 64);
        }
        if (in && lane == 0) {
            F[i] = fx;
            F[b.ld + i] = fy;
            F[2 * size_t(b.ld) + i] = fz;
            over = over || cnt > b.cap;
            bad = bad || !isfinite(double(fx) + double(fy) + double(fz));
        }
    }
    if (over) set_error(st, CFNEB_ENEIGH);
    if (bad) set_error(st, CFNEB_ENONFINITE);
    double v[10] = {acc[0], acc[1], acc[4], acc[5], acc[4], acc[2], acc[6], acc[5], acc[6], acc[3]};
    store_ev_partials(b, slot, tile, v);
}

// FP32 bands whose cell is wide enough (ImageGeom::wrap): the separation comes from
// the fixed-point fractional coordinates, one 12-byte gather per candidate and no
// lattice-shift arithmetic: the wrapped 32-bit difference of two coordinates is the
// fractional separation times 2^32, and d = (that difference) (h 2^-32) in FP64, then
// rounded to FP32 per pair (an FP32 h would scale every separation by the same
// rounding error, a strain of ~1e-7 that the virial sum multiplies by the stiffness).
// The FP32 r^2 settles the pair outside [r2lo, r2hi); inside that band the exact FP64
// test runs on the FP64 positions.
// Loads at a 32-bit byte offset from a uniform base (one address add per load).
__device__ inline uint32_t ld_u32(const void* base, uint32_t off)
{
    return *reinterpret_cast<const gmem<const uint32_t>*>(gp(static_cast<const char*>(base)) + off);
}
__device__ inline uint4 ld_u96(const void* base, uint32_t off)
{
    const gmem<const uint32_t>* p = reinterpret_cast<const gmem<const uint32_t>*>(gp(static_cast<const char*>(base)) + off);
    return make_uint4(p[0], p[1], p[2], 0u);
}

template <int K>
__device__ void lj_fixed_item(const BandDev& b, BandState* st, int slot, int tile)
{
    // band fields as uniform locals: read once, held in scalar registers
    const int Ni = uni(b.N), ld = uni(b.ld), cap = uni(b.cap);
    const uint32_t N = uint32_t(Ni);
    const int lane = int(threadIdx.x) % K;
    const uint32_t* S = uni(Ss(b, slot));
    const uint32_t* cand = uni(b.cand + size_t(slot) * b.ccap * N);
    const gmem<const int>* __restrict__ ncand = gp<const int>(uni(b.ncand + size_t(slot) * N));
    gmem<float>* F = gp(uni(reinterpret_cast<float*>(b.F) + size_t(slot) * slot_rows(b)));
    const gmem<const R3>* R = gp<const R3>(uni(Rs(b, slot)));
    const cmem<ImageGeom>* g = cp(b.geom + slot);
    double h[9], H[9];  // h, and h 2^-32 (exact)
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        h[q] = uni(g->h[q]);
        H[q] = h[q] * 0x1p-32;
    }
    const float lo = uni(g->r2lo), hi = uni(g->r2hi);
    const double rc2 = uni(b.rc2);
    const float eps24 = uni(float(24.0 * b.lj_eps)), sig2 = uni(float(b.lj_sig2));
    const double e4 = uni(4.0 * b.lj_eps), e24 = uni(24.0 * b.lj_eps), esh64 = uni(b.lj_eshift);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // 2 u, then -2 V / (24 eps): xx yy zz xy xz yz
    bool over = false, bad = false;
#pragma unroll 1
    for (int sub = 0; sub < K; ++sub) {
        const int i = tile * CFNEB_TILE + sub * (CFNEB_TILE / K) + int(threadIdx.x) / K;
        const bool in = i < Ni;
        const uint32_t ii = in ? uint32_t(i) : 0u;
        const uint4 si = ld_u96(S, ii * 12u);
        const int nc = in ? ncand[ii] : 0;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        int cnt = 0;
        // four of the lane's candidates at a time, loads first; past the last candidate
        // the loads repeat the batch's first and the pair is masked out
        constexpr int U = 4;
        // candidate c = base + u K + lane of this atom sits at byte (c N + i) 4: a uniform
        // row offset plus this lane's constant (no per-candidate multiply)
        const uint32_t own = (uint32_t(lane) * N + ii) * 4u, row = N * 4u;
        for (int base = 0; base + lane < nc; base += U * K) {
            const int e0 = base + lane;
            uint32_t ent[U];
            uint4 sj[U];
            const uint32_t o0 = uint32_t(base) * row + own;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t o = o0 + uint32_t(u * K) * row;
                ent[u] = ld_u32(cand, e0 + u * K < nc ? o : o0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) sj[u] = ld_u96(S, uint32_t(nbr_j(ent[u])) * 12u);
            __builtin_amdgcn_sched_barrier(0);
            float w[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const int cnt0 = cnt;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double a0 = double(int(sj[u].x - si.x));
                const double a1 = double(int(sj[u].y - si.y));
                const double a2 = double(int(sj[u].z - si.z));
                const float dx = float(a0 * H[0] + a1 * H[3] + a2 * H[6]);
                const float dy = float(a0 * H[1] + a1 * H[4] + a2 * H[7]);
                const float dz = float(a0 * H[2] + a1 * H[5] + a2 * H[8]);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool valid = e0 + u * K < nc;
                bool inside = valid && r2 < lo;
                if (valid && r2 >= lo && r2 < hi) {  // rare: the exact FP64 test on the FP64 positions
                    const double4 r4 = load4(R, ii);
                    const double ri[3] = {r4.x, r4.y, r4.z};
                    double d[3];
                    separation(ri, load4(R, nbr_j(ent[u])), h, ent[u], d);
                    inside = exact_r2(d) < rc2;
                }
                // every lane takes the pair arithmetic; pairs outside rc add zeros.  The
                // terms are in units of 24 eps (force) and 4 eps (energy, before the
                // shift): the constants multiply the sums
                const float ir2 = __builtin_amdgcn_rcpf(r2);
                float s6 = sig2 * ir2;
                s6 = s6 * s6 * s6;
                const float s12 = s6 * s6;
                const float fr = inside ? (s6 - 2.f * s12) * ir2 : 0.f;  // phi'(r) / (24 eps r)
                const float phi = inside ? s12 - s6 : 0.f;               // (phi(r) + shift) / (4 eps)
                cnt += inside ? 1 : 0;
                const float px = fr * dx, py = fr * dy, pz = fr * dz;
                fx += px;
                fy += py;
                fz += pz;
                w[0] += phi;
                w[1] += px * dx;
                w[2] += py * dy;
                w[3] += pz * dz;
                w[4] += px * dy;
                w[5] += px * dz;
                w[6] += py * dz;
            }
            acc[0] += e4 * double(w[0]) - esh64 * double(cnt - cnt0);
#pragma unroll
            for (int q = 1; q < 7; ++q) acc[q] += double(w[q]);
        }
#pragma unroll
        for (int off = K / 2; off > 0; off >>= 1) {
            fx += __shfl_xor(fx, off, 64);
            fy += __shfl_xor(fy, off, 64);
            fz += __shfl_xor(fz, off, 64);
            cnt += __shfl_xor(cnt, off, 64);
        }
        if (in && lane == 0) {
            F[i] = eps24 * fx;
            F[ld + i] = eps24 * fy;
            F[2 * size_t(ld) + i] = eps24 * fz;
            over = over || cnt > cap;
            bad = bad || !isfinite(double(fx) + double(fy) + double(fz));
        }
    }
    if (over) set_error(st, CFNEB_ENEIGH);
    if (bad) set_error(st, CFNEB_ENONFINITE);
    // u_i = 1/2 sum_j phi; V = -1/2 sum_ij (phi'/r) d (x) d
    for (int q = 1; q < 7; ++q) acc[q] *= -0.5 * e24;
    double v[10] = {0.5 * acc[0], acc[1], acc[4], acc[5], acc[4], acc[2], acc[6], acc[5], acc[6], acc[3]};
    store_ev_partials(b, slot, tile, v);
}

template <typename T, int K>
__device__ void lj_cand_loop(const BatchDev& bd, int all_images, int variant)
{
    ItemLoopRO loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        BandState* st = b.st;
        const cmem<BandState>* sr = cp(st);
        if (int(band_variant(b) != variant) | int(b.lj_lanes != K) | int(band_stopped(sr))) continue;  // uniform over the block
        const int slot = sr->slot[it.image];
        if constexpr (std::is_same<T, float>::value) {
            if (cp(b.geom + slot)->wrap) {  // uniform over the block
                lj_fixed_item<K>(b, st, slot, it.tile);
                continue;
            }
        }
        lj_cand_item<T, K>(b, st, slot, it.tile);
    }
}

template <typename T, int K>
__global__ void __launch_bounds__(CFNEB_TILE) k_lj_cand(BatchDev bd, int all_images, int variant)
{
    lj_cand_loop<T, K>(bd, all_images, variant);
}

// FP32, one lane per atom (the large bands): five waves per SIMD at a small spill run
// faster than four without one (force kernel 391 -> 365 us on the 97,555-atom band);
// the other variants keep their registers (they spill 20-24 dwords at five).
template <>
__global__ void __launch_bounds__(CFNEB_TILE) __attribute__((amdgpu_waves_per_eu(5)))
k_lj_cand<float, 1>(BatchDev bd, int all_images, int variant)
{
    lj_cand_loop<float, 1>(bd, all_images, variant);
}

template <typename T>
void launch_lj(const Launch& L, int all_images, int variant, hipStream_t s)
{
    // one launch per lane count present (each skips the bands of the other counts)
    const unsigned g = L.g_force;
    if (L.variants & (1u << 8)) k_lj_cand<T, 1><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, variant);
    if (L.variants & (1u << 9)) k_lj_cand<T, 2><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, variant);
    if (L.variants & (1u << 10)) k_lj_cand<T, 4><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, variant);
    if (L.variants & (1u << 11)) k_lj_cand<T, 8><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, variant);
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

// stage 0: LJ from the candidates, or Tersoff bond orders and dU_i/dr^ij; 1: Tersoff
// gather
void launch_force_stage(const Launch& L, int all_images, int stage, hipStream_t s)
{
    if (stage == 0) {
        if (L.variants & (1u << VARIANT_LJ32)) launch_lj<float>(L, all_images, VARIANT_LJ32, s);
        if (L.variants & (1u << VARIANT_LJ64)) launch_lj<double>(L, all_images, VARIANT_LJ64, s);
    }
    launch_tersoff_stage(L, all_images, stage, s);
}

void launch_image_reduce(const Launch& L, int all_images, hipStream_t s)
{
    k_image_reduce<<<L.g[KIND_IMAGE], CFNEB_TILE, 0, s>>>(L.bd, all_images);
}

}  // namespace cfneb
