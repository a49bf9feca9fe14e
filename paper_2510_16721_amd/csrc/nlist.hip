// Per-image cell lists, candidate lists and full neighbour lists.
//
// The neighbours of atom i are every (j, n) != (i, 0) with
//     r = (R_j - R_i) + ((n0 h_0 + n1 h_1) + n2 h_2),  (r_x r_x + r_y r_y) + r_z r_z < rc^2,
// evaluated in FP64 with every operation rounded on its own (no contraction), on the
// unwrapped positions R = R~ D.  This is the local environment of Sec. II.B, Eq. (4).
//
// Candidates (Verlet skin): a cell-list scan keeps every pair closer than
// rcl = rc + skin; each step re-tests the candidates with the exact inclusion test
// above, so the neighbour set is the one a full scan would give.  The candidates are
// rebuilt when a pair could have come from outside rcl: with h = h_ref (I + E) and
// d_i = |R_i - R_i,ref (I + E)|, a pair's separation at the build is at most
// (r + d_i + d_j) / (1 - |E|), so 2 max d_i + rcl |E| < skin keeps the list complete.
// R_ref is kept in FP32: each component within 2^-24 of its magnitude, so d_i measured
// against it is within 2^-24 |R_ref,i| (1 + |E|) of the true one, added to the bound.
//
// Kernels, in order (each a persistent walk over the items of every live band):
//   k_skin_check   (steps) the previous step's move of the atom rows; R = R~ D (and
//                  its fixed-point fractional coordinates); max_i d_i^2 per 1024-atom tile
//   k_skin_decide  max over an image's tiles, rebuild flag per image; a rebuild takes
//                  the current cell as reference
//   k_bin_assign   (rebuilds) wrapped fractional coordinate, bin id; the count atomic
//                  returns the atom's rank inside its bin
//   k_bin_scan     (rebuilds) exclusive prefix sum of the bin counts (one block per
//                  image, 4096 counts per pass, coalesced); zeroes the counts
//   k_bin_scatter  (rebuilds) atom -> bin-ordered 32-byte record (position, id, image)
//   k_bin_sort     (rebuilds) sort each bin by atom id, so lists are deterministic
//   k_cand         (rebuilds) stencil walk over bin-ordered records, pairs within rcl,
//                  packed entry-major candidate lists; R_ref = R (threads take atoms in
//                  bin order when the bins are half-width)
//   k_filter       (host readouts only: the force kernels test their candidates
//                  themselves) exact test of every candidate, packed entry-major
//                  neighbour lists (entry e of atom i at [e][i])
#include <type_traits>

#include "cfneb_dev.h"

namespace cfneb {

__device__ inline size_t bin_base(const BandDev& b, int slot) { return size_t(slot) * (b.nbcap + 1); }

__device__ inline long long pack_info(int j, int n0, int n1, int n2)
{
    return (long long)j | ((long long)(n0 + 512) << 20) | ((long long)(n1 + 512) << 30) |
           ((long long)(n2 + 512) << 40);
}
__device__ inline int info_j(long long v) { return int(v & 0xFFFFF); }
__device__ inline int info_n(long long v, int k) { return int((v >> (20 + 10 * k)) & 0x3FF) - 512; }

// Fractional coordinates s = R h^-1 wrapped to [0, 1) and rounded to multiples of
// 2^-32 (1.0 wraps to 0); a non-finite coordinate gives 0 (the energy check reports
// the band).
__device__ inline uint4 fixed_fraction(const double* r, const double* hi)
{
    uint32_t u[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double s = (r[0] * hi[q] + r[1] * hi[3 + q]) + r[2] * hi[6 + q];
        const double t = isfinite(s) ? s - floor(s) : 0.0;
        u[q] = uint32_t((unsigned long long)(long long)rint(t * 0x1p32));
    }
    return make_uint4(u[0], u[1], u[2], 0u);
}

// 1024 atoms per item, four per thread: all loads of the four atoms are issued before
// any position is stored.  In a step, first the previous step's pending move of these
// atom rows (X += scale dt v', written back); R = R~ D (and its fixed-point fractional
// coordinates for FP32 LJ bands); d_i^2 against the strained reference when a list
// exists; the tile's maximum goes to its own slot (no atomics: many tiles per image
// would contend on one address).
__global__ void __launch_bounds__(CFNEB_TILE) k_skin_check(BatchDev bd, int all_images)
{
    __shared__ double lds[(CFNEB_TILE / 64) * 2];
    constexpr int Q = CFNEB_TILE4 / CFNEB_TILE;
    ItemLoopRO loop(bd, KIND_ATOM4, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        const cmem<BandState>* st = cp(b.st);
        if (band_stopped(st)) continue;  // uniform over the block
        const int slot = st->slot[it.image];
        const cmem<ImageGeom>* g = cp(b.geom + slot);
        double D[9], E[9], hi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            D[q] = g->D[q];
            E[q] = g->E[q];
            hi[q] = g->hinv[q];
        }
        const bool valid = cp(b.skst + slot)->valid != 0;
        gmem<uint32_t>* __restrict__ S = b.S ? gp(Ss(b, slot)) : nullptr;
        gmem<double>* __restrict__ X = gp(Xs(b, slot));
        const gmem<const float>* __restrict__ Rr = gp<const float>(b.Rref + size_t(slot) * slot_rows(b));
        double x[Q][3], a[Q][3];
        if (move_pending(st, all_images)) {  // uniform over the block
            // the previous step's move of these rows: X += scale (dt v')
            const gmem<const double>* __restrict__ V = gp<const double>(Vs(b, st->vcur, slot));
            const double sc = st->scale, dt = st->dt;
            double v[Q][3];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = it.tile * CFNEB_TILE4 + q * CFNEB_TILE + threadIdx.x;
                const bool in = i < b.N;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[q][c] = in ? X[size_t(c) * b.ld + i] : 0.0;
                    v[q][c] = in ? V[size_t(c) * b.ld + i] : 0.0;
                    a[q][c] = (in && valid) ? double(Rr[size_t(c) * b.ld + i]) : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = it.tile * CFNEB_TILE4 + q * CFNEB_TILE + threadIdx.x;
                if (i >= b.N) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[q][c] += sc * (dt * v[q][c]);
                    X[size_t(c) * b.ld + i] = x[q][c];
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = it.tile * CFNEB_TILE4 + q * CFNEB_TILE + threadIdx.x;
                const bool in = i < b.N;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[q][c] = in ? X[size_t(c) * b.ld + i] : 0.0;
                    a[q][c] = (in && valid) ? double(Rr[size_t(c) * b.ld + i]) : 0.0;
                }
            }
        }
        // max d_i^2 against the FP32 reference, and max |R_ref,i|^2 for its rounding
        double m[2] = {0.0, 0.0};
        gmem<R3>* __restrict__ R = gp(Rs(b, slot));
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = it.tile * CFNEB_TILE4 + q * CFNEB_TILE + threadIdx.x;
            if (i >= b.N) continue;
            double r[3];
            for (int c = 0; c < 3; ++c) r[c] = (x[q][0] * D[c] + x[q][1] * D[3 + c]) + x[q][2] * D[6 + c];
            store3(R, i, r[0], r[1], r[2]);
            if (S) {
                const uint4 f = fixed_fraction(r, hi);
                S[3 * size_t(i)] = f.x;
                S[3 * size_t(i) + 1] = f.y;
                S[3 * size_t(i) + 2] = f.z;
            }
            if (valid) {
                double d2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double ref = a[q][c] + ((a[q][0] * E[c] + a[q][1] * E[3 + c]) + a[q][2] * E[6 + c]);
                    const double d = r[c] - ref;
                    d2 += d * d;
                }
                m[0] = fmax(m[0], d2);
                m[1] = fmax(m[1], (a[q][0] * a[q][0] + a[q][1] * a[q][1]) + a[q][2] * a[q][2]);
            }
        }
        block_max<2>(m, lds);
        if (threadIdx.x == 0) {
            double* out = b.skmax + (size_t(slot) * kind_tiles(b, KIND_ATOM4) + it.tile) * 2;
            out[0] = m[0];
            out[1] = m[1];
        }
    }
}

// One block per band, sixteen threads per image: the maximum over the image's tile
// maxima (max is exact in any order), then the decision.
__global__ void __launch_bounds__(16 * CFNEB_MAX_IMAGES) k_skin_decide(BatchDev bd, int all_images)
{
    ItemLoop loop(bd, KIND_BAND, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        const int k = threadIdx.x >> 4, lane = threadIdx.x & 15;
        // the geometry and skin passes have applied the pending move
        if (threadIdx.x == 0 && all_images == 0) st->move = 0;
        const bool act = !band_stopped(st) && k < b.Mcap && image_active(st, k, all_images);
        const int slot = act ? st->slot[k] : 0;
        const int nt = kind_tiles(b, KIND_ATOM4);
        double m = 0.0, ma = 0.0;
        if (act) {
            const gmem<const double>* mx = gp<const double>(b.skmax + size_t(slot) * nt * 2);
#pragma unroll 4
            for (int t = lane; t < nt; t += 16) {
                m = fmax(m, mx[2 * t]);
                ma = fmax(ma, mx[2 * t + 1]);
            }
        }
        for (int off = 8; off > 0; off >>= 1) {
            m = fmax(m, __shfl_xor(m, off, 16));
            ma = fmax(ma, __shfl_xor(ma, off, 16));
        }
        if (!act || lane != 0) continue;
        SkinState& sk = b.skst[slot];
        const ImageGeom& g = b.geom[slot];
        bool rebuild = true;
        // the FP32 reference is within 2^-24 |R_ref,i| of the build positions, so every
        // displacement is within that times (1 + |E|) of the one measured against it
        const double dmax = sqrt(m) + 0x1p-24 * (1.0 + 1e-6) * sqrt(ma) * (1.0 + g.enorm);
        if (b.skin > 0.0 && sk.valid) rebuild = !(2.0 * dmax + b.rcl * g.enorm < b.skin * (1.0 - 1e-6));
        sk.rebuild = rebuild ? 1 : 0;
        if (rebuild) {
            for (int q = 0; q < 9; ++q) {
                sk.href[q] = g.h[q];
                sk.hrefinv[q] = g.hinv[q];
            }
            sk.valid = 1;
            *rebuild_flag(bd) = 1;
        }
    }
}

__device__ void bin_assign_item(const BandDev& b, int slot, int i)
{
    const ImageGeom& g = b.geom[slot];
    const double4 ri = load4(gp<const R3>(Rs(b, slot)), i);
    const double r[3] = {ri.x, ri.y, ri.z};
    int bi[3], img[3];
    for (int q = 0; q < 3; ++q) {
        const double s = (r[0] * g.hinv[q] + r[1] * g.hinv[3 + q]) + r[2] * g.hinv[6 + q];
        double fl = floor(s);
        if (!isfinite(fl) || fabs(fl) > 500.0) fl = 0.0;  // non-finite input: caught by the energy check
        img[q] = int(fl);
        const double sw = s - fl;
        int bq = int(floor(sw * g.nb[q]));
        bq = bq < 0 ? 0 : (bq >= g.nb[q] ? g.nb[q] - 1 : bq);
        bi[q] = bq;
    }
    const int bin = (bi[0] * g.nb[1] + bi[1]) * g.nb[2] + bi[2];
    const int rank = atomicAdd(&b.bcount[bin_base(b, slot) + bin], 1);
    const int packed = (img[0] + 512) | ((img[1] + 512) << 10) | ((img[2] + 512) << 20);
    b.binfo[size_t(slot) * b.N + i] = make_int4(bin, rank, packed, 0);
}

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_assign(BatchDev bd, int all_images)
{
    if (*rebuild_flag(bd) == 0) return;  // no image rebuilds this step
    ItemLoop loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        const int i = it.tile * CFNEB_TILE + threadIdx.x;
        if (band_stopped(st) || i >= b.N) continue;
        const int slot = st->slot[it.image];
        if (!b.skst[slot].rebuild) continue;
        bin_assign_item(b, slot, i);
    }
}

// Exclusive scan of one image's counts, 4 per thread and 4096 per pass.
__device__ void bin_scan_item(const BandDev& b, int slot)
{
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int nbins = b.geom[slot].nbins;
    int* cnt = b.bcount + bin_base(b, slot);
    int* start = b.bstart + bin_base(b, slot);
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int carry = 0;
    for (int base = 0; base < nbins; base += 4096) {
        const int idx = base + 4 * t;
        int c[4];
        for (int q = 0; q < 4; ++q) c[q] = (idx + q < nbins) ? cnt[idx + q] : 0;
        const int s1 = c[0] + c[1], s2 = s1 + c[2], tot = s2 + c[3];
        int incl = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        if (t == 0) {
            int run = 0;
            for (int w = 0; w < 16; ++w) {
                const int v = wsum[w];
                wsum[w] = run;
                run += v;
            }
            carry_s = run;
        }
        __syncthreads();
        const int excl = carry + wsum[wid] + incl - tot;
        const int pre[4] = {0, c[0], s1, s2};
        for (int q = 0; q < 4; ++q)
            if (idx + q < nbins) {
                start[idx + q] = excl + pre[q];
                cnt[idx + q] = 0;
            }
        carry += carry_s;
        __syncthreads();
    }
    if (t == 0) start[nbins] = carry;
}

__global__ void __launch_bounds__(1024) k_bin_scan(BatchDev bd, int all_images)
{
    if (*rebuild_flag(bd) == 0) return;  // no image rebuilds this step
    ItemLoop loop(bd, KIND_IMAGE, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        if (band_stopped(b.st)) continue;  // uniform over the block
        const int slot = b.st->slot[it.image];
        if (!b.skst[slot].rebuild) continue;  // uniform over the block
        bin_scan_item(b, slot);
    }
}

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_scatter(BatchDev bd, int all_images)
{
    if (*rebuild_flag(bd) == 0) return;  // no image rebuilds this step
    ItemLoop loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        const int i = it.tile * CFNEB_TILE + threadIdx.x;
        if (band_stopped(st) || i >= b.N) continue;
        const int slot = st->slot[it.image];
        if (!b.skst[slot].rebuild) continue;
        const int4 bi = b.binfo[size_t(slot) * b.N + i];
        const int pos = b.bstart[bin_base(b, slot) + bi.x] + bi.y;
        if (pos < 0 || pos >= b.N) continue;
        const double4 ri = load4(gp<const R3>(Rs(b, slot)), i);
        BinAtom a;
        a.x = ri.x;
        a.y = ri.y;
        a.z = ri.z;
        a.info = pack_info(i, (bi.z & 0x3FF) - 512, ((bi.z >> 10) & 0x3FF) - 512, ((bi.z >> 20) & 0x3FF) - 512);
        b.bpos[size_t(slot) * b.N + pos] = a;
    }
}

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_sort(BatchDev bd, int all_images)
{
    if (*rebuild_flag(bd) == 0) return;  // no image rebuilds this step
    ItemLoop loop(bd, KIND_BIN, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        const int bin = it.tile * CFNEB_TILE + threadIdx.x;
        if (band_stopped(st)) continue;
        const int slot = st->slot[it.image];
        if (!b.skst[slot].rebuild || bin >= b.geom[slot].nbins) continue;
        const int* start = b.bstart + bin_base(b, slot);
        BinAtom* a = b.bpos + size_t(slot) * b.N;
        const int lo = start[bin], hi = min(start[bin + 1], b.N);
        for (int p = lo + 1; p < hi; ++p) {
            const BinAtom v = a[p];
            const int key = info_j(v.info);
            int q = p - 1;
            while (q >= lo && info_j(a[q].info) > key) {
                a[q + 1] = a[q];
                --q;
            }
            a[q + 1] = v;
        }
    }
}

__device__ inline void wrap_bin(int v, int nb, int& a, int& m)
{
    // periodic wrap without division (the stencil reach is small)
    a = v;
    m = 0;
    while (a < 0) {
        a += nb;
        --m;
    }
    while (a >= nb) {
        a -= nb;
        ++m;
    }
}

// Candidates of atom i: every (j, n) within rcl, in stencil order; R_ref = R.
// A run of bin records is read four at a time (the loads of a batch are in flight
// together); with a one-bin stencil and no wrap along the third axis, the bounds of
// all nine runs are read before the first run.
__device__ void cand_item(const BandDev& b, BandState* st, int slot, int i)
{
    const ImageGeom& g = b.geom[slot];
    const double4 r4 = load4(gp<const R3>(Rs(b, slot)), i);
    const gmem<const int>* __restrict__ start = gp<const int>(b.bstart + bin_base(b, slot));
    const gmem<const double4>* __restrict__ bp =
        gp<const double4>(reinterpret_cast<const double4*>(b.bpos + size_t(slot) * b.N));
    const size_t N = b.N;
    gmem<uint32_t>* __restrict__ cand = gp(b.cand + size_t(slot) * b.ccap * N);

    double h[9];
    for (int q = 0; q < 9; ++q) h[q] = g.h[q];
    const double ri[3] = {r4.x, r4.y, r4.z};
    gmem<float>* __restrict__ Rr = gp(b.Rref + size_t(slot) * slot_rows(b));
    Rr[i] = float(ri[0]);
    Rr[b.ld + i] = float(ri[1]);
    Rr[2 * size_t(b.ld) + i] = float(ri[2]);
    const int4 me = b.binfo[size_t(slot) * N + i];
    const int im0 = (me.z & 0x3FF) - 512, im1 = ((me.z >> 10) & 0x3FF) - 512, im2 = ((me.z >> 20) & 0x3FF) - 512;
    const int nb0 = g.nb[0], nb1 = g.nb[1], nb2 = g.nb[2];
    const int b0 = me.x / (nb1 * nb2), b1 = (me.x / nb2) % nb1, b2 = me.x % nb2;
    const int r0 = g.reach[0], r1 = g.reach[1], r2 = g.reach[2];
    const double rcl2 = b.rcl2;
    const int ccap = b.ccap, natoms = b.N;
    int cnt = 0;
    bool bad_shift = false;
    // records lo..hi-1 of the bin-ordered array, seen from bin shift (m0, m1, m2)
    auto scan = [&](int lo, int hi, int m0, int m1, int m2) {
        hi = min(hi, natoms);
        constexpr int U = 4;
        for (int p0 = lo; p0 < hi; p0 += U) {
            double4 a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = load4(bp, min(p0 + u, hi - 1));
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p0 + u >= hi) break;
                const long long info = __double_as_longlong(a[u].w);
                const int j = info_j(info);
                const int n0 = m0 + im0 - info_n(info, 0);
                const int n1 = m1 + im1 - info_n(info, 1);
                const int n2 = m2 + im2 - info_n(info, 2);
                if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                double d[3];
                const double rr = exact_r2(ri, a[u].x, a[u].y, a[u].z, h, n0, n1, n2, d);
                if (!(rr < rcl2)) continue;
                if (abs(n0) > CFNEB_MAX_SHIFT || abs(n1) > CFNEB_MAX_SHIFT || abs(n2) > CFNEB_MAX_SHIFT) {
                    bad_shift = true;
                    continue;
                }
                if (cnt < ccap) cand[size_t(cnt) * N + i] = pack_nbr(j, n0, n1, n2);
                ++cnt;
            }
        }
    };
    // The z bins b2-r2 .. b2+r2 of a row are one contiguous run of records unless the
    // stencil wraps; then each bin is its own segment.
    const bool flat = (b2 - r2 >= 0) && (b2 + r2 < nb2);
    if (flat && r0 == 1 && r1 == 1) {
        int lo[9], hi[9], m0s[9], m1s[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            int a0, a1;
            wrap_bin(b0 + q / 3 - 1, nb0, a0, m0s[q]);
            wrap_bin(b1 + q % 3 - 1, nb1, a1, m1s[q]);
            const int row = (a0 * nb1 + a1) * nb2;
            lo[q] = start[row + b2 - r2];
            hi[q] = start[row + b2 + r2 + 1];
        }
        for (int q = 0; q < 9; ++q) scan(lo[q], hi[q], m0s[q], m1s[q], 0);
    } else {
        for (int dx = -r0; dx <= r0; ++dx) {
            int a0, m0;
            wrap_bin(b0 + dx, nb0, a0, m0);
            for (int dy = -r1; dy <= r1; ++dy) {
                int a1, m1;
                wrap_bin(b1 + dy, nb1, a1, m1);
                const int row = (a0 * nb1 + a1) * nb2;
                const int nseg = flat ? 1 : 2 * r2 + 1;
                for (int sgi = 0; sgi < nseg; ++sgi) {
                    if (flat) {
                        scan(start[row + b2 - r2], start[row + b2 + r2 + 1], m0, m1, 0);
                    } else {
                        int a2, m2;
                        wrap_bin(b2 - r2 + sgi, nb2, a2, m2);
                        scan(start[row + a2], start[row + a2 + 1], m0, m1, m2);
                    }
                }
            }
        }
    }
    b.ncand[size_t(slot) * N + i] = min(cnt, ccap);
    if (bad_shift) set_error(st, CFNEB_ECELL);
    if (cnt > ccap) set_error(st, CFNEB_ENEIGH);
}

__global__ void __launch_bounds__(CFNEB_TILE) k_cand(BatchDev bd, int all_images)
{
    if (*rebuild_flag(bd) == 0) return;  // no image rebuilds this step
    ItemLoop loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        const int p = it.tile * CFNEB_TILE + threadIdx.x;
        if (band_stopped(st) || p >= b.N) continue;
        const int slot = st->slot[it.image];
        if (!b.skst[slot].rebuild) continue;
        // with half-width bins (dense systems) threads take the atoms in bin order
        // (record p of the sorted bins), so the lanes of a wave share their stencil
        // rows; each atom's list is the same in either order
        int i = p;
        if (b.geom[slot].sub == 2) {
            const double4 rec =
                load4(gp<const double4>(reinterpret_cast<const double4*>(b.bpos + size_t(slot) * b.N)), p);
            i = info_j(__double_as_longlong(rec.w));
        }
        cand_item(b, st, slot, i);
    }
}

// Exact test of atom i's candidates with the current R and h: the packed neighbour
// list.  Four candidates at a time: their entries, then their positions, are in
// flight together before any test (past the last candidate the loads repeat it, so
// no branch separates them; the tests stop there).
__device__ void filter_item(const BandDev& b, BandState* st, int slot, int i)
{
    const ImageGeom& g = b.geom[slot];
    const gmem<const R3>* __restrict__ R = gp<const R3>(Rs(b, slot));
    const size_t N = b.N;
    const gmem<const uint32_t>* __restrict__ cand = gp<const uint32_t>(b.cand + size_t(slot) * b.ccap * N);
    gmem<uint32_t>* __restrict__ nbr = gp(b.nbr + size_t(slot) * b.cap * N);
    double h[9];
    for (int q = 0; q < 9; ++q) h[q] = g.h[q];
    const double4 r4 = load4(R, i);
    const double ri[3] = {r4.x, r4.y, r4.z};
    const int nc = gp<const int>(b.ncand)[size_t(slot) * N + i];
    const double rc2 = b.rc2;
    const int cap = b.cap;
    int cnt = 0;
    constexpr int U = 4;
    for (int e0 = 0; e0 < nc; e0 += U) {
        uint32_t ent[U];
        double4 rj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ent[u] = cand[size_t(min(e0 + u, nc - 1)) * N + i];
#pragma unroll
        for (int u = 0; u < U; ++u) rj[u] = load4(R, nbr_j(ent[u]));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e0 + u >= nc) break;
            double d[3];
            const double rr = exact_r2(ri, rj[u].x, rj[u].y, rj[u].z, h, nbr_n(ent[u], 0), nbr_n(ent[u], 1),
                                       nbr_n(ent[u], 2), d);
            if (!(rr < rc2)) continue;
            if (cnt < cap) nbr[size_t(cnt) * N + i] = ent[u];
            ++cnt;
        }
    }
    gp(b.ncnt)[size_t(slot) * N + i] = cnt;
    if (cnt > cap) set_error(st, CFNEB_ENEIGH);
}

// vmask: the band variants (potential, force precision) this launch serves
__global__ void __launch_bounds__(CFNEB_TILE) k_filter(BatchDev bd, int all_images, unsigned vmask, int ignore_stop)
{
    ItemLoop loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        if (!((vmask >> band_variant(b)) & 1u)) continue;
        BandState* st = b.st;
        const int i = it.tile * CFNEB_TILE + threadIdx.x;
        if ((!ignore_stop && band_stopped(st)) || i >= b.N) continue;
        filter_item(b, st, st->slot[it.image], i);
    }
}

__global__ void k_skin_hold(BatchDev bd, int hold)
{
    for (int q = int(blockIdx.x); q < bd.cap; q += int(gridDim.x)) {
        if (!bd.live[q]) continue;
        const BandDev& b = bd.bands[q];
        for (int slot = int(threadIdx.x); slot < b.Mcap; slot += int(blockDim.x)) {
            SkinState& sk = b.skst[slot];
            if (hold) {
                sk.held = sk.rebuild;
                sk.rebuild = 0;
            } else {
                sk.rebuild = sk.held;
            }
        }
    }
}

void launch_skin_hold(const Launch& L, int hold, hipStream_t s)
{
    k_skin_hold<<<L.g[KIND_BAND], 64, 0, s>>>(L.bd, hold);
}

void launch_skin(const Launch& L, int all_images, hipStream_t s)
{
    k_skin_check<<<L.g[KIND_ATOM4], CFNEB_TILE, 0, s>>>(L.bd, all_images);
    k_skin_decide<<<L.g[KIND_BAND], 16 * CFNEB_MAX_IMAGES, 0, s>>>(L.bd, all_images);
}

void launch_bins(const Launch& L, int all_images, hipStream_t s)
{
    k_bin_assign<<<L.g[KIND_ATOM], CFNEB_TILE, 0, s>>>(L.bd, all_images);
    k_bin_scan<<<L.g[KIND_IMAGE], 1024, 0, s>>>(L.bd, all_images);
    k_bin_scatter<<<L.g[KIND_ATOM], CFNEB_TILE, 0, s>>>(L.bd, all_images);
    k_bin_sort<<<L.g[KIND_BIN], CFNEB_TILE, 0, s>>>(L.bd, all_images);
}

void launch_list(const Launch& L, int all_images, hipStream_t s)
{
    k_cand<<<L.g[KIND_ATOM], CFNEB_TILE, 0, s>>>(L.bd, all_images);
}

// The force kernels of both potentials test their candidates themselves; a step
// writes no packed neighbour list.
void launch_filter(const Launch& L, int all_images, hipStream_t s)
{
    (void)L;
    (void)all_images;
    (void)s;
}

// Packed neighbour lists of every image of the table, for a host readout (the step
// path keeps candidates only): the exact test of the current candidates on the
// positions and cell of the last evaluation.
void launch_neighbour_lists(const Launch& L, hipStream_t s)
{
    launch_plan(L, 1, 1, s);
    k_filter<<<L.g[KIND_ATOM], CFNEB_TILE, 0, s>>>(L.bd, 1, (1u << NVARIANT) - 1u, 1);
}

}  // namespace cfneb
