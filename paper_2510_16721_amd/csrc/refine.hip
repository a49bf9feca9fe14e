// Adaptive image insertion and deletion (Sec. III) and the band readout.
//
// The paper adjusts the image distribution after iterations from the local spacing
// of images in configuration space.  Here the squared spacing of every interval,
//     d_k^2 = sum over all (N+3) x 3 entries of (X_{k+1} - X_k)^2,
// is summed exactly: each rounded FP64 term is converted without error to an
// unsigned fixed-point integer in units of 2^-64 (terms must lie in [0, 2^40)) and
// the integers are added, so the sum does not depend on the reduction order and
// every decision is bit-reproducible.  Rule, with M images and S = sum_k d_k^2:
//   insert the midpoint of the longest interval k* (lowest index on ties) if
//       M < max_images and ins_den (M-1) d_k*^2 > ins_num S;
//   otherwise delete the moving image j* (not the climbing image) whose longer
//   neighbouring interval is shortest (lowest index on ties) if
//       M > min_images and del_den (M-1) max(d_{j*-1}^2, d_j*^2) < del_num S.
// After a change the FIRE velocities are zeroed, alpha and N_P reset, dt kept.
#include "cfneb_dev.h"

namespace cfneb {

struct U128 {
    uint64_t lo, hi;
};

__device__ inline void add128(U128& a, const U128& b)
{
    const uint64_t lo = a.lo + b.lo;
    a.hi += b.hi + (lo < a.lo ? 1u : 0u);
    a.lo = lo;
}

__device__ inline bool less128(const U128& a, const U128& b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// floor(t * 2^64) for 0 <= t < 2^40, exactly, from the bits of t.
__device__ inline bool to_fixed(double t, U128& out)
{
    out.lo = out.hi = 0;
    if (!(t >= 0.0) || !(t < 1099511627776.0)) return false;  // 2^40
    const uint64_t bits = uint64_t(__double_as_longlong(t));
    const int ex = int((bits >> 52) & 0x7FF);
    if (ex == 0) return true;  // zero or subnormal: below 2^-64
    const uint64_t m = (bits & ((uint64_t(1) << 52) - 1)) | (uint64_t(1) << 52);
    const int sh = ex - 1011;  // t * 2^64 = m * 2^(ex - 1075 + 64)
    if (sh >= 0) {
        out.lo = (sh < 64) ? (m << sh) : 0;
        out.hi = (sh == 0) ? 0 : ((sh < 64) ? (m >> (64 - sh)) : (m << (sh - 64)));
    } else {
        const int s = -sh;
        out.lo = (s < 64) ? (m >> s) : 0;
    }
    return true;
}

// 256-bit value as four little-endian limbs.
struct U256 {
    uint64_t w[4];
};

__device__ inline U256 widen(const U128& a)
{
    U256 r = {{a.lo, a.hi, 0, 0}};
    return r;
}

__device__ inline U256 add256(const U256& a, const U256& b)
{
    U256 r;
    uint64_t carry = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t s = a.w[i] + carry;
        const uint64_t c1 = (s < carry) ? 1u : 0u;
        const uint64_t t = s + b.w[i];
        const uint64_t c2 = (t < s) ? 1u : 0u;
        r.w[i] = t;
        carry = c1 + c2;
    }
    return r;
}

__device__ inline U256 mul256_small(const U256& a, uint32_t m)
{
    U256 r;
    uint64_t carry = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t lo = (a.w[i] & 0xFFFFFFFFu) * m;
        const uint64_t hi = (a.w[i] >> 32) * m;
        // a.w[i] * m + carry = hi * 2^32 + lo + carry
        const uint64_t s = lo + (hi << 32);
        uint64_t c = (s < lo) ? 1u : 0u;
        const uint64_t t = s + carry;
        c += (t < s) ? 1u : 0u;
        r.w[i] = t;
        carry = (hi >> 32) + c;
    }
    return r;
}

__device__ inline int cmp256(const U256& a, const U256& b)
{
    for (int i = 3; i >= 0; --i) {
        if (a.w[i] < b.w[i]) return -1;
        if (a.w[i] > b.w[i]) return 1;
    }
    return 0;
}

__device__ inline U128 wave_sum128(U128 v)
{
    for (int off = 32; off > 0; off >>= 1) {
        U128 o;
        o.lo = __shfl_xor(v.lo, off, 64);
        o.hi = __shfl_xor(v.hi, off, 64);
        add128(v, o);
    }
    return v;
}

// Exact squared spacing of one 256-row tile of interval k (images k, k+1).
__device__ void dist_item(const BandDev& b, BandState* st, int k, int tile)
{
    __shared__ U128 lds[4];
    __shared__ int bad[4];
    const int r = tile * CFNEB_TILE + threadIdx.x;
    U128 acc = {0, 0};
    int ok = 1;
    if (r < b.N + 3) {
        const double* Xa = Xs(b, st->slot[k]);
        const double* Xb = Xs(b, st->slot[k + 1]);
        for (int c = 0; c < 3; ++c) {
            const size_t o = size_t(c) * b.ld + r;
            const double d = Xb[o] - Xa[o];
            const double t = d * d;
            U128 q;
            if (!to_fixed(t, q)) ok = 0;
            add128(acc, q);
        }
    }
    acc = wave_sum128(acc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) ok = min(ok, __shfl_xor(ok, off, 64));
    if (lane == 0) {
        lds[wid] = acc;
        bad[wid] = ok;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        U128 s = lds[0];
        add128(s, lds[1]);
        add128(s, lds[2]);
        add128(s, lds[3]);
        uint64_t* out = b.refpart + (size_t(k) * b.ntR + tile) * 2;
        out[0] = s.lo;
        out[1] = s.hi;
        if (!(bad[0] && bad[1] && bad[2] && bad[3])) set_error(st, CFNEB_ERANGE);
    }
    __syncthreads();
}

// mode 0: only when the step set refine_due; mode 1: always (explicit call)
__global__ void __launch_bounds__(CFNEB_TILE) k_refine_dist(BatchDev bd, int mode)
{
    if (mode == 0 && *refine_flag(bd) == 0) return;  // no band is due this step
    ItemLoop loop(bd, KIND_IVAL, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (mode == 0 && (band_stopped(st) || !st->refine_due)) continue;  // uniform
        dist_item(b, st, it.image, it.tile);
    }
}

// mode 0: step-end check of the bands due; mode 1: forced decision.  Both apply the
// decision to the slot table.
__device__ void decide_item(const BandDev& b, BandState* st, int mode)
{
    __shared__ U128 d2[CFNEB_MAX_IMAGES];
    const int M = st->M;
    const int t = threadIdx.x;
    // one wave per interval: integer sums are exact, so the order is free
    const int lane = t & 63, nw = int(blockDim.x) >> 6;
    for (int k = t >> 6; k < M - 1; k += nw) {
        U128 s = {0, 0};
        const uint64_t* p = b.refpart + size_t(k) * b.ntR * 2;
        for (int q = lane; q < b.ntR; q += 64) {
            const U128 v = {p[2 * q], p[2 * q + 1]};
            add128(s, v);
        }
        s = wave_sum128(s);
        if (lane == 0) {
            d2[k] = s;
            st->d2[k] = double(s.hi) + double(s.lo) * 5.421010862427522e-20;  // 2^-64
        }
    }
    __syncthreads();
    if (t == 0) {
        st->ins = -1;
        st->del = -1;
        st->changed = 0;
        if (st->err == 0) {
            U256 total = {{0, 0, 0, 0}};
            int kstar = 0;
            for (int k = 0; k < M - 1; ++k) {
                total = add256(total, widen(d2[k]));
                if (less128(d2[kstar], d2[k])) kstar = k;
            }
            if (M < b.max_images && M < b.Mcap) {
                const U256 lhs = mul256_small(widen(d2[kstar]), uint32_t(b.ins_den) * uint32_t(M - 1));
                const U256 rhs = mul256_small(total, uint32_t(b.ins_num));
                if (cmp256(lhs, rhs) > 0) {
                    bool used[CFNEB_MAX_IMAGES];
                    for (int q = 0; q < CFNEB_MAX_IMAGES; ++q) used[q] = false;
                    for (int q = 0; q < M; ++q) used[st->slot[q]] = true;
                    int fresh = 0;
                    while (fresh < b.Mcap && used[fresh]) ++fresh;
                    const int a = st->slot[kstar], c = st->slot[kstar + 1];
                    for (int q = M; q > kstar + 1; --q) st->slot[q] = st->slot[q - 1];
                    st->slot[kstar + 1] = fresh;
                    st->M = M + 1;
                    st->new_slot = fresh;
                    b.skst[fresh].valid = 0;  // its candidate list is built at the next step
                    st->ins_a = a;
                    st->ins_b = c;
                    st->ins = kstar + 1;
                    st->changed = 1;
                    // until it is evaluated, the new image reports its neighbours' mean
                    b.scal[fresh].H = 0.5 * (b.scal[a].H + b.scal[c].H);
                    b.scal[fresh].E = 0.5 * (b.scal[a].E + b.scal[c].E);
                }
            }
            if (!st->changed && M > b.min_images) {
                int jstar = -1;
                U128 best = {0, 0};
                for (int j = 1; j <= M - 2; ++j) {
                    if (j == st->ci) continue;
                    const U128 m = less128(d2[j - 1], d2[j]) ? d2[j] : d2[j - 1];
                    if (jstar < 0 || less128(m, best)) {
                        jstar = j;
                        best = m;
                    }
                }
                if (jstar >= 0) {
                    const U256 lhs = mul256_small(widen(best), uint32_t(b.del_den) * uint32_t(M - 1));
                    const U256 rhs = mul256_small(total, uint32_t(b.del_num));
                    if (cmp256(lhs, rhs) < 0) {
                        for (int q = jstar; q < M - 1; ++q) st->slot[q] = st->slot[q + 1];
                        st->M = M - 1;
                        st->del = jstar;
                        st->changed = 1;
                    }
                }
            }
            if (st->changed) {
                st->alpha = b.astart;
                st->n_pos = 0;
                st->fresh = 1;
                st->ci = -1;
            }
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_refine_decide(BatchDev bd, int mode)
{
    if (mode == 0 && *refine_flag(bd) == 0) return;  // no band is due this step
    ItemLoop loop(bd, KIND_BAND, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (mode == 0 && (band_stopped(st) || !st->refine_due)) continue;  // uniform
        decide_item(b, st, mode);
    }
}

// Midpoint X_a + (X_b - X_a) / 2 into the new slot; zero velocities after a change.
// Walks every slot of the capacity, since the image count just changed.
__global__ void __launch_bounds__(CFNEB_TILE) k_refine_apply(BatchDev bd, int mode)
{
    if (mode == 0 && *refine_flag(bd) == 0) return;  // no band is due this step
    ItemLoop loop(bd, KIND_SLOTROW, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (mode == 0 && (band_stopped(st) || !st->refine_due)) continue;
        if (!st->changed || st->err != 0) continue;
        const int r = it.tile * CFNEB_TILE + threadIdx.x;
        const int k = it.image;  // logical image after the change
        if (r >= b.N + 3 || k >= st->M) continue;
        const int slot = st->slot[k];
        if (st->ins >= 0 && k == st->ins) {
            const double* Xa = Xs(b, st->ins_a);
            const double* Xb = Xs(b, st->ins_b);
            double* Xn = Xs(b, slot);
            {
#pragma clang fp contract(off)
                for (int c = 0; c < 3; ++c) {
                    const size_t o = size_t(c) * b.ld + r;
                    Xn[o] = Xa[o] + 0.5 * (Xb[o] - Xa[o]);
                }
            }
        }
        double* V = Vs(b, st->vcur, slot);
        for (int c = 0; c < 3; ++c) V[size_t(c) * b.ld + r] = 0.0;
    }
}

// Readout partials of interval k, one 256-row tile: the sum of d^2 over every row and
// the atom-row sums of each component of d = X_{k+1} - X_k (fixed-order block sums),
// at dotpart[(k * ntR + tile) * 4 ...] (the band dots' partials are free outside a step).
__global__ void __launch_bounds__(CFNEB_TILE) k_readout_dist(BatchDev bd)
{
    __shared__ double lds[(CFNEB_TILE / 64) * 4];
    ItemLoop loop(bd, KIND_IVAL, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        const int r = it.tile * CFNEB_TILE + threadIdx.x;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (r < b.N + 3) {
            const double* Xa = Xs(b, st->slot[it.image]);
            const double* Xb = Xs(b, st->slot[it.image + 1]);
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * b.ld + r;
                const double d = Xb[o] - Xa[o];
                v[0] += d * d;
                if (r < b.N) v[1 + c] = d;
            }
        }
        block_sum<4>(v, lds);
        if (threadIdx.x == 0) {
            double* out = b.dotpart + (size_t(it.image) * b.ntR + it.tile) * 4;
            for (int q = 0; q < 4; ++q) out[q] = v[q];
        }
    }
}

// H in logical order, barrier, and the path coordinate xi_k = s_k / s_{M-1}, where
// s is the arc length of the translation-free image differences (the metric of the
// band's springs, tangent and energy profile): |d - mean_atoms(d)|^2 =
// sum d^2 - |sum_atoms d|^2 / N.  One wave per band; lanes sum the tiles of an
// interval in a fixed order.
__global__ void __launch_bounds__(64) k_readout(BatchDev bd)
{
    ItemLoop loop(bd, KIND_BAND, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        const int M = st->M;
        const int lane = threadIdx.x;
        if (lane == 0) {
            double hmax = b.scal[st->slot[0]].H;
            for (int k = 0; k < M; ++k) {
                const double h = b.scal[st->slot[k]].H;
                st->Hlog[k] = h;
                hmax = fmax(hmax, h);
            }
            st->barrier = hmax - st->Hlog[0];
            st->xi[0] = 0.0;
        }
        double acc = 0.0;
        for (int k = 0; k < M - 1; ++k) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            const double* part = b.dotpart + size_t(k) * b.ntR * 4;
            for (int t = lane; t < b.ntR; t += 64)
                for (int q = 0; q < 4; ++q) v[q] += part[size_t(t) * 4 + q];
            for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
            const double tr = (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / double(b.N);
            acc += sqrt(fmax(v[0] - tr, 0.0));
            if (lane == 0) st->xi[k + 1] = acc;
        }
        if (lane == 0)
            for (int k = 1; k < M; ++k) st->xi[k] = acc > 0.0 ? st->xi[k] / acc : 0.0;
    }
}

// Step-end adaptive-image check (kernels act only on bands whose step set refine_due),
// or a forced decision (mode 1) after launch_plan(..., ignore_stop = 1).
void launch_refine(const Launch& L, int forced, hipStream_t s)
{
    const int mode = forced ? 1 : 0;
    k_refine_dist<<<L.g[KIND_IVAL], CFNEB_TILE, 0, s>>>(L.bd, mode);
    k_refine_decide<<<L.g[KIND_BAND], 1024, 0, s>>>(L.bd, mode);
    k_refine_apply<<<L.g[KIND_SLOTROW], CFNEB_TILE, 0, s>>>(L.bd, mode);
}

// Readout after launch_plan(..., ignore_stop = 1).
void launch_readout(const Launch& L, hipStream_t s)
{
    k_readout_dist<<<L.g[KIND_IVAL], CFNEB_TILE, 0, s>>>(L.bd);
    k_readout<<<L.g[KIND_BAND], 64, 0, s>>>(L.bd);
}

}  // namespace cfneb
