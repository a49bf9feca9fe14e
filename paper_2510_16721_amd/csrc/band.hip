// Band-wide NEB projection (Eq. (1)), climbing image, springs and FIRE.
//
// Every moving image k's NEB force is
//     F_NEB = Fg + c+ tau+ + c- tau-,   tau+ = X_{k+1} - X_k,  tau- = X_k - X_{k-1}
// because the improved tangent is a combination a tau+ + b tau-: with
// t = (a tau+ + b tau-) / |.|, the projection Fg - (Fg.t) t + k (|tau+| - |tau-|) t
// (or Fg - 2 (Fg.t) t for the climbing image) only needs ten dot products per image.
// A rigid translation of the atoms costs no energy in a periodic cell, so tau+, tau-
// and Fg are taken with their atom-row means removed; the centred dots follow from the
// raw ones and the atom-row sums of tau+, tau-, Fg and v (twelve more sums), e.g.
// |tau+ - m+|^2 = |tau+|^2 - N |m+|^2 over the N atom rows.
// Pass 1 (k_band_dots) streams X, Fg and v once to get them; one block per band then
// forms the coefficients and the band-global FIRE quantities P = F.v, |F|, |v| from
// them; pass 2 (k_band_update) forms F_NEB row by row, the new velocity and the row
// maxima; pass 3 (k_band_move) moves X once fmax and the step clamp are known.
//
// Generalized forces are formed on the fly: atom rows F D^T from the stored
// Cartesian forces, cell rows from the per-image lattice force (Eq. (17)).
#include "cfneb_dev.h"

namespace cfneb {

template <typename T>
__device__ inline void gen_force_row(const BandDev& b, int slot, int r, double* f)
{
    if (r < b.N) {
        const T* F = reinterpret_cast<const T*>(b.F) + size_t(slot) * slot_rows(b);
        const double fx = double(F[r]), fy = double(F[b.ld + r]), fz = double(F[2 * size_t(b.ld) + r]);
        const double* D = b.geom[slot].D;
        for (int c = 0; c < 3; ++c) f[c] = fx * D[3 * c] + fy * D[3 * c + 1] + fz * D[3 * c + 2];
    } else {
        const double* G = b.scal[slot].Fcell + 3 * (r - b.N);
        f[0] = G[0];
        f[1] = G[1];
        f[2] = G[2];
    }
}

// Start of a cfneb_step / cfneb_batch_step call for every band in the table.
__global__ void k_begin_call(BatchDev bd, double f_tol, int only)
{
    const int t = threadIdx.x;
    if (t >= bd.cap || !bd.live[t] || (only >= 0 && t != only)) return;
    BandState* st = bd.bands[t].st;
    st->f_tol = f_tol;
    st->steps_call = 0;
    st->done = 0;
    st->err = 0;
}

// 10 dots per moving image: |t+|^2 |t-|^2 t+.t- F.t+ F.t- F.F F.v v.v v.t+ v.t-,
// then the atom-row sums of t+ (3), t- (3), F (3) and v (3).
__device__ inline void dots_row(double* a, const double (&x0)[3], const double (&xm)[3], const double (&xp)[3],
                                const double (&v)[3], const double (&f)[3], bool atom)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double tp = xp[c] - x0[c], tm = x0[c] - xm[c];
        a[0] += tp * tp;
        a[1] += tm * tm;
        a[2] += tp * tm;
        a[3] += f[c] * tp;
        a[4] += f[c] * tm;
        a[5] += f[c] * f[c];
        a[6] += f[c] * v[c];
        a[7] += v[c] * v[c];
        a[8] += v[c] * tp;
        a[9] += v[c] * tm;
        if (atom) {
            a[10 + c] += tp;
            a[13 + c] += tm;
            a[16 + c] += f[c];
            a[19 + c] += v[c];
        }
    }
}

// Generalized force of an atom row from its Cartesian force: F D^T.
template <typename T, typename DP>
__device__ inline void atom_gen_force(const DP D, const T (&fr)[3], double (&f)[3])
{
    const double fx = double(fr[0]), fy = double(fr[1]), fz = double(fr[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = fx * D[3 * c] + fy * D[3 * c + 1] + fz * D[3 * c + 2];
}

// An item is 1024 rows, four per thread (rows tile*1024 + q*256 + thread, so every
// load is coalesced).  A tile of atom rows only issues all loads of its four rows
// before any arithmetic; the image's last tile (cell rows, ragged end) first reduces
// the image's energy and virial, then goes row by row.
template <typename T>
__device__ void dots_item(const BandDev& b, const BandState* st, int k, int tile, double* lds)
{
    constexpr int Q = CFNEB_TILE4 / CFNEB_TILE;
    const int s0 = st->slot[k], sm = st->slot[k - 1], sp = st->slot[k + 1];
    double a[CFNEB_NDOT];
#pragma unroll
    for (int q = 0; q < CFNEB_NDOT; ++q) a[q] = 0.0;
    const gmem<const double>* __restrict__ X0 = gp<const double>(Xs(b, s0));
    const gmem<const double>* __restrict__ Xm = gp<const double>(Xs(b, sm));
    const gmem<const double>* __restrict__ Xp = gp<const double>(Xs(b, sp));
    const gmem<const double>* __restrict__ V = gp<const double>(Vs(b, st->vcur, s0));
    const gmem<const T>* __restrict__ F = gp<const T>(reinterpret_cast<const T*>(b.F) + size_t(s0) * slot_rows(b));
    const size_t ld = b.ld;
    const int r0 = tile * CFNEB_TILE4 + int(threadIdx.x);
    if ((tile + 1) * CFNEB_TILE4 <= b.N) {  // uniform over the block
        double x0[Q][3], xm[Q][3], xp[Q][3], v[Q][3];
        T fr[Q][3];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + (r0 + q * CFNEB_TILE);
                x0[q][c] = X0[o];
                xm[q][c] = Xm[o];
                xp[q][c] = Xp[o];
                v[q][c] = V[o];
                fr[q][c] = F[o];
            }
        const gmem<const double>* D = gp<const double>(b.geom[s0].D);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double f[3];
            atom_gen_force<T>(D, fr[q], f);
            dots_row(a, x0[q], xm[q], xp[q], v[q], f, true);
        }
    } else {
        // the image's last tile holds its cell rows, whose force needs the image's
        // energy and virial: this block reduces them first
        image_reduce_item(b, const_cast<BandState*>(st), s0, lds);
        __syncthreads();
        for (int q = 0; q < Q; ++q) {
            const int r = r0 + q * CFNEB_TILE;
            if (r >= b.N + 3) break;
            double x0[3], xm[3], xp[3], v[3], f[3];
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + r;
                x0[c] = X0[o];
                xm[c] = Xm[o];
                xp[c] = Xp[o];
                v[c] = V[o];
            }
            gen_force_row<T>(b, s0, r, f);
            dots_row(a, x0, xm, xp, v, f, r < b.N);
        }
    }
    // each wave stores its own partials (no block barrier): [image][dot][tile][wave],
    // so the reduction reads consecutive partials
    const double s = wave_sum_t<CFNEB_NDOT>(a);
    constexpr int LOGP = wave_sum_logp<CFNEB_NDOT>();
    const int lane = int(threadIdx.x) & 63, idx = lane >> (6 - LOGP);
    if ((lane & ((64 >> LOGP) - 1)) == 0 && idx < CFNEB_NDOT) {
        const int parts = b.ntR4 * CFNEB_WAVES;
        b.dotpart[(size_t(k) * CFNEB_NDOT + idx) * parts + tile * CFNEB_WAVES + (int(threadIdx.x) >> 6)] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_band_dots(BatchDev bd, unsigned vmask)
{
    __shared__ double lds[(CFNEB_TILE / 64) * CFNEB_NDOT];
    ItemLoop loop(bd, KIND_ROW4, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        if (!((vmask >> band_variant(b)) & 1u) || band_stopped(b.st)) continue;  // uniform
        dots_item<T>(b, b.st, it.image, it.tile, lds);
    }
}

// One block per moving image, one wave per dot (waves take dots w and w + 16): each
// lane sums every 64th tile partial, then the wave sums its lanes, in a fixed order.
__global__ void __launch_bounds__(1024) k_band_dots_reduce(BatchDev bd)
{
    ItemLoopRO loop(bd, KIND_IMAGE, 0);
    Item it;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        if (band_stopped(cp(b.st))) continue;  // uniform over the block
        const int k = it.image;
        const int parts = b.ntR4 * CFNEB_WAVES;
        const gmem<const double>* part = gp<const double>(b.dotpart + size_t(k) * CFNEB_NDOT * parts);
        // a wave sums dots w and w + 16 together, each lane its every 64th partial in
        // order; the unrolled loop keeps several partials' loads in flight
        static_assert(CFNEB_NDOT <= 32, "two dots per wave");
        const int q1 = w + 16;
        const bool two = q1 < CFNEB_NDOT;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 4
        for (int t = lane; t < parts; t += 64) {
            a0 += part[size_t(w) * parts + t];
            if (two) a1 += part[size_t(q1) * parts + t];
        }
        a0 = wave_sum(a0);
        if (lane == 0) b.dotred[size_t(k) * CFNEB_NDOT + w] = a0;
        if (two) {
            a1 = wave_sum(a1);
            if (lane == 0) b.dotred[size_t(k) * CFNEB_NDOT + q1] = a1;
        }
    }
}

__device__ inline void tangent_coeffs(double Hm, double H0, double Hp, double& a, double& c)
{
    if (Hp > H0 && H0 > Hm) {
        a = 1.0;
        c = 0.0;
    } else if (Hp < H0 && H0 < Hm) {
        a = 0.0;
        c = 1.0;
    } else {
        const double up = fabs(Hp - H0), dn = fabs(Hm - H0);
        const double big = fmax(up, dn), small = fmin(up, dn);
        if (Hp > Hm) {
            a = big;
            c = small;
        } else {
            a = small;
            c = big;
        }
    }
}

// One block per band: reduce the dot partials, choose tangents and the climbing
// image, form the projection coefficients and the FIRE proposal.
__device__ void scalars_item(const BandDev& b, BandState* st)
{
    __shared__ double dots[CFNEB_MAX_IMAGES][CFNEB_NDOT];
    __shared__ double H[CFNEB_MAX_IMAGES];
    __shared__ double contrib[3][CFNEB_MAX_IMAGES];
    __shared__ int ci_s;
    const int M = st->M;
    for (int e = threadIdx.x; e < (M - 2) * CFNEB_NDOT; e += int(blockDim.x))
        dots[1 + e / CFNEB_NDOT][e % CFNEB_NDOT] = b.dotred[CFNEB_NDOT + size_t(e)];
    // image enthalpies, loaded in parallel
    const int t = threadIdx.x;
    if (t < M) H[t] = b.scal[st->slot[t]].H;
    __syncthreads();
    if (t == 0) {
        int ci = -1;
        if (b.climb_after >= 0 && st->step >= b.climb_after) {
            for (int k = 1; k <= M - 2; ++k)
                if (ci < 0 || H[k] > H[ci]) ci = k;
        }
        ci_s = ci;
        st->ci = ci;
    }
    __syncthreads();
    // one thread per moving image: tangent, projection coefficients, FIRE terms
    if (t >= 1 && t <= M - 2) {
        const int k = t, ci = ci_s;
        const double* raw = dots[k];
        // atom-row means of tau+, tau-, Fg and v, then the dots of the centred vectors
        const double N = double(b.N);
        double m[12];
        for (int q = 0; q < 12; ++q) m[q] = raw[10 + q] / N;
        const double *mp = m, *mm = m + 3, *mf = m + 6, *mv = m + 9;
        auto mdot = [&](const double* x, const double* y) {
            return N * ((x[0] * y[0] + x[1] * y[1]) + x[2] * y[2]);
        };
        double d[10];
        d[0] = raw[0] - mdot(mp, mp);
        d[1] = raw[1] - mdot(mm, mm);
        d[2] = raw[2] - mdot(mp, mm);
        d[3] = raw[3] - mdot(mf, mp);
        d[4] = raw[4] - mdot(mf, mm);
        d[5] = raw[5] - mdot(mf, mf);
        d[6] = raw[6] - mdot(mf, mv);
        d[7] = raw[7];
        d[8] = raw[8] - mdot(mv, mp);
        d[9] = raw[9] - mdot(mv, mm);
        for (int q = 0; q < 9; ++q) st->tmean[k][q] = m[q];
        double a, c;
        tangent_coeffs(H[k - 1], H[k], H[k + 1], a, c);
        const double tt = a * a * d[0] + 2.0 * a * c * d[2] + c * c * d[1];
        const double nt = sqrt(fmax(tt, 0.0));
        double cp = 0.0, cm = 0.0;
        if (nt > 0.0 && !b.relax) {
            const double ft = (a * d[3] + c * d[4]) / nt;
            const double s = (k == ci) ? -2.0 * ft : b.k_spring * (sqrt(d[0]) - sqrt(d[1])) - ft;
            cp = s * a / nt;
            cm = s * c / nt;
        }
        st->cplus[k] = cp;
        st->cminus[k] = cm;
        contrib[0][k] = d[6] + cp * d[8] + cm * d[9];
        contrib[1][k] = d[5] + cp * cp * d[0] + cm * cm * d[1] + 2.0 * cp * d[3] + 2.0 * cm * d[4] +
                        2.0 * cp * cm * d[2];
        contrib[2][k] = d[7];
    }
    __syncthreads();
    if (t == 0) {
        double Pw = 0.0, FF = 0.0, VV = 0.0;
        for (int k = 1; k <= M - 2; ++k) {
            Pw += contrib[0][k];
            FF += contrib[1][k];
            VV += contrib[2][k];
        }
        // FIRE (Bitzek et al. 2006) proposal; committed only if the band moves.
        double cv = 1.0, cf = 0.0, dt = st->dt, alpha = st->alpha;
        int np = st->n_pos;
        if (!st->fresh) {
            if (Pw > 0.0) {
                const double nf = sqrt(fmax(FF, 0.0)), nv = sqrt(fmax(VV, 0.0));
                if (nf > 0.0) {
                    cv = 1.0 - alpha;
                    cf = alpha * nv / nf;
                }
                if (np > b.nmin) {
                    dt = fmin(dt * b.finc, b.dtmax);
                    alpha *= b.fa;
                }
                np += 1;
            } else {
                cv = 0.0;
                cf = 0.0;
                alpha = b.astart;
                dt *= b.fdec;
                np = 0;
            }
        }
        st->cv = cv;
        st->cf = cf;
        st->dt_new = dt;
        st->alpha_new = alpha;
        st->n_pos_new = np;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_band_scalars(BatchDev bd)
{
    ItemLoop loop(bd, KIND_BAND, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        if (band_stopped(b.st)) continue;  // uniform over the block
        scalars_item(b, b.st);
    }
}

// One row of F_NEB = Fg - mean + cp (tau+ - mean) + cm (tau- - mean) (means for atom
// rows only), v' = (cv v + cf F_NEB) + dt' F_NEB; returns |F_NEB|^2 and |dt' v'|^2.
struct UpdateCoef {
    double cp, cm, cv, cf, dt;
    double mean[9];
};
__device__ inline void update_row(const UpdateCoef& u, const double (&x0)[3], const double (&xm)[3],
                                  const double (&xp)[3], const double (&v)[3], const double (&f)[3], bool atom,
                                  double (&fn)[3], double (&vn)[3], double& f2, double& v2)
{
    f2 = 0.0;
    v2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double tp = xp[c] - x0[c], tm = x0[c] - xm[c], fc = f[c];
        if (atom) {
            tp -= u.mean[c];
            tm -= u.mean[3 + c];
            fc -= u.mean[6 + c];
        }
        fn[c] = fc + u.cp * tp + u.cm * tm;
        vn[c] = (u.cv * v[c] + u.cf * fn[c]) + u.dt * fn[c];
        f2 += fn[c] * fn[c];
        const double dr = u.dt * vn[c];
        v2 += dr * dr;
    }
}

// F_NEB per row, the new velocity into the other buffer, and the row maxima of
// |F_NEB| and |dt' v'|; 1024 rows per item, four per thread, loads of atom-row tiles
// all issued before the first store.
template <typename T>
__device__ void update_item(const BandDev& b, const cmem<BandState>* st, int k, int tile, double* lds)
{
    constexpr int Q = CFNEB_TILE4 / CFNEB_TILE;
    const int s0 = st->slot[k], sm = st->slot[k - 1], sp = st->slot[k + 1];
    double m[3] = {0.0, 0.0, 0.0};  // max |F_NEB row|^2, max |dr row|^2, non-finite flag
    UpdateCoef u;
    u.cp = st->cplus[k];
    u.cm = st->cminus[k];
    u.cv = st->cv;
    u.cf = st->cf;
    u.dt = st->dt_new;
#pragma unroll
    for (int q = 0; q < 9; ++q) u.mean[q] = st->tmean[k][q];
    const gmem<const double>* __restrict__ X0 = gp<const double>(Xs(b, s0));
    const gmem<const double>* __restrict__ Xm = gp<const double>(Xs(b, sm));
    const gmem<const double>* __restrict__ Xp = gp<const double>(Xs(b, sp));
    const gmem<const double>* __restrict__ V = gp<const double>(Vs(b, st->vcur, s0));
    const gmem<const T>* __restrict__ F = gp<const T>(reinterpret_cast<const T*>(b.F) + size_t(s0) * slot_rows(b));
    gmem<double>* __restrict__ Vn = gp(Vs(b, st->vcur ^ 1, s0));
    gmem<double>* __restrict__ FN = gp(b.FN + size_t(s0) * slot_rows(b));
    const int rec = st->record_fneb;
    const size_t ld = b.ld;
    const int r0 = tile * CFNEB_TILE4 + int(threadIdx.x);
    if ((tile + 1) * CFNEB_TILE4 <= b.N) {  // uniform over the block
        double x0[Q][3], xm[Q][3], xp[Q][3], v[Q][3];
        T fr[Q][3];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + (r0 + q * CFNEB_TILE);
                x0[q][c] = X0[o];
                xm[q][c] = Xm[o];
                xp[q][c] = Xp[o];
                v[q][c] = V[o];
                fr[q][c] = F[o];
            }
        const gmem<const double>* D = gp<const double>(b.geom[s0].D);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double f[3], fn[3], vn[3], f2, v2;
            atom_gen_force<T>(D, fr[q], f);
            update_row(u, x0[q], xm[q], xp[q], v[q], f, true, fn, vn, f2, v2);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + (r0 + q * CFNEB_TILE);
                Vn[o] = vn[c];
                if (rec) FN[o] = fn[c];
            }
            m[0] = fmax(m[0], f2);
            m[1] = fmax(m[1], v2);
            if (!(isfinite(f2) && isfinite(v2))) m[2] = 1.0;
        }
    } else {
        for (int q = 0; q < Q; ++q) {
            const int r = r0 + q * CFNEB_TILE;
            if (r >= b.N + 3) break;
            double x0[3], xm[3], xp[3], v[3], f[3], fn[3], vn[3], f2, v2;
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + r;
                x0[c] = X0[o];
                xm[c] = Xm[o];
                xp[c] = Xp[o];
                v[c] = V[o];
            }
            gen_force_row<T>(b, s0, r, f);
            update_row(u, x0, xm, xp, v, f, r < b.N, fn, vn, f2, v2);
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * ld + r;
                Vn[o] = vn[c];
                if (rec) FN[o] = fn[c];
            }
            m[0] = fmax(m[0], f2);
            m[1] = fmax(m[1], v2);
            if (!(isfinite(f2) && isfinite(v2))) m[2] = 1.0;
        }
    }
    block_max<3>(m, lds);
    if (threadIdx.x == 0) {
        double* out = b.maxpart + size_t(k) * 3 * b.ntR4 + tile;  // [image][q][tile]
        out[0] = m[0];
        out[b.ntR4] = m[1];
        out[2 * size_t(b.ntR4)] = m[2];
    }
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_band_update(BatchDev bd, unsigned vmask)
{
    __shared__ double lds[4 * 3];
    ItemLoopRO loop(bd, KIND_ROW4, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        if (!((vmask >> band_variant(b)) & 1u) || band_stopped(cp(b.st))) continue;  // uniform
        update_item<T>(b, cp(b.st), it.image, it.tile, lds);
    }
}

// fmax, convergence, step clamp; commit the FIRE proposal when the band moves (the
// move itself, X += scale dt v', is left pending for the next pass over X).
__device__ void finalize_item(const BandDev& b, BandState* st, double* lds)
{
    const int M = st->M;
    double m[3] = {0.0, 0.0, 0.0};
    const int total = (M - 2) * b.ntR4;
    for (int t = threadIdx.x; t < total; t += int(blockDim.x)) {
        const int k = 1 + t / b.ntR4, tile = t % b.ntR4;
        const double* p = b.maxpart + size_t(k) * 3 * b.ntR4 + tile;
        m[0] = fmax(m[0], p[0]);
        m[1] = fmax(m[1], p[b.ntR4]);
        m[2] = fmax(m[2], p[2 * size_t(b.ntR4)]);
    }
    block_max<3>(m, lds);
    if (threadIdx.x != 0) return;
    const double fmaxv = sqrt(m[0]);
    st->fmax = fmaxv;
    st->move = 0;
    st->refine_due = 0;
    if (m[2] != 0.0 || !isfinite(fmaxv) || !isfinite(m[1])) {
        set_error(st, CFNEB_ENONFINITE);
        return;
    }
    if (fmaxv < st->f_tol) {
        st->done = 1;
        return;
    }
    const double maxdr = sqrt(m[1]);
    st->scale = (maxdr > b.maxstep) ? b.maxstep / maxdr : 1.0;
    st->move = 1;
    st->dt = st->dt_new;
    st->alpha = st->alpha_new;
    st->n_pos = st->n_pos_new;
    st->fresh = 0;
    st->vcur ^= 1;
    st->step += 1;
    st->steps_call += 1;
    st->image_steps += M - 2;
    st->refine_due = (b.refine_every > 0 && st->step % b.refine_every == 0) ? 1 : 0;
}

__device__ inline void note_refine(const BatchDev& bd, const BandState* st)
{
    if (st->refine_due) *refine_flag(bd) = 1;
}

__global__ void __launch_bounds__(1024) k_band_finalize(BatchDev bd)
{
    __shared__ double lds[16 * 3];
    ItemLoop loop(bd, KIND_BAND, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        BandState* st = b.st;
        if (band_stopped(st)) {  // uniform over the block
            if (threadIdx.x == 0) {
                st->move = 0;
                st->refine_due = 0;  // finalize sets it afresh on every step that runs
            }
            continue;
        }
        finalize_item(b, st, lds);
        __syncthreads();
        if (threadIdx.x == 0) note_refine(bd, st);
    }
}

__global__ void __launch_bounds__(CFNEB_TILE) k_band_move(BatchDev bd)
{
    ItemLoop loop(bd, KIND_ROW, 0);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        if (!st->move || st->err != 0) continue;
        const int r = it.tile * CFNEB_TILE + threadIdx.x;
        if (r >= b.N + 3) continue;
        const int s0 = st->slot[it.image];
        gmem<double>* __restrict__ X = gp(Xs(b, s0));
        const gmem<const double>* __restrict__ V = gp<const double>(Vs(b, st->vcur, s0));
        const double sc = st->scale, dt = st->dt;
        for (int c = 0; c < 3; ++c) {
            const size_t o = size_t(c) * b.ld + r;
            X[o] += sc * (dt * V[o]);
        }
    }
}

// ---------------------------------------------------------------- energy profile
// Readout of the enthalpy along the path, the form in which the transitions of
// Sec. III are reported.  After an evaluation of every image, each image gets 14
// sums over its rows: |t+|^2, |t-|^2, t+.t-, Fg.t+, Fg.t- and the atom-row sums of
// t+, t- and Fg (t+ = X_{k+1} - X_k, absent at the last image; t- = X_k - X_{k-1},
// absent at the first).  From their translation-free forms one block per band takes
// the arc length of each interval and the slope dH/ds = -Fg.tau/|tau| (improved
// tangent for the moving images, the one-sided difference at the ends), then
// samples the cubic Hermite interpolant of H over the arc length and finds its
// maximum from the nodes and the critical points inside each interval.
template <typename T>
__device__ void profile_dots_item(const BandDev& b, const BandState* st, int k, int tile, double* lds)
{
    const int M = st->M;
    const int s0 = st->slot[k];
    const int sp = k + 1 < M ? st->slot[k + 1] : s0;
    const int sm = k > 0 ? st->slot[k - 1] : s0;
    const gmem<const double>* __restrict__ X0 = gp<const double>(Xs(b, s0));
    const gmem<const double>* __restrict__ Xp = gp<const double>(Xs(b, sp));
    const gmem<const double>* __restrict__ Xm = gp<const double>(Xs(b, sm));
    double a[CFNEB_NPROF];
#pragma unroll
    for (int q = 0; q < CFNEB_NPROF; ++q) a[q] = 0.0;
    for (int q = 0; q < CFNEB_TILE4 / CFNEB_TILE; ++q) {
        const int r = tile * CFNEB_TILE4 + q * CFNEB_TILE + int(threadIdx.x);
        if (r >= b.N + 3) break;
        double f[3];
        gen_force_row<T>(b, s0, r, f);
        const bool atom = r < b.N;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t o = size_t(c) * b.ld + r;
            const double x0 = X0[o];
            const double tp = Xp[o] - x0, tm = x0 - Xm[o];
            a[0] += tp * tp;
            a[1] += tm * tm;
            a[2] += tp * tm;
            a[3] += f[c] * tp;
            a[4] += f[c] * tm;
            if (atom) {
                a[5 + c] += tp;
                a[8 + c] += tm;
                a[11 + c] += f[c];
            }
        }
    }
    block_sum_t<CFNEB_NPROF>(a, lds);
    if (threadIdx.x == 0) {
        double* out = b.dotpart + size_t(k) * CFNEB_NDOT * b.ntR4 + tile;
        for (int q = 0; q < CFNEB_NPROF; ++q) out[size_t(q) * b.ntR4] = a[q];
    }
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_profile_dots(BatchDev bd, unsigned vmask)
{
    __shared__ double lds[(CFNEB_TILE / 64) * CFNEB_NPROF];
    ItemLoop loop(bd, KIND_ROW4, 1);
    Item it;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        if (!((vmask >> band_variant(b)) & 1u)) continue;  // uniform
        profile_dots_item<T>(b, b.st, it.image, it.tile, lds);
    }
}

// One block per image, one wave per sum.
__global__ void __launch_bounds__(1024) k_profile_reduce(BatchDev bd)
{
    ItemLoop loop(bd, KIND_IMAGE, 1);
    Item it;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const int k = it.image;
        const double* part = b.dotpart + size_t(k) * CFNEB_NDOT * b.ntR4;
        if (w < CFNEB_NPROF) {
            double a = 0.0;
            for (int t = lane; t < b.ntR4; t += 64) a += part[size_t(w) * b.ntR4 + t];
            a = wave_sum(a);
            if (lane == 0) b.dotred[size_t(k) * CFNEB_NDOT + w] = a;
        }
    }
}

// Cubic Hermite interpolant on one interval of length d at t in [0, 1].
__device__ inline double hermite_at(double H0, double H1, double m0, double m1, double d, double t)
{
    const double u = 1.0 - t;
    // h00 = (1 + 2t) u^2, h10 = t u^2, h01 = t^2 (3 - 2t), h11 = -t^2 u
    return (1.0 + 2.0 * t) * u * u * H0 + t * u * u * (d * m0) + t * t * (3.0 - 2.0 * t) * H1 -
           t * t * u * (d * m1);
}

__global__ void __launch_bounds__(CFNEB_TILE) k_profile(BatchDev bd, int n_samples)
{
    __shared__ double s[CFNEB_MAX_IMAGES], H[CFNEB_MAX_IMAGES], m[CFNEB_MAX_IMAGES], len[CFNEB_MAX_IMAGES];
    __shared__ double bv[CFNEB_MAX_IMAGES], ba[CFNEB_MAX_IMAGES];
    ItemLoop loop(bd, KIND_BAND, 0);
    Item it;
    const int t = threadIdx.x;
    while (loop.next(it)) {
        const BandDev& b = bd.bands[it.band];
        const BandState* st = b.st;
        const int M = st->M;
        if (t < M) H[t] = b.scal[st->slot[t]].H;
        __syncthreads();
        if (t < M) {
            const double* raw = b.dotred + size_t(t) * CFNEB_NDOT;
            const double N = double(b.N);
            double mp[3], mm[3], mf[3];
            for (int c = 0; c < 3; ++c) {
                mp[c] = raw[5 + c] / N;
                mm[c] = raw[8 + c] / N;
                mf[c] = raw[11 + c] / N;
            }
            auto nd = [&](const double* x, const double* y) {
                return N * ((x[0] * y[0] + x[1] * y[1]) + x[2] * y[2]);
            };
            const double pp = raw[0] - nd(mp, mp), qq = raw[1] - nd(mm, mm), pq = raw[2] - nd(mp, mm);
            const double fp = raw[3] - nd(mf, mp), fq = raw[4] - nd(mf, mm);
            double a = 1.0, c = 0.0;
            if (t == M - 1) {
                a = 0.0;
                c = 1.0;
            } else if (t > 0) {
                tangent_coeffs(H[t - 1], H[t], H[t + 1], a, c);
            }
            const double nt = sqrt(fmax(a * a * pp + 2.0 * a * c * pq + c * c * qq, 0.0));
            m[t] = nt > 0.0 ? -(a * fp + c * fq) / nt : 0.0;
            len[t] = sqrt(fmax(pp, 0.0));
        }
        __syncthreads();
        if (t == 0) {
            s[0] = 0.0;
            for (int k = 0; k + 1 < M; ++k) s[k + 1] = s[k] + len[k];
        }
        __syncthreads();
        // each interval: the largest of its right node and its interior critical points
        if (t + 1 < M) {
            const double d = s[t + 1] - s[t];
            double best = H[t + 1], at = s[t + 1];
            if (d > 0.0) {
                const double g0 = d * m[t], g1 = d * m[t + 1];
                // derivative in t of the interval's cubic: A t^2 + B t + C
                const double A = 6.0 * (H[t] - H[t + 1]) + 3.0 * (g0 + g1);
                const double B = 6.0 * (H[t + 1] - H[t]) - 4.0 * g0 - 2.0 * g1;
                const double C = g0;
                double r[2];
                int nr = 0;
                if (A == 0.0) {
                    if (B != 0.0) r[nr++] = -C / B;
                } else {
                    const double disc = B * B - 4.0 * A * C;
                    if (disc >= 0.0) {
                        const double q = -0.5 * (B + copysign(sqrt(disc), B));
                        r[nr++] = q / A;
                        if (q != 0.0) r[nr++] = C / q;
                    }
                }
                for (int j = 0; j < nr; ++j)
                    if (r[j] > 0.0 && r[j] < 1.0) {
                        const double v = hermite_at(H[t], H[t + 1], m[t], m[t + 1], d, r[j]);
                        if (v > best) {
                            best = v;
                            at = s[t] + r[j] * d;
                        }
                    }
            }
            bv[t] = best;
            ba[t] = at;
        }
        __syncthreads();
        double* out = b.staging;
        const double S = s[M - 1];
        if (t == 0) {
            double best = H[0], at = 0.0;
            for (int k = 0; k + 1 < M; ++k)
                if (bv[k] > best) {
                    best = bv[k];
                    at = ba[k];
                }
            out[CFNEB_PROF_OUT] = best - H[0];
            out[CFNEB_PROF_OUT + 1] = S > 0.0 ? at / S : 0.0;
            out[CFNEB_PROF_OUT + 2] = best;
        }
        if (t < M) {
            out[CFNEB_PROF_S + t] = s[t];
            out[CFNEB_PROF_H + t] = H[t];
            out[CFNEB_PROF_SLOPE + t] = m[t];
        }
        for (int j = t; j < n_samples; j += int(blockDim.x)) {
            const double x = double(j) / double(n_samples - 1) * S;
            int k = 0;  // the last interval starting at or before x
            for (int q = 1; q + 1 < M; ++q)
                if (s[q] <= x) k = q;
            const double d = s[k + 1] - s[k];
            const double u = d > 0.0 ? fmin(fmax((x - s[k]) / d, 0.0), 1.0) : 0.0;
            out[CFNEB_PROF_SAMP + j] = hermite_at(H[k], H[k + 1], m[k], m[k + 1], d, u);
        }
        __syncthreads();
    }
}

static unsigned f32_mask(unsigned variants)
{
    return variants & ((1u << VARIANT_LJ32) | (1u << VARIANT_TS32));
}
static unsigned f64_mask(unsigned variants)
{
    return variants & ((1u << VARIANT_LJ64) | (1u << VARIANT_TS64));
}

void launch_begin_call(const Launch& L, double f_tol, int only, hipStream_t s)
{
    k_begin_call<<<1, CFNEB_MAX_BANDS, 0, s>>>(L.bd, f_tol, only);
}

void launch_dots(const Launch& L, hipStream_t s)
{
    const unsigned g = L.g[KIND_ROW4];
    if (f32_mask(L.variants)) k_band_dots<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, f32_mask(L.variants));
    if (f64_mask(L.variants)) k_band_dots<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, f64_mask(L.variants));
    k_band_dots_reduce<<<L.g[KIND_IMAGE], 1024, 0, s>>>(L.bd);
}

// Energy profile after an evaluation of every image (launch_evaluate(L, 1, s)).
void launch_profile(const Launch& L, int n_samples, hipStream_t s)
{
    const unsigned g = L.g[KIND_ROW4];
    if (f32_mask(L.variants)) k_profile_dots<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, f32_mask(L.variants));
    if (f64_mask(L.variants)) k_profile_dots<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, f64_mask(L.variants));
    k_profile_reduce<<<L.g[KIND_IMAGE], 1024, 0, s>>>(L.bd);
    k_profile<<<L.g[KIND_BAND], CFNEB_TILE, 0, s>>>(L.bd, n_samples);
}

void launch_scalars(const Launch& L, hipStream_t s) { k_band_scalars<<<L.g[KIND_BAND], 1024, 0, s>>>(L.bd); }

void launch_update(const Launch& L, hipStream_t s)
{
    const unsigned g = L.g[KIND_ROW4];
    if (f32_mask(L.variants)) k_band_update<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, f32_mask(L.variants));
    if (f64_mask(L.variants)) k_band_update<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, f64_mask(L.variants));
}

void launch_finalize(const Launch& L, hipStream_t s) { k_band_finalize<<<L.g[KIND_BAND], 1024, 0, s>>>(L.bd); }

// A step's move is applied by the next step's geometry (cell rows) and skin check
// (atom rows), which read X anyway; this pair applies a pending move on its own, at
// the end of a step call and before a refinement, and then clears the flag.
__global__ void k_move_clear(BatchDev bd)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < bd.cap && bd.live[t]) bd.bands[t].st->move = 0;
}

void launch_flush_move(const Launch& L, hipStream_t s)
{
    k_band_move<<<L.g[KIND_ROW], CFNEB_TILE, 0, s>>>(L.bd);
    k_move_clear<<<(L.bd.cap + 63) / 64, 64, 0, s>>>(L.bd);
}

}  // namespace cfneb
