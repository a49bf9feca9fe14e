// Tersoff bond-order carbon: energies, dU_i/dr^ij per bond, force gather (Sec. II.B).
//
//   U_i = 1/2 sum_j fc(r_ij) [A exp(-l1 r_ij) - b_ij B exp(-l2 r_ij)],
//   b_ij = (1 + beta^n zeta_ij^n)^(-1/2n),  zeta_ij = sum_{k != j} fc(r_ik) g(cos theta_ijk),
//   fc = 1 below R, 1/2 + 1/2 cos(pi (r - R)/(S - R)) between R and S, 0 beyond.
// U_i depends only on i's bond vectors, so one thread per atom finds its neighbours
// among its candidates (exact test), keeps the bond vectors in registers and forms
// every P_ij = dU_i/dr^ij, stored in the pair's candidate slot (zero for candidates
// that are not bonds); a second kernel gathers F_i = sum_j (P_ij - P_ji) over the
// candidates, P_ji read from the reverse candidate (i, -n) of j's list.  The exact
// inclusion test is symmetric to the last bit (the separation of (j, i, -n) is the
// negated separation of (i, j, n) in every rounding), so a pair and its reverse are
// bonds together.  The reverse slots are found once per candidate build.  No
// atomics: the result is deterministic.
//
// g is evaluated as 1 + (c^2/d^2) x / (d^2 + x), x = (h - cos)^2: the textbook form
// 1 + c^2/d^2 - c^2/(d^2 + x) cancels two numbers near 7.7e7 and loses about four
// digits in FP32.
#include <type_traits>

#include "cfneb_dev.h"

namespace cfneb {

// Quotients of the FP32 path use the hardware reciprocal (about 1 ulp): every
// quotient here feeds a cosine or g(cos), whose relative errors reach the bond
// order damped by |d ln b / d ln zeta| < 0.1.  The FP64 path divides exactly.
__device__ inline float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double qdiv(double a, double b) { return a / b; }

// FP64 natural logarithm and exponential for the FP32 bond order and the bond
// energies.  FP64 vector operations run at the FP32 rate on this GPU, so two short
// polynomial evaluations cost a fraction of two accurately rounded FP32 powers, and
// their results are far more accurate than FP32 before the final rounding.
// ln: u = m 2^e with m in [1/sqrt 2, sqrt 2); ln m = 2 atanh(s), s = (m - 1)/(m + 1),
// |s| <= 0.1716, by its series through s^11 (absolute error below 2e-11); the
// quotient takes the hardware reciprocal refined by two Newton steps.
__device__ inline double ln64(double u)
{
    int e;
    double m = frexp(u, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    const double s = (m - 1.0) * r;
    const double s2 = s * s;
    double p = 1.0 / 11.0;
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    return fma(double(e), 0.69314718055994531, 2.0 * s * p);
}
// exp: y = k ln 2 + r with ln 2 in two parts (k ln2_hi exact), |r| <= ln 2 / 2; exp r
// by its Taylor series through r^9 / 9! (relative error below 3e-11), then 2^k.
__device__ inline double exp64(double y)
{
    const double k = rint(y * 1.4426950408889634);
    double r = fma(-k, 6.93147180369123816490e-01, y);
    r = fma(-k, 1.90821492927058770002e-10, r);
    double p = 1.0 / 362880.0;
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, int(k));
}

template <typename T>
struct TersoffT {
    T A, B, l1, l2, c2, d2, c2d2, h, R, S, pi_w;
    double n, bn, lnbeta, inv2n, A64, B64, l1_64, l2_64;
    __device__ explicit TersoffT(const BandDev& b)
        : A(uni(T(b.ts_A))), B(uni(T(b.ts_B))), l1(uni(T(b.ts_l1))), l2(uni(T(b.ts_l2))),
          c2(uni(T(b.ts_c2))), d2(uni(T(b.ts_d2))), c2d2(uni(T(b.ts_c2d2))), h(uni(T(b.ts_h))),
          R(uni(T(b.ts_R))), S(uni(T(b.ts_S))), pi_w(uni(T(3.14159265358979323846 / (b.ts_S - b.ts_R)))),
          n(uni(b.ts_n)), bn(uni(b.ts_bn)), lnbeta(uni(b.ts_lnbeta)), inv2n(uni(0.5 / b.ts_n)),
          A64(uni(b.ts_A)), B64(uni(b.ts_B)), l1_64(uni(b.ts_l1)), l2_64(uni(b.ts_l2))
    {
    }
    __device__ T fc(T r) const
    {
        if (r < R) return T(1);
        if (r >= S) return T(0);
        return T(0.5) + T(0.5) * cos(pi_w * (r - R));
    }
    __device__ T dfc(T r) const
    {
        if (r < R || r >= S) return T(0);
        return T(-0.5) * pi_w * sin(pi_w * (r - R));
    }
    __device__ void g_dg(T cs, T& g, T& dg) const
    {
        const T t = h - cs;
        const T x = t * t;
        const T den = d2 + x;
        const T iden = qdiv(T(1), den);
        g = T(1) + c2d2 * x * iden;
        dg = T(-2) * c2 * t * (iden * iden);
    }
    // bond order b = (1 + x)^(-1/2n), x = (beta zeta)^n, and its zeta derivative; b64
    // is b before rounding to T
    __device__ void bond_order(T z, T& b, T& db, double& b64) const
    {
        b = T(1);
        db = T(0);
        b64 = 1.0;
        if (z > T(0)) {
            if constexpr (sizeof(T) == 4) {
                const double x = exp64(n * (ln64(double(z)) + lnbeta));
                const double u = 1.0 + x;
                b64 = exp64(-inv2n * ln64(u));
                b = T(b64);
                db = T(-0.5) * qdiv(T(x), z) * qdiv(b, T(u));
            } else {
                const T x = T(bn) * pow(z, T(n));
                const T base = T(1) + x;
                b = pow(base, T(-0.5) / T(n));
                db = T(-0.5) * qdiv(x, z) * qdiv(b, base);
                b64 = double(b);
            }
        }
    }
    // Pair terms A exp(-l1 r) and B exp(-l2 r) and the bond energy.  On the FP32 path
    // the energy is summed in FP64 from FP64 terms of the FP32 bond length: in a
    // perfect crystal every bond rounds alike, so FP32 terms would add their roundings
    // coherently (about 2e-6 eV/atom on diamond).  Both terms take the same FP32 r, so
    // its rounding cancels in fr - b fa near the bond's minimum.  Each term is formed
    // once in FP64 and rounded for the force; the repulsive energy half is added at
    // once, the attractive one when the bond order is known.  On the FP64 path the
    // whole bond energy is added with the attractive half.
    __device__ T repulsive(T r) const
    {
        if constexpr (sizeof(T) == 4)
            return T(A64 * exp64(-l1_64 * double(r)));
        else
            return A * exp(-l1 * r);
    }
    __device__ T repulsive(T r, T fcr, double& e) const
    {
        if constexpr (sizeof(T) == 4) {
            const double f = A64 * exp64(-l1_64 * double(r));
            e += 0.5 * double(fcr) * f;
            return T(f);
        } else {
            return repulsive(r);
        }
    }
    // B exp(-l2 r): the FP64 value (FP32 path; for the energy) and its rounding
    __device__ T attractive(T r, double& fa64) const
    {
        if constexpr (sizeof(T) == 4) {
            fa64 = B64 * exp64(-l2_64 * double(r));
            return T(fa64);
        } else {
            fa64 = 0.0;
            return B * exp(-l2 * r);
        }
    }
    __device__ void attractive_energy(T fcr, T fa, T bb, double b64, double fa64, T fr, double& e) const
    {
        if constexpr (sizeof(T) == 4)
            e -= 0.5 * double(fcr) * (b64 * fa64);
        else
            e += double(T(0.5) * fcr * (fr - bb * fa));
    }
};

template <typename T>
using vec4_t = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
template <typename T>
using vec2_t = typename std::conditional<sizeof(T) == 4, float2, double2>::type;

// acc[0] += u_i, acc[1..9] -= r^ij (x) P_ij (row-major)
template <typename T>
__device__ inline void add_virial(double* acc, T dx, T dy, T dz, T px, T py, T pz)
{
    const double x = double(dx), y = double(dy), z = double(dz);
    acc[1] -= x * double(px);
    acc[2] -= x * double(py);
    acc[3] -= x * double(pz);
    acc[4] -= y * double(px);
    acc[5] -= y * double(py);
    acc[6] -= y * double(pz);
    acc[7] -= z * double(px);
    acc[8] -= z * double(py);
    acc[9] -= z * double(pz);
}


// Atoms with at most MAXB bonds: every bond quantity lives in registers.  cos,
// g(cos) and g'(cos) are symmetric in the two bonds, so each unordered bond pair is
// evaluated once: it adds to both zetas, and its derivative to both P's.  P_ij goes
// to the bond's candidate slot cid (LDS, one per bond at the given stride).
template <typename T, int MAXB>
__device__ void ts_atom_regs(const TersoffT<T>& P, const vec4_t<T> (&bond)[MAXB], const int* cid, int stride,
                             gmem<P3<T>>* Pout, size_t N, int i, int cnt, double* acc)
{
    constexpr int NP = MAXB * (MAXB - 1) / 2;
    T dx[MAXB], dy[MAXB], dz[MAXB], ir[MAXB], fc[MAXB], dfc[MAXB], fr[MAXB], fa[MAXB];
    double fa64[MAXB];
#pragma unroll
    for (int e = 0; e < MAXB; ++e) {
        if (e < cnt) {
            const vec4_t<T> d = bond[e];
            dx[e] = d.x;
            dy[e] = d.y;
            dz[e] = d.z;
            ir[e] = qdiv(T(1), d.w);
            fc[e] = P.fc(d.w);
            dfc[e] = P.dfc(d.w);
            fr[e] = P.repulsive(d.w, fc[e], acc[0]);
            fa[e] = P.attractive(d.w, fa64[e]);
        } else {
            dx[e] = dy[e] = dz[e] = T(0);
            ir[e] = T(1);
            fc[e] = dfc[e] = fr[e] = fa[e] = T(0);
            fa64[e] = 0.0;
        }
    }
    // pass 1: zeta of every bond from the unordered pairs (each zeta sums its pairs in
    // increasing order of the other bond)
    T csp[NP], gp[NP], dgp[NP], z[MAXB];
#pragma unroll
    for (int e = 0; e < MAXB; ++e) z[e] = T(0);
    {
        int p = 0;
#pragma unroll
        for (int e = 0; e < MAXB; ++e) {
#pragma unroll
            for (int q = e + 1; q < MAXB; ++q, ++p) {
                csp[p] = gp[p] = dgp[p] = T(0);
                if (q < cnt) {
                    const T cs = (dx[e] * dx[q] + dy[e] * dy[q] + dz[e] * dz[q]) * (ir[e] * ir[q]);
                    T g, dg;
                    P.g_dg(cs, g, dg);
                    csp[p] = cs;
                    gp[p] = g;
                    dgp[p] = dg;
                    z[e] += fc[q] * g;
                    z[q] += fc[e] * g;
                }
            }
        }
    }
    // bond orders, energy, radial derivative at fixed bond order, prefactor of zeta
    T dV[MAXB], pre[MAXB];
#pragma unroll
    for (int e = 0; e < MAXB; ++e) {
        dV[e] = pre[e] = T(0);
        if (e < cnt) {
            T bb, db;
            double b64;
            P.bond_order(z[e], bb, db, b64);
            P.attractive_energy(fc[e], fa[e], bb, b64, fa64[e], fr[e], acc[0]);
            dV[e] = dfc[e] * (fr[e] - bb * fa[e]) + fc[e] * (-P.l1 * fr[e] + bb * P.l2 * fa[e]);
            pre[e] = fc[e] * fa[e] * db;
        }
    }
    // pass 2: P_e = dU_i/dr^e
    T px[MAXB], py[MAXB], pz[MAXB], hx[MAXB], hy[MAXB], hz[MAXB];
#pragma unroll
    for (int e = 0; e < MAXB; ++e) {
        hx[e] = dx[e] * ir[e];
        hy[e] = dy[e] * ir[e];
        hz[e] = dz[e] * ir[e];
        px[e] = T(0.5) * dV[e] * hx[e];
        py[e] = T(0.5) * dV[e] * hy[e];
        pz[e] = T(0.5) * dV[e] * hz[e];
    }
    {
        int p = 0;
#pragma unroll
        for (int e = 0; e < MAXB; ++e) {
#pragma unroll
            for (int q = e + 1; q < MAXB; ++q, ++p) {
                if (q >= cnt) continue;
                const T a = ir[e] * ir[q];
                const T cs = csp[p];
                // zeta_e holds fc(r_q) g(cos), zeta_q holds fc(r_e) g(cos)
                const T ang = T(0.5) * (pre[e] * fc[q] + pre[q] * fc[e]) * dgp[p];
                // d cos / d r^e and d cos / d r^q
                const T ce = cs * ir[e] * ir[e], cq = cs * ir[q] * ir[q];
                const T ex = dx[q] * a - ce * dx[e], ey = dy[q] * a - ce * dy[e], ez = dz[q] * a - ce * dz[e];
                const T qx = dx[e] * a - cq * dx[q], qy = dy[e] * a - cq * dy[q], qz = dz[e] * a - cq * dz[q];
                const T rad_e = T(0.5) * pre[q] * dfc[e] * gp[p];
                const T rad_q = T(0.5) * pre[e] * dfc[q] * gp[p];
                px[e] -= ang * ex + rad_e * hx[e];
                py[e] -= ang * ey + rad_e * hy[e];
                pz[e] -= ang * ez + rad_e * hz[e];
                px[q] -= ang * qx + rad_q * hx[q];
                py[q] -= ang * qy + rad_q * hy[q];
                pz[q] -= ang * qz + rad_q * hz[q];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < MAXB; ++e) {
        if (e >= cnt) continue;
        store3(Pout, size_t(cid[e * stride]) * N + i, px[e], py[e], pz[e]);
        add_virial<T>(acc, dx[e], dy[e], dz[e], px[e], py[e], pz[e]);
    }
}

// Any number of bonds: bond orders go through the per-bond scratch array; bcid holds
// each bond's candidate slot.
template <typename T>
__device__ void ts_atom_generic(const TersoffT<T>& P, const vec4_t<T>* dv, vec2_t<T>* bo, const int* bcid,
                                P3<T>* Pout, size_t N, int i, int cnt, double* acc)
{
    for (int e = 0; e < cnt; ++e) {
        const vec4_t<T> de = dv[size_t(e) * N + i];
        T z = 0;
        for (int q = 0; q < cnt; ++q) {
            if (q == e) continue;
            const vec4_t<T> dq = dv[size_t(q) * N + i];
            const T cs = (de.x * dq.x + de.y * dq.y + de.z * dq.z) / (de.w * dq.w);
            T g, dg;
            P.g_dg(cs, g, dg);
            z += P.fc(dq.w) * g;
        }
        vec2_t<T> o;
        double b64, fa64;
        P.bond_order(z, o.x, o.y, b64);
        bo[size_t(e) * N + i] = o;
        const T fce = P.fc(de.w);
        const T fr = P.repulsive(de.w, fce, acc[0]), fa = P.attractive(de.w, fa64);
        P.attractive_energy(fce, fa, o.x, b64, fa64, fr, acc[0]);
    }
    for (int e = 0; e < cnt; ++e) {
        const vec4_t<T> de = dv[size_t(e) * N + i];
        const vec2_t<T> be = bo[size_t(e) * N + i];
        const T re = de.w, ire = T(1) / re;
        const T hx = de.x * ire, hy = de.y * ire, hz = de.z * ire;
        const T fce = P.fc(re), dfce = P.dfc(re);
        double fa64;
        const T fre = P.repulsive(re), fae = P.attractive(re, fa64);
        const T dV = dfce * (fre - be.x * fae) + fce * (-P.l1 * fre + be.x * P.l2 * fae);
        T px = T(0.5) * dV * hx, py = T(0.5) * dV * hy, pz = T(0.5) * dV * hz;
        const T pre_e = fce * fae * be.y;
        for (int q = 0; q < cnt; ++q) {
            if (q == e) continue;
            const vec4_t<T> dq = dv[size_t(q) * N + i];
            const vec2_t<T> bq = bo[size_t(q) * N + i];
            const T rq = dq.w;
            const T a = T(1) / (re * rq);
            const T cs = (de.x * dq.x + de.y * dq.y + de.z * dq.z) * a;
            const T c = cs * ire * ire;
            const T cx = dq.x * a - c * de.x, cy = dq.y * a - c * de.y, cz = dq.z * a - c * de.z;
            T g, dg;
            P.g_dg(cs, g, dg);
            const T fcq = P.fc(rq);
            double faq64;
            const T pre_q = fcq * P.attractive(rq, faq64) * bq.y;
            const T ang = T(0.5) * (pre_e * fcq + pre_q * fce) * dg;
            const T rad = T(0.5) * pre_q * dfce * g;
            px -= ang * cx + rad * hx;
            py -= ang * cy + rad * hy;
            pz -= ang * cz + rad * hz;
        }
        Pout[size_t(bcid[size_t(e) * N + i]) * N + i] = P3<T>{px, py, pz};
        add_virial<T>(acc, de.x, de.y, de.z, px, py, pz);
    }
}

// Reverse candidate of each of atom i's candidates: the slot q of (i, -n) in j's list,
// stored as its index q N + j in P (the gather's one load).  Runs on the steps that
// rebuild the image's candidates.
__device__ void ts_reverse_candidates(const BandDev& b, BandState* st, int slot, int i, int nc)
{
    const size_t N = b.N;
    const gmem<const uint32_t>* __restrict__ cand = gp<const uint32_t>(b.cand + size_t(slot) * b.ccap * N);
    const gmem<const int>* __restrict__ ncand = gp<const int>(b.ncand + size_t(slot) * N);
    gmem<uint32_t>* __restrict__ crev = gp(b.crev + size_t(slot) * b.ccap * N);
    bool missing = false;
    for (int c = 0; c < nc; ++c) {
        const uint32_t ent = cand[size_t(c) * N + i];
        const int j = nbr_j(ent);
        const uint32_t want = pack_nbr(i, -nbr_n(ent, 0), -nbr_n(ent, 1), -nbr_n(ent, 2));
        const int cj = ncand[j];
        int found = -1;
        for (int q = 0; q < cj; ++q)
            if (cand[size_t(q) * N + j] == want) {
                found = q;
                break;
            }
        if (found < 0) {
            missing = true;
            found = 0;
        }
        crev[size_t(c) * N + i] = uint32_t(size_t(found) * N + size_t(j));
    }
    if (missing) set_error(st, CFNEB_ENEIGH);
}

// Bonds held in LDS per thread, for atoms with at most this many (carbon: 3 or 4).
#define TS_LDS_BONDS 4

// Neighbours of atom i by the exact test of its candidates (as the candidate filter
// does for LJ), then u_i, P_ij and the per-atom virial from the bond vectors; wave
// partials of (E, V) in FP64.  The first four bonds go to this thread's LDS slots
// (an LDS store at a per-lane index, where registers would need a select per slot)
// and then to registers; an atom with more bonds writes them to global scratch and
// takes the general path.
template <typename T>
__device__ void ts_filter_bonds_item(const BandDev& b, BandState* st, int slot, int tile,
                                     vec4_t<T>* lbond, int* lcid)
{
    constexpr int MB = TS_LDS_BONDS;
    const int tid = threadIdx.x;
    const int i = tile * CFNEB_TILE + tid;
    const size_t N = b.N;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < b.N) {
        const cmem<ImageGeom>* g = cp(b.geom + slot);
        const gmem<const R3>* __restrict__ R = gp<const R3>(Rs(b, slot));
        const gmem<const uint32_t>* __restrict__ cand = gp<const uint32_t>(b.cand + size_t(slot) * b.ccap * N);
        P3<T>* Praw = reinterpret_cast<P3<T>*>(b.P) + size_t(slot) * b.ccap * N;
        gmem<P3<T>>* __restrict__ Pout = gp(Praw);
        vec4_t<T>* dv = reinterpret_cast<vec4_t<T>*>(b.dvec) + size_t(slot) * b.cap * N;
        int* bcid = reinterpret_cast<int*>(b.bcid) + size_t(slot) * b.cap * N;
        double h[9];
        for (int q = 0; q < 9; ++q) h[q] = g->h[q];
        const double4 r4 = load4(R, i);
        const double ri[3] = {r4.x, r4.y, r4.z};
        const int nc = gp<const int>(b.ncand)[size_t(slot) * N + i];
        const double rc2 = b.rc2;
        const int cap = b.cap;
        if (cp(b.skst + slot)->rebuild) ts_reverse_candidates(b, st, slot, i, nc);
        const vec4_t<T> zero{};
        int cnt = 0;
        // four candidates at a time (carbon atoms have three or four): one round of
        // dependent loads for most atoms; the tests stop at the atom's last candidate
        constexpr int U = 4;
        for (int e0 = 0; e0 < nc; e0 += U) {
            uint32_t ent[U];
            double4 rj[U];
            // past the last candidate the loads repeat it (in bounds, no branch
            // between the loads); the tests below stop there
#pragma unroll
            for (int u = 0; u < U; ++u) ent[u] = cand[size_t(min(e0 + u, nc - 1)) * N + i];
#pragma unroll
            for (int u = 0; u < U; ++u) rj[u] = load4(R, nbr_j(ent[u]));
            __builtin_amdgcn_sched_barrier(0);  // the batch's positions are in flight together
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u >= nc) break;
                double d[3];
                const double rr = exact_r2(ri, rj[u].x, rj[u].y, rj[u].z, h, nbr_n(ent[u], 0), nbr_n(ent[u], 1),
                                           nbr_n(ent[u], 2), d);
                if (!(rr < rc2)) {
                    store3(Pout, size_t(e0 + u) * N + i, T(0), T(0), T(0));
                    continue;
                }
                if (cnt < cap) {
                    vec4_t<T> v;
                    v.x = T(d[0]);
                    v.y = T(d[1]);
                    v.z = T(d[2]);
                    v.w = sqrt(T(rr));  // the FP32 bond length from the rounded r^2
                    if (cnt < MB) {
                        lbond[cnt * CFNEB_TILE + tid] = v;
                        lcid[cnt * CFNEB_TILE + tid] = e0 + u;
                    } else {
                        dv[size_t(cnt) * N + i] = v;
                        bcid[size_t(cnt) * N + i] = e0 + u;
                    }
                }
                ++cnt;
            }
        }
        if (cnt > cap) set_error(st, CFNEB_ENEIGH);
        const int nb = min(cnt, cap);
        const TersoffT<T> P(b);
        if (nb <= MB) {
            vec4_t<T> bond[MB];
#pragma unroll
            for (int e = 0; e < MB; ++e) bond[e] = (e < nb) ? lbond[e * CFNEB_TILE + tid] : zero;
            ts_atom_regs<T, MB>(P, bond, lcid + tid, CFNEB_TILE, Pout, N, i, nb, acc);
        } else {
            for (int e = 0; e < MB; ++e) {
                dv[size_t(e) * N + i] = lbond[e * CFNEB_TILE + tid];
                bcid[size_t(e) * N + i] = lcid[e * CFNEB_TILE + tid];
            }
            vec2_t<T>* bo = reinterpret_cast<vec2_t<T>*>(b.bo) + size_t(slot) * b.cap * N;
            ts_atom_generic<T>(P, dv, bo, bcid, Praw, N, i, nb, acc);
        }
    }
    store_ev_partials(b, slot, tile, acc);
}

template <typename T>
__device__ void ts_filter_bonds_loop(const BatchDev& bd, int all_images, int variant)
{
    __shared__ vec4_t<T> lbond[TS_LDS_BONDS * CFNEB_TILE];
    __shared__ int lcid[TS_LDS_BONDS * CFNEB_TILE];
    ItemLoopRO loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        const cmem<BandState>* sr = cp(b.st);
        if (int(band_variant(b) != variant) | int(band_stopped(sr))) continue;  // uniform over the block
        ts_filter_bonds_item<T>(b, b.st, sr->slot[it.image], it.tile, lbond, lcid);
    }
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_ts_filter_bonds(BatchDev bd, int all_images, int variant)
{
    ts_filter_bonds_loop<T>(bd, all_images, variant);
}

// FP32 bonds: four waves per SIMD (at most 128 VGPRs); left alone the FP64 energy
// terms take more registers and the kernel runs slower at three.
template <>
__global__ void __launch_bounds__(CFNEB_TILE) __attribute__((amdgpu_waves_per_eu(4)))
k_ts_filter_bonds<float>(BatchDev bd, int all_images, int variant)
{
    ts_filter_bonds_loop<float>(bd, all_images, variant);
}

// F_i = sum_c (P_c - P_rev(c)) over i's candidates (tersoff_gather), one atom per
// thread.
template <typename T>
__device__ void ts_gather_item(const BandDev& b, BandState* st, int slot, int i)
{
    T f[1][3];
    tersoff_gather<T, 1>(b, slot, i, 0, f);
    gmem<T>* F = gp(reinterpret_cast<T*>(b.F) + size_t(slot) * slot_rows(b));
    F[i] = f[0][0];
    F[b.ld + i] = f[0][1];
    F[2 * size_t(b.ld) + i] = f[0][2];
    if (!isfinite(double(f[0][0]) + double(f[0][1]) + double(f[0][2]))) set_error(st, CFNEB_ENONFINITE);
}

// stage 0: bond orders, P_ij, energy and virial; stage 1: force gather
template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_ts_gather(BatchDev bd, int all_images, int variant)
{
    ItemLoopRO loop(bd, KIND_ATOM, all_images);
    Item it;
    while (loop.next(it)) {
        const BandDev b = band_ro(bd, it.band);
        const cmem<BandState>* sr = cp(b.st);
        const int i = it.tile * CFNEB_TILE + threadIdx.x;
        if ((int(band_variant(b) != variant) | int(band_stopped(sr))) || i >= b.N) continue;
        ts_gather_item<T>(b, b.st, sr->slot[it.image], i);
    }
}

void launch_tersoff_stage(const Launch& L, int all_images, int stage, hipStream_t s)
{
    const unsigned g = L.g_force;
    if (L.variants & (1u << VARIANT_TS32)) {
        if (stage == 0) k_ts_filter_bonds<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_TS32);
        if (stage == 1) k_ts_gather<float><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_TS32);
    }
    if (L.variants & (1u << VARIANT_TS64)) {
        if (stage == 0) k_ts_filter_bonds<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_TS64);
        if (stage == 1) k_ts_gather<double><<<g, CFNEB_TILE, 0, s>>>(L.bd, all_images, VARIANT_TS64);
    }
}

}  // namespace cfneb
