// Energies, forces and virials of every image (Sec. II.B).
//
// Each atom's energy U_i is a function of the bond vectors r^ij to its neighbours
// (Eq. (4)).  With P_ij = dU_i/dr^ij the force is F_i = sum_j (P_ij - P_ji) (the
// pair force of Eq. (5) in the index order of the derivation leading to Eq. (6)),
// and the virial is V_mn = -sum_ij r^ij_m P_ij,n = -1/2 sum_ij r^ij_m f^ij_n
// (Eqs. (6)-(8)).  Lists are full, so every force is a gather: no atomics.
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
__global__ void __launch_bounds__(CFNEB_TILE) k_lj(BandDev b, int all_images)
{
    __shared__ double lds[4 * 10];
    BandState* st = b.st;
    const int k = blockIdx.y;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    const int slot = st->slot[k];
    const size_t N = b.N;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // u, then V row-major
    if (i < b.N) {
        const double* R = Rs(b, slot);
        const ImageGeom& g = b.geom[slot];
        double h[9];
        for (int q = 0; q < 9; ++q) h[q] = g.h[q];
        const double ri0 = R[i], ri1 = R[b.ld + i], ri2 = R[2 * size_t(b.ld) + i];
        const uint32_t* nbr = b.nbr + size_t(slot) * b.cap * N;
        const int cnt = min(b.ncnt[size_t(slot) * N + i], b.cap);
        const T eps4 = T(4.0 * b.lj_eps), eps24 = T(24.0 * b.lj_eps), sig2 = T(b.lj_sig2),
                esh = T(b.lj_eshift);
        T fx = 0, fy = 0, fz = 0;
        for (int e = 0; e < cnt; ++e) {
            const uint32_t ent = nbr[size_t(e) * N + i];
            const int j = nbr_j(ent);
            const int n0 = nbr_n(ent, 0), n1 = nbr_n(ent, 1), n2 = nbr_n(ent, 2);
            const double d0 = (R[j] - ri0) + ((n0 * h[0] + n1 * h[3]) + n2 * h[6]);
            const double d1 = (R[b.ld + j] - ri1) + ((n0 * h[1] + n1 * h[4]) + n2 * h[7]);
            const double d2 = (R[2 * size_t(b.ld) + j] - ri2) + ((n0 * h[2] + n1 * h[5]) + n2 * h[8]);
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
        T* F = reinterpret_cast<T*>(b.F) + size_t(slot) * slot_rows(b);
        F[i] = fx;
        F[b.ld + i] = fy;
        F[2 * size_t(b.ld) + i] = fz;
        if (!isfinite(double(fx) + double(fy) + double(fz))) set_error(st, CFNEB_ENONFINITE);
    }
    block_sum<10>(acc, lds);
    if (threadIdx.x == 0) {
        double* out = b.evpart + (size_t(slot) * b.ntA + blockIdx.x) * 10;
        for (int q = 0; q < 10; ++q) out[q] = acc[q];
    }
}

// ------------------------------------------------------------ Tersoff
// U_i = 1/2 sum_j fc(r_ij) [A exp(-l1 r_ij) - b_ij B exp(-l2 r_ij)],
// b_ij = (1 + beta^n zeta_ij^n)^(-1/2n), zeta_ij = sum_{k != j} fc(r_ik) g(cos theta_ijk).
// g is evaluated as 1 + (c^2/d^2) x / (d^2 + x), x = (h - cos)^2: the textbook form
// 1 + c^2/d^2 - c^2/(d^2 + x) cancels two numbers near 7.7e7 and loses about four
// digits in FP32.
template <typename T>
struct TersoffT {
    T A, B, l1, l2, bn, n, c2, d2, c2d2, h, R, S, pi_w;
    __device__ explicit TersoffT(const BandDev& b)
        : A(T(b.ts_A)), B(T(b.ts_B)), l1(T(b.ts_l1)), l2(T(b.ts_l2)), bn(T(b.ts_bn)), n(T(b.ts_n)),
          c2(T(b.ts_c2)), d2(T(b.ts_d2)), c2d2(T(b.ts_c2d2)), h(T(b.ts_h)), R(T(b.ts_R)), S(T(b.ts_S)),
          pi_w(T(3.14159265358979323846 / (b.ts_S - b.ts_R)))
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
        g = T(1) + c2d2 * x / den;
        dg = T(-2) * c2 * t / (den * den);
    }
};

template <typename T>
using vec4_t = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
template <typename T>
using vec2_t = typename std::conditional<sizeof(T) == 4, float2, double2>::type;

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_ts_zeta(BandDev b, int all_images)
{
    __shared__ double lds[4];
    BandState* st = b.st;
    const int k = blockIdx.y;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    const int slot = st->slot[k];
    const size_t N = b.N;
    double acc[1] = {0.0};
    if (i < b.N) {
        const TersoffT<T> P(b);
        const vec4_t<T>* dv = reinterpret_cast<const vec4_t<T>*>(b.dvec) + size_t(slot) * b.cap * N;
        vec2_t<T>* bo = reinterpret_cast<vec2_t<T>*>(b.bo) + size_t(slot) * b.cap * N;
        const int cnt = min(b.ncnt[size_t(slot) * N + i], b.cap);
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
            T bij = T(1), dbij = T(0);
            if (z > T(0)) {
                const T zn = pow(z, P.n);
                const T base = T(1) + P.bn * zn;
                bij = pow(base, T(-0.5) / P.n);
                dbij = T(-0.5) * P.bn * (zn / z) * (bij / base);
            }
            vec2_t<T> o;
            o.x = bij;
            o.y = dbij;
            bo[size_t(e) * N + i] = o;
            const T r = de.w;
            const T fr = P.A * exp(-P.l1 * r), fa = P.B * exp(-P.l2 * r);
            acc[0] += double(T(0.5) * P.fc(r) * (fr - bij * fa));
        }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) b.evpart[(size_t(slot) * b.ntA + blockIdx.x) * 10] = acc[0];
}

template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_ts_partial(BandDev b, int all_images)
{
    __shared__ double lds[4 * 9];
    BandState* st = b.st;
    const int k = blockIdx.y;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    const int slot = st->slot[k];
    const size_t N = b.N;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < b.N) {
        const TersoffT<T> P(b);
        const vec4_t<T>* dv = reinterpret_cast<const vec4_t<T>*>(b.dvec) + size_t(slot) * b.cap * N;
        const vec2_t<T>* bo = reinterpret_cast<const vec2_t<T>*>(b.bo) + size_t(slot) * b.cap * N;
        vec4_t<T>* Pout = reinterpret_cast<vec4_t<T>*>(b.P) + size_t(slot) * b.cap * N;
        const int cnt = min(b.ncnt[size_t(slot) * N + i], b.cap);
        for (int e = 0; e < cnt; ++e) {
            const vec4_t<T> de = dv[size_t(e) * N + i];
            const vec2_t<T> be = bo[size_t(e) * N + i];
            const T re = de.w, ire = T(1) / re;
            const T hx = de.x * ire, hy = de.y * ire, hz = de.z * ire;
            const T fce = P.fc(re), dfce = P.dfc(re);
            const T fre = P.A * exp(-P.l1 * re), fae = P.B * exp(-P.l2 * re);
            // radial derivative at fixed bond order
            const T dV = dfce * (fre - be.x * fae) + fce * (-P.l1 * fre + be.x * P.l2 * fae);
            T px = T(0.5) * dV * hx, py = T(0.5) * dV * hy, pz = T(0.5) * dV * hz;
            const T pre_e = fce * fae * be.y;
            for (int q = 0; q < cnt; ++q) {
                if (q == e) continue;
                const vec4_t<T> dq = dv[size_t(q) * N + i];
                const vec2_t<T> bq = bo[size_t(q) * N + i];
                const T rq = dq.w;
                const T cs = (de.x * dq.x + de.y * dq.y + de.z * dq.z) / (re * rq);
                const T a = T(1) / (re * rq), c = cs * ire * ire;
                // d cos / d r^ie
                const T cx = dq.x * a - c * de.x, cy = dq.y * a - c * de.y, cz = dq.z * a - c * de.z;
                T g, dg;
                P.g_dg(cs, g, dg);
                const T fcq = P.fc(rq);
                const T pre_q = fcq * (P.B * exp(-P.l2 * rq)) * bq.y;
                // zeta_ie holds fc(r_q) g(cos); zeta_iq holds fc(r_e) g(cos)
                const T ang = T(0.5) * (pre_e * fcq + pre_q * fce) * dg;
                const T rad = T(0.5) * pre_q * dfce * g;
                px -= ang * cx + rad * hx;
                py -= ang * cy + rad * hy;
                pz -= ang * cz + rad * hz;
            }
            vec4_t<T> o;
            o.x = px;
            o.y = py;
            o.z = pz;
            o.w = T(0);
            Pout[size_t(e) * N + i] = o;
            const double dx = double(de.x), dy = double(de.y), dz = double(de.z);
            acc[0] -= dx * double(px);
            acc[1] -= dx * double(py);
            acc[2] -= dx * double(pz);
            acc[3] -= dy * double(px);
            acc[4] -= dy * double(py);
            acc[5] -= dy * double(pz);
            acc[6] -= dz * double(px);
            acc[7] -= dz * double(py);
            acc[8] -= dz * double(pz);
        }
    }
    block_sum<9>(acc, lds);
    if (threadIdx.x == 0) {
        double* out = b.evpart + (size_t(slot) * b.ntA + blockIdx.x) * 10 + 1;
        for (int q = 0; q < 9; ++q) out[q] = acc[q];
    }
}

// F_i = sum_e (P_e - P_rev(e)), rev(e) = the entry (i, -n) in j's list.
template <typename T>
__global__ void __launch_bounds__(CFNEB_TILE) k_ts_gather(BandDev b, int all_images)
{
    BandState* st = b.st;
    const int k = blockIdx.y;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    if (i >= b.N) return;
    const int slot = st->slot[k];
    const size_t N = b.N;
    const uint32_t* nbr = b.nbr + size_t(slot) * b.cap * N;
    const int* ncnt = b.ncnt + size_t(slot) * N;
    const vec4_t<T>* Pb = reinterpret_cast<const vec4_t<T>*>(b.P) + size_t(slot) * b.cap * N;
    const int cnt = min(ncnt[i], b.cap);
    T fx = 0, fy = 0, fz = 0;
    bool missing = false;
    for (int e = 0; e < cnt; ++e) {
        const uint32_t ent = nbr[size_t(e) * N + i];
        const int j = nbr_j(ent);
        const vec4_t<T> pe = Pb[size_t(e) * N + i];
        fx += pe.x;
        fy += pe.y;
        fz += pe.z;
        const uint32_t want = pack_nbr(i, -nbr_n(ent, 0), -nbr_n(ent, 1), -nbr_n(ent, 2));
        const int cj = min(ncnt[j], b.cap);
        int found = -1;
        for (int q = 0; q < cj; ++q)
            if (nbr[size_t(q) * N + j] == want) {
                found = q;
                break;
            }
        if (found < 0) {
            missing = true;
            continue;
        }
        const vec4_t<T> pr = Pb[size_t(found) * N + j];
        fx -= pr.x;
        fy -= pr.y;
        fz -= pr.z;
    }
    T* F = reinterpret_cast<T*>(b.F) + size_t(slot) * slot_rows(b);
    F[i] = fx;
    F[b.ld + i] = fy;
    F[2 * size_t(b.ld) + i] = fz;
    if (missing) set_error(st, CFNEB_ENEIGH);
    if (!isfinite(double(fx) + double(fy) + double(fz))) set_error(st, CFNEB_ENONFINITE);
}

// ------------------------------------------------------------ per-image reduction
// E and V in a fixed order; enthalpy and the rotation-free lattice force
// G = D^-T (V - P Omega I) D^-1 / c_f (Eqs. (16)-(17)).
__global__ void __launch_bounds__(CFNEB_TILE) k_image_reduce(BandDev b, int all_images)
{
    __shared__ double lds[4 * 10];
    BandState* st = b.st;
    const int k = blockIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int slot = st->slot[k];
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double* part = b.evpart + size_t(slot) * b.ntA * 10;
    for (int t = threadIdx.x; t < b.ntA; t += CFNEB_TILE)
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
    double DinvT[9], T1[9], G[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) DinvT[3 * r + c] = g.Dinv[3 * c + r];
    mm3(DinvT, Veff, T1);
    mm3(T1, g.Dinv, G);
    const double sc = (b.cell_filter == 2) ? b.bscale / b.cf : 0.0;
    for (int q = 0; q < 9; ++q) s.Fcell[q] = sc * G[q];
    if (!finite) set_error(st, CFNEB_ENONFINITE);
}

// stage 0: LJ, or Tersoff zeta and bond orders; 1: Tersoff dU_i/dr^ij; 2: Tersoff gather
void launch_force_stage(const BandDev& b, int all_images, int stage, hipStream_t s)
{
    const dim3 gA(b.ntA, b.Mcap);
    if (b.potential == CFNEB_LJ) {
        if (stage != 0) return;
        if (b.fp64)
            k_lj<double><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        else
            k_lj<float><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        return;
    }
    if (b.fp64) {
        if (stage == 0) k_ts_zeta<double><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        if (stage == 1) k_ts_partial<double><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        if (stage == 2) k_ts_gather<double><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    } else {
        if (stage == 0) k_ts_zeta<float><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        if (stage == 1) k_ts_partial<float><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        if (stage == 2) k_ts_gather<float><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    }
}

void launch_image_reduce(const BandDev& b, int all_images, hipStream_t s)
{
    k_image_reduce<<<b.Mcap, CFNEB_TILE, 0, s>>>(b, all_images);
}

void launch_forces(const BandDev& b, int all_images, hipStream_t s)
{
    for (int stage = 0; stage < 3; ++stage) launch_force_stage(b, all_images, stage, s);
    launch_image_reduce(b, all_images, s);
}

void launch_evaluate(const BandDev& b, int all_images, hipStream_t s)
{
    launch_geom(b, all_images, s);
    launch_nlist(b, all_images, s);
    launch_forces(b, all_images, s);
}

}  // namespace cfneb
