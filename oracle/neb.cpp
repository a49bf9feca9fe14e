// Oracle (test infrastructure only): NEB projection, climbing image, FIRE and
// adaptive images, for any band whose images are flat vectors of rows.
//
//   NEB force (Sec. II.A, Eq. (1)):  F_NEB = F - (F . t) t + k (|tau+| - |tau-|) t
//   climbing image (cited in Sec. I):  F_CI = F - 2 (F . t) t, no spring
//   improved tangent (cited in Sec. I): energy-weighted upwind choice of tau+ / tau-
//   FIRE (the usual optimizer of the band, Secs. II.C / III), band-global, unit mass
//   adaptive images (Sec. III): after an iteration, insert an image into a long
//   interval or delete an image between two short ones.
#include "internal.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace orc {

struct Fire {
    double dt, alpha;
    int n_pos, fresh;
};

struct NebCore {
    int M = 0, dim = 0, roww = 3;
    int natoms = 0;  // leading atom rows of a periodic structure (0: none)
    std::vector<std::vector<double>> X, v, Fg, Fneb;
    std::vector<double> H;
    Fire fire{};
    int step = 0, ci = -1;
};

double dot(const std::vector<double>& a, const std::vector<double>& b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

}  // namespace orc

// Improved tangent (Henkelman & Jonsson 2000, cited by the paper):
// upwind neighbour on a monotonic energy profile, else an energy-weighted mix.
extern "C" void orc_tangent_coeffs(double Hm, double H0, double Hp, double* a, double* b)
{
    if (Hp > H0 && H0 > Hm) {
        *a = 1.0;
        *b = 0.0;
    } else if (Hp < H0 && H0 < Hm) {
        *a = 0.0;
        *b = 1.0;
    } else {
        const double dp = std::fabs(Hp - H0), dm = std::fabs(Hm - H0);
        const double dmax = std::max(dp, dm), dmin = std::min(dp, dm);
        if (Hp > Hm) {
            *a = dmax;
            *b = dmin;
        } else {
            *a = dmin;
            *b = dmax;
        }
    }
}

namespace orc {

// A rigid translation of all atoms of a periodic structure changes no energy.  It is
// removed from the atom rows of image differences and forces: each of the three
// components has its mean over the atom rows subtracted (cell rows untouched).
void remove_translation(std::vector<double>& a, int natoms)
{
    if (natoms <= 0) return;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int i = 0; i < natoms; ++i) s += a[3 * size_t(i) + q];
        const double m = s / natoms;
        for (int i = 0; i < natoms; ++i) a[3 * size_t(i) + q] -= m;
    }
}

// NEB forces on the moving images from X, H and the true generalized forces Fg,
// all taken modulo a rigid translation of the atoms.
void neb_forces(NebCore& c, double k_spring, int climb_after)
{
    const int M = c.M;
    c.ci = -1;
    if (climb_after >= 0 && c.step >= climb_after) {
        double best = 0.0;
        for (int k = 1; k <= M - 2; ++k)
            if (c.ci < 0 || c.H[k] > best) {
                c.ci = k;
                best = c.H[k];
            }
    }
    std::vector<double> tp(c.dim), tm(c.dim), tau(c.dim), F(c.dim);
    c.Fneb.assign(M, std::vector<double>(c.dim, 0.0));
    for (int k = 1; k <= M - 2; ++k) {
        for (int i = 0; i < c.dim; ++i) {
            tp[i] = c.X[k + 1][i] - c.X[k][i];
            tm[i] = c.X[k][i] - c.X[k - 1][i];
        }
        F = c.Fg[k];
        remove_translation(tp, c.natoms);
        remove_translation(tm, c.natoms);
        remove_translation(F, c.natoms);
        double a, b;
        orc_tangent_coeffs(c.H[k - 1], c.H[k], c.H[k + 1], &a, &b);
        for (int i = 0; i < c.dim; ++i) tau[i] = a * tp[i] + b * tm[i];
        const double nt = std::sqrt(dot(tau, tau));
        if (nt > 0.0)
            for (double& t : tau) t /= nt;
        const double ft = dot(F, tau);
        auto& out = c.Fneb[k];
        if (k == c.ci) {
            for (int i = 0; i < c.dim; ++i) out[i] = F[i] - 2.0 * ft * tau[i];
        } else {
            const double spring = k_spring * (std::sqrt(dot(tp, tp)) - std::sqrt(dot(tm, tm)));
            for (int i = 0; i < c.dim; ++i) out[i] = F[i] - ft * tau[i] + spring * tau[i];
        }
    }
}

double fmax_of(const NebCore& c)
{
    double m = 0.0;
    for (int k = 1; k <= c.M - 2; ++k)
        for (int r = 0; r < c.dim / c.roww; ++r) {
            double s = 0.0;
            for (int q = 0; q < c.roww; ++q) s += c.Fneb[k][c.roww * r + q] * c.Fneb[k][c.roww * r + q];
            m = std::max(m, std::sqrt(s));
        }
    return m;
}

// FIRE (Bitzek et al. 2006) on the moving images as one vector.
void fire_move(NebCore& c, double dtmax, double maxstep, int nmin, double finc, double fdec,
               double astart, double fa)
{
    const int M = c.M;
    auto& st = c.fire;
    if (!st.fresh) {
        double P = 0.0, ff = 0.0, vv = 0.0;
        for (int k = 1; k <= M - 2; ++k) {
            P += dot(c.Fneb[k], c.v[k]);
            ff += dot(c.Fneb[k], c.Fneb[k]);
            vv += dot(c.v[k], c.v[k]);
        }
        if (P > 0.0) {
            const double nf = std::sqrt(ff), nv = std::sqrt(vv);
            if (nf > 0.0)
                for (int k = 1; k <= M - 2; ++k)
                    for (int i = 0; i < c.dim; ++i)
                        c.v[k][i] = (1.0 - st.alpha) * c.v[k][i] + st.alpha * nv * c.Fneb[k][i] / nf;
            if (st.n_pos > nmin) {
                st.dt = std::min(st.dt * finc, dtmax);
                st.alpha *= fa;
            }
            st.n_pos += 1;
        } else {
            for (int k = 1; k <= M - 2; ++k) std::fill(c.v[k].begin(), c.v[k].end(), 0.0);
            st.alpha = astart;
            st.dt *= fdec;
            st.n_pos = 0;
        }
    }
    st.fresh = 0;
    double maxrow = 0.0;
    for (int k = 1; k <= M - 2; ++k) {
        for (int i = 0; i < c.dim; ++i) c.v[k][i] += st.dt * c.Fneb[k][i];
        for (int r = 0; r < c.dim / c.roww; ++r) {
            double s = 0.0;
            for (int q = 0; q < c.roww; ++q) {
                const double d = st.dt * c.v[k][c.roww * r + q];
                s += d * d;
            }
            maxrow = std::max(maxrow, std::sqrt(s));
        }
    }
    const double scale = (maxrow > maxstep) ? maxstep / maxrow : 1.0;
    for (int k = 1; k <= M - 2; ++k)
        for (int i = 0; i < c.dim; ++i) c.X[k][i] += scale * (st.dt * c.v[k][i]);
}

}  // namespace orc

// One FIRE move of a band of M images (the endpoints, images 0 and M-1, stay fixed)
// from the NEB forces F: the same routine the band step uses, exposed for pinning.
extern "C" int orc_fire_step(int M, int dim, int roww, double* X, double* v, const double* F,
                             orc_fire_state* st, double dtmax, double maxstep, int nmin, double finc,
                             double fdec, double astart, double fa)
{
    if (M < 3 || dim <= 0 || roww <= 0 || dim % roww != 0) return ORC_EINVAL;
    orc::NebCore c;
    c.M = M;
    c.dim = dim;
    c.roww = roww;
    c.X.assign(M, std::vector<double>(dim));
    c.v.assign(M, std::vector<double>(dim));
    c.Fneb.assign(M, std::vector<double>(dim));
    for (int k = 0; k < M; ++k)
        for (int i = 0; i < dim; ++i) {
            c.X[k][i] = X[size_t(k) * dim + i];
            c.v[k][i] = v[size_t(k) * dim + i];
            c.Fneb[k][i] = F[size_t(k) * dim + i];
        }
    c.fire = {st->dt, st->alpha, st->n_pos, st->fresh};
    orc::fire_move(c, dtmax, maxstep, nmin, finc, fdec, astart, fa);
    for (int k = 0; k < M; ++k)
        for (int i = 0; i < dim; ++i) {
            X[size_t(k) * dim + i] = c.X[k][i];
            v[size_t(k) * dim + i] = c.v[k][i];
        }
    st->dt = c.fire.dt;
    st->alpha = c.fire.alpha;
    st->n_pos = c.fire.n_pos;
    st->fresh = c.fire.fresh;
    return ORC_OK;
}

namespace orc {

// ---- exact integer spacings for the refine decision ------------------------
using u128 = unsigned __int128;

struct U256 {  // little-endian 64-bit limbs
    uint64_t w[4] = {0, 0, 0, 0};
};

U256 u256_from(u128 x)
{
    U256 r;
    r.w[0] = uint64_t(x);
    r.w[1] = uint64_t(x >> 64);
    return r;
}

U256 u256_add(const U256& a, const U256& b)
{
    U256 r;
    u128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        const u128 s = u128(a.w[i]) + b.w[i] + carry;
        r.w[i] = uint64_t(s);
        carry = s >> 64;
    }
    return r;
}

U256 u256_mul_small(const U256& a, uint64_t m)
{
    U256 r;
    u128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        const u128 p = u128(a.w[i]) * m + carry;
        r.w[i] = uint64_t(p);
        carry = p >> 64;
    }
    return r;
}

int u256_cmp(const U256& a, const U256& b)
{
    for (int i = 3; i >= 0; --i) {
        if (a.w[i] < b.w[i]) return -1;
        if (a.w[i] > b.w[i]) return 1;
    }
    return 0;
}

// floor(t * 2^64) for 0 <= t < 2^40; the conversion is exact.
bool fixed_point(double t, u128* out)
{
    if (!(t >= 0.0) || !(t < 0x1p40)) return false;
    *out = u128(t * 0x1p64);
    return true;
}

}  // namespace orc

extern "C" int orc_refine_decide(int M, int dim, const double* X, int ci, int max_images,
                                 int min_images, int ins_num, int ins_den, int del_num, int del_den,
                                 int* inserted_at, int* deleted_at, double* d2_report)
{
    using namespace orc;
    *inserted_at = -1;
    *deleted_at = -1;
    if (M < 2) return ORC_EINVAL;
    std::vector<u128> d2(M - 1, 0);
    U256 total;
    for (int k = 0; k + 1 < M; ++k) {
        u128 s = 0;
        for (int i = 0; i < dim; ++i) {
            const double diff = X[size_t(k + 1) * dim + i] - X[size_t(k) * dim + i];
            u128 q;
            if (!fixed_point(diff * diff, &q)) return ORC_ERANGE;
            s += q;
        }
        d2[k] = s;
        total = u256_add(total, u256_from(s));
        if (d2_report) d2_report[k] = double(s) * 0x1p-64;
    }
    int kstar = 0;
    for (int k = 1; k + 1 < M; ++k)
        if (d2[k] > d2[kstar]) kstar = k;
    if (M < max_images) {
        const U256 lhs = u256_mul_small(u256_from(d2[kstar]), uint64_t(ins_den) * uint64_t(M - 1));
        const U256 rhs = u256_mul_small(total, uint64_t(ins_num));
        if (u256_cmp(lhs, rhs) > 0) {
            *inserted_at = kstar + 1;
            return ORC_OK;
        }
    }
    if (M > min_images) {
        int jstar = -1;
        u128 best = 0;
        for (int j = 1; j <= M - 2; ++j) {
            if (j == ci) continue;
            const u128 m = std::max(d2[j - 1], d2[j]);
            if (jstar < 0 || m < best) {
                jstar = j;
                best = m;
            }
        }
        if (jstar >= 0) {
            const U256 lhs = u256_mul_small(u256_from(best), uint64_t(del_den) * uint64_t(M - 1));
            const U256 rhs = u256_mul_small(total, uint64_t(del_num));
            if (u256_cmp(lhs, rhs) < 0) *deleted_at = jstar;
        }
    }
    return ORC_OK;
}

// ---------------------------------------------------------------------------
// atomistic band
struct orc_band {
    orc_params p;
    int n = 0;
    double h0[9];
    orc::NebCore c;
    // per image, from its last evaluation
    std::vector<double> E;
    std::vector<std::vector<double>> V, F, R, h;
};

namespace {

int eval_image(orc_band* b, int k)
{
    const int n = b->n;
    b->c.Fg[k].assign(3 * size_t(n + 3), 0.0);
    b->F[k].assign(3 * size_t(n), 0.0);
    b->R[k].assign(3 * size_t(n), 0.0);
    b->V[k].assign(9, 0.0);
    b->h[k].assign(9, 0.0);
    return orc_cf_eval(&b->p, n, b->h0, b->c.X[k].data(), &b->c.H[k], &b->E[k], b->c.Fg[k].data(),
                       b->V[k].data(), b->F[k].data(), b->R[k].data(), b->h[k].data());
}

int eval_range(orc_band* b, int k0, int k1)
{
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : err)
    for (int k = k0; k <= k1; ++k) {
        const int rc = eval_image(b, k);
        err = std::min(err, rc);
    }
    return err;
}

void resize_images(orc_band* b, int M)
{
    auto& c = b->c;
    c.M = M;
    c.X.resize(M);
    c.v.resize(M);
    c.Fg.resize(M);
    c.Fneb.resize(M);
    c.H.resize(M);
    b->E.resize(M);
    b->V.resize(M);
    b->F.resize(M);
    b->R.resize(M);
    b->h.resize(M);
}

template <class T>
void insert_at(std::vector<T>& v, int k, const T& val) { v.insert(v.begin() + k, val); }
template <class T>
void erase_at(std::vector<T>& v, int k) { v.erase(v.begin() + k); }

int apply_refine(orc_band* b, int* ins, int* del)
{
    auto& c = b->c;
    const int M = c.M;
    std::vector<double> flat(size_t(M) * c.dim);
    for (int k = 0; k < M; ++k) std::memcpy(&flat[size_t(k) * c.dim], c.X[k].data(), sizeof(double) * c.dim);
    const int rc = orc_refine_decide(M, c.dim, flat.data(), c.ci, b->p.max_images, b->p.min_images,
                                     b->p.ins_num, b->p.ins_den, b->p.del_num, b->p.del_den, ins, del,
                                     nullptr);
    if (rc != ORC_OK) return rc;
    if (*ins >= 0) {
        const int k = *ins - 1;
        std::vector<double> mid(c.dim);
        for (int i = 0; i < c.dim; ++i) mid[i] = c.X[k][i] + 0.5 * (c.X[k + 1][i] - c.X[k][i]);
        insert_at(c.X, *ins, mid);
        insert_at(c.v, *ins, std::vector<double>(c.dim, 0.0));
        insert_at(c.Fg, *ins, std::vector<double>(c.dim, 0.0));
        insert_at(c.Fneb, *ins, std::vector<double>(c.dim, 0.0));
        // the new image is evaluated at the next step; until then it reports the
        // mean of its neighbours' enthalpies
        insert_at(c.H, *ins, 0.5 * (c.H[k] + c.H[k + 1]));
        insert_at(b->E, *ins, 0.5 * (b->E[k] + b->E[k + 1]));
        insert_at(b->V, *ins, std::vector<double>(9, 0.0));
        insert_at(b->F, *ins, std::vector<double>());
        insert_at(b->R, *ins, std::vector<double>());
        insert_at(b->h, *ins, std::vector<double>());
        c.M += 1;
    } else if (*del >= 0) {
        const int k = *del;
        erase_at(c.X, k);
        erase_at(c.v, k);
        erase_at(c.Fg, k);
        erase_at(c.Fneb, k);
        erase_at(c.H, k);
        erase_at(b->E, k);
        erase_at(b->V, k);
        erase_at(b->F, k);
        erase_at(b->R, k);
        erase_at(b->h, k);
        c.M -= 1;
    }
    if (*ins >= 0 || *del >= 0) {
        for (auto& vk : c.v) std::fill(vk.begin(), vk.end(), 0.0);
        c.fire.alpha = b->p.fire_astart;
        c.fire.n_pos = 0;
        c.fire.fresh = 1;
        c.ci = -1;
    }
    return ORC_OK;
}

}  // namespace

extern "C" orc_band* orc_band_create(const orc_params* p, int n, const int32_t* /*types*/,
                                     const double* pos_init, const double* cell_init,
                                     const double* pos_final, const double* cell_final, int* err)
{
    *err = ORC_EINVAL;
    if (n < 1 || p->n_images < 3 || p->max_images < p->n_images) return nullptr;
    if (p->potential != ORC_LJ && p->potential != ORC_TERSOFF) return nullptr;
    if (p->cell_filter < 0 || p->cell_filter > 2) return nullptr;
    auto* b = new orc_band();
    b->p = *p;
    b->n = n;
    for (int k = 0; k < 9; ++k) b->h0[k] = cell_init[k];
    const int M = p->n_images;
    auto& c = b->c;
    c.dim = 3 * (n + 3);
    c.roww = 3;
    c.natoms = n;
    resize_images(b, M);
    std::vector<double> XA(c.dim), XB(c.dim);
    *err = orc_build_endpoints(p, n, pos_init, cell_init, pos_final, cell_final, XA.data(), XB.data());
    if (*err != ORC_OK) {
        delete b;
        return nullptr;
    }
    for (int k = 0; k < M; ++k) {
        c.X[k].resize(c.dim);
        c.v[k].assign(c.dim, 0.0);
        const double t = double(k) / double(M - 1);
        for (int i = 0; i < c.dim; ++i) {
            if (k == 0)
                c.X[k][i] = XA[i];
            else if (k == M - 1)
                c.X[k][i] = XB[i];
            else
                c.X[k][i] = XA[i] + t * (XB[i] - XA[i]);
        }
    }
    c.fire = {p->fire_dt0, p->fire_astart, 0, 1};
    c.step = 0;
    c.ci = -1;
    *err = eval_range(b, 0, M - 1);
    if (*err != ORC_OK) {
        delete b;
        return nullptr;
    }
    return b;
}

extern "C" int orc_band_step(orc_band* b, int max_steps, double f_tol, int* steps_done,
                             double* fmax, int* converged)
{
    auto& c = b->c;
    const auto& p = b->p;
    *steps_done = 0;
    *converged = 0;
    *fmax = 0.0;
    for (int s = 0; s < max_steps; ++s) {
        const int rc = eval_range(b, 1, c.M - 2);
        if (rc != ORC_OK) return rc;
        orc::neb_forces(c, p.k_spring, p.climb_after);
        *fmax = orc::fmax_of(c);
        if (!std::isfinite(*fmax)) return ORC_ENONFINITE;
        if (*fmax < f_tol) {
            *converged = 1;
            return ORC_OK;
        }
        orc::fire_move(c, p.fire_dtmax, p.fire_maxstep, p.fire_nmin, p.fire_finc, p.fire_fdec,
                       p.fire_astart, p.fire_fa);
        c.step += 1;
        *steps_done += 1;
        if (p.refine_every > 0 && c.step % p.refine_every == 0) {
            int ins, del;
            const int r2 = apply_refine(b, &ins, &del);
            if (r2 != ORC_OK) return r2;
        }
    }
    return ORC_OK;
}

extern "C" int orc_band_refine(orc_band* b, int* inserted_at, int* deleted_at)
{
    return apply_refine(b, inserted_at, deleted_at);
}

extern "C" int orc_band_n_images(const orc_band* b) { return b->c.M; }

extern "C" int orc_band_energies(const orc_band* b, double* H, int cap, int* n_images,
                                 double* barrier, int* ci_index, double* path_coord)
{
    const auto& c = b->c;
    *n_images = c.M;
    if (cap < c.M) return ORC_EINVAL;
    double hmax = c.H[0];
    for (int k = 0; k < c.M; ++k) {
        H[k] = c.H[k];
        hmax = std::max(hmax, c.H[k]);
    }
    *barrier = hmax - c.H[0];
    *ci_index = c.ci;
    if (path_coord) {
        std::vector<double> X(size_t(c.M) * c.dim);
        for (int k = 0; k < c.M; ++k) std::copy(c.X[k].begin(), c.X[k].end(), X.begin() + size_t(k) * c.dim);
        orc_path_coord(c.M, c.natoms, c.dim, X.data(), path_coord);
    }
    return ORC_OK;
}

extern "C" int orc_band_get_state(const orc_band* b, double* X, double* v, int cap_images,
                                  orc_fire_state* st, double* h0)
{
    const auto& c = b->c;
    if (cap_images < c.M) return ORC_EINVAL;
    for (int k = 0; k < c.M; ++k) {
        if (X) std::memcpy(X + size_t(k) * c.dim, c.X[k].data(), sizeof(double) * c.dim);
        if (v) std::memcpy(v + size_t(k) * c.dim, c.v[k].data(), sizeof(double) * c.dim);
    }
    if (st) {
        st->dt = c.fire.dt;
        st->alpha = c.fire.alpha;
        st->n_pos = c.fire.n_pos;
        st->fresh = c.fire.fresh;
        st->step = c.step;
        st->ci = c.ci;
    }
    if (h0)
        for (int k = 0; k < 9; ++k) h0[k] = b->h0[k];
    return ORC_OK;
}

extern "C" int orc_band_set_state(orc_band* b, int n_images, const double* X, const double* v,
                                  const orc_fire_state* st)
{
    auto& c = b->c;
    if (n_images < 3 || n_images > b->p.max_images) return ORC_EINVAL;
    resize_images(b, n_images);
    for (int k = 0; k < n_images; ++k) {
        c.X[k].assign(X + size_t(k) * c.dim, X + size_t(k + 1) * c.dim);
        if (v)
            c.v[k].assign(v + size_t(k) * c.dim, v + size_t(k + 1) * c.dim);
        else
            c.v[k].assign(c.dim, 0.0);
    }
    std::fill(c.v.front().begin(), c.v.front().end(), 0.0);
    std::fill(c.v.back().begin(), c.v.back().end(), 0.0);
    c.fire.dt = st->dt;
    c.fire.alpha = st->alpha;
    c.fire.n_pos = st->n_pos;
    c.fire.fresh = st->fresh;
    c.step = st->step;
    c.ci = st->ci;
    // endpoints may have changed with the state: evaluate every image again
    return eval_range(b, 0, n_images - 1);
}

extern "C" int orc_band_image(const orc_band* b, int k, double* E, double* H, double* V, double* F,
                              double* Fg, double* Fneb, double* R, double* h)
{
    const auto& c = b->c;
    if (k < 0 || k >= c.M) return ORC_EINVAL;
    const int n = b->n;
    if (E) *E = b->E[k];
    if (H) *H = c.H[k];
    if (V)
        for (int i = 0; i < 9; ++i) V[i] = b->V[k].size() == 9 ? b->V[k][i] : 0.0;
    auto cp = [](double* dst, const std::vector<double>& src, size_t len) {
        if (!dst) return;
        for (size_t i = 0; i < len; ++i) dst[i] = i < src.size() ? src[i] : 0.0;
    };
    cp(F, b->F[k], 3 * size_t(n));
    cp(Fg, c.Fg[k], 3 * size_t(n + 3));
    cp(Fneb, c.Fneb.size() > size_t(k) ? c.Fneb[k] : std::vector<double>(), 3 * size_t(n + 3));
    cp(R, b->R[k], 3 * size_t(n));
    cp(h, b->h[k], 9);
    return ORC_OK;
}

extern "C" void orc_band_destroy(orc_band* b) { delete b; }

// Threads of the image loop (the band's images are evaluated in parallel; each image
// is sequential, so results do not depend on the count).
extern "C" void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
extern "C" int orc_max_threads(void) { return omp_get_max_threads(); }

// Energy profile of the band at its current coordinates: every image is evaluated
// afresh, then the Hermite interpolant of H over the path coordinate is sampled at
// n_samples evenly spaced normalized coordinates and its maximum is located.
extern "C" int orc_band_profile(orc_band* b, int n_samples, double* s, double* H, double* slope,
                                double* samples, double* barrier, double* xi_max)
{
    auto& c = b->c;
    const int M = c.M;
    if (n_samples < 0 || n_samples == 1) return ORC_EINVAL;
    int rc = eval_range(b, 0, M - 1);
    if (rc != ORC_OK) return rc;
    std::vector<double> X(size_t(M) * c.dim), Fg(size_t(M) * c.dim);
    for (int k = 0; k < M; ++k) {
        std::copy(c.X[k].begin(), c.X[k].end(), X.begin() + size_t(k) * c.dim);
        std::copy(c.Fg[k].begin(), c.Fg[k].end(), Fg.begin() + size_t(k) * c.dim);
        H[k] = c.H[k];
    }
    rc = orc_profile(M, b->n, c.dim, X.data(), H, Fg.data(), s, slope);
    if (rc != ORC_OK) return rc;
    const double S = s[M - 1];
    std::vector<double> sq(n_samples);
    for (int j = 0; j < n_samples; ++j) sq[j] = double(j) / double(n_samples - 1) * S;
    if (n_samples > 0) orc_spline_eval(M, s, H, slope, n_samples, sq.data(), samples);
    double hmax, at;
    orc_spline_max(M, s, H, slope, &hmax, &at);
    *barrier = hmax - H[0];
    *xi_max = S > 0.0 ? at / S : 0.0;
    return ORC_OK;
}

// ---------------------------------------------------------------------------
// analytic two-dimensional surface, through the same NEB and FIRE code
extern "C" int orc_neb2d(double kappa, int M, double* xy, double k_spring, int climb_after,
                         double dt0, double dtmax, double maxstep, int max_steps, double f_tol,
                         double* energies, int* ci, double* fmax)
{
    orc::NebCore c;
    c.M = M;
    c.dim = 2;
    c.roww = 2;
    c.X.assign(M, std::vector<double>(2));
    c.v.assign(M, std::vector<double>(2, 0.0));
    c.Fg.assign(M, std::vector<double>(2, 0.0));
    c.H.assign(M, 0.0);
    for (int k = 0; k < M; ++k) {
        c.X[k][0] = xy[2 * k];
        c.X[k][1] = xy[2 * k + 1];
    }
    auto eval = [&](int k) {
        const double x = c.X[k][0], y = c.X[k][1];
        const double a = 1.0 - x * x, q = y - x * x;
        c.H[k] = a * a + kappa * q * q;
        c.Fg[k][0] = 4.0 * x * a + 4.0 * kappa * x * q;  // -dV/dx
        c.Fg[k][1] = -2.0 * kappa * q;                    // -dV/dy
    };
    c.fire = {dt0, 0.1, 0, 1};
    for (int k = 0; k < M; ++k) eval(k);
    int s = 0;
    *fmax = 0.0;
    for (; s < max_steps; ++s) {
        for (int k = 1; k <= M - 2; ++k) eval(k);
        orc::neb_forces(c, k_spring, climb_after);
        *fmax = orc::fmax_of(c);
        if (*fmax < f_tol) break;
        orc::fire_move(c, dtmax, maxstep, 5, 1.1, 0.5, 0.1, 0.99);
        c.step += 1;
    }
    for (int k = 0; k < M; ++k) {
        xy[2 * k] = c.X[k][0];
        xy[2 * k + 1] = c.X[k][1];
        energies[k] = c.H[k];
    }
    *ci = c.ci;
    return s;
}

// ---------------------------------------------------------------------------
// single-image relaxation through the cell filter (used to make relaxed endpoints)
extern "C" int orc_relax(const orc_params* p, int n, double* R, double* h, int max_steps,
                         double f_tol, int* steps_done, double* fmax)
{
    orc::NebCore c;  // three "images": fixed copies around the one that moves
    c.M = 3;
    c.dim = 3 * (n + 3);
    c.roww = 3;
    c.natoms = n;
    double h0[9];
    for (int k = 0; k < 9; ++k) h0[k] = h[k];
    const double cf = orc::cell_factor_of(p, n, h0);
    c.X.assign(3, std::vector<double>(c.dim, 0.0));
    c.v.assign(3, std::vector<double>(c.dim, 0.0));
    c.Fneb.assign(3, std::vector<double>(c.dim, 0.0));
    for (int i = 0; i < 3 * n; ++i) c.X[1][i] = R[i];
    for (int k = 0; k < 9; ++k) c.X[1][3 * n + k] = (k % 4 == 0) ? cf : 0.0;
    c.fire = {p->fire_dt0, p->fire_astart, 0, 1};
    std::vector<double> Fg(c.dim);
    double H, E, V[9];
    *steps_done = 0;
    for (int s = 0; s < max_steps; ++s) {
        const int rc = orc_cf_eval(p, n, h0, c.X[1].data(), &H, &E, Fg.data(), V, nullptr, nullptr, nullptr);
        if (rc != ORC_OK) return rc;
        c.Fneb[1] = Fg;
        orc::remove_translation(c.Fneb[1], n);
        *fmax = orc::fmax_of(c);
        if (*fmax < f_tol) break;
        orc::fire_move(c, p->fire_dtmax, p->fire_maxstep, p->fire_nmin, p->fire_finc, p->fire_fdec,
                       p->fire_astart, p->fire_fa);
        *steps_done += 1;
    }
    double B[9], D[9];
    for (int k = 0; k < 9; ++k) B[k] = c.X[1][3 * n + k] / cf;
    if (orc::cell_gauge(p, B, D) != ORC_OK) return ORC_ECELL;
    orc::rows_times(n, c.X[1].data(), D, R);
    orc::matmul3(h0, D, h);
    return ORC_OK;
}
