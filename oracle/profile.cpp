// Oracle (test infrastructure only): energy profile of a band.
//
// The paper reports each transition as the enthalpy of the images against a
// normalized path coordinate (the energy panels of its Sec. III figures) and
// reads barriers off that curve.  Between images the curve here is the cubic
// Hermite interpolant whose slopes are the tangential true forces:
//
//   path coordinate   s_0 = 0,  s_{k+1} = s_k + |X_{k+1} - X_k|
//   slope             dH/ds at image k = -Fg_k . tau_k / |tau_k|
//   tangent           improved tangent of the band (cited in Sec. I) for the
//                     moving images, the one-sided difference at the two ends
//   interpolant       on [s_k, s_{k+1}], t = (s - s_k) / (s_{k+1} - s_k):
//                     H = h00(t) H_k + h10(t) d m_k + h01(t) H_{k+1} + h11(t) d m_{k+1}
//                     with h00 = 2t^3 - 3t^2 + 1, h10 = t^3 - 2t^2 + t,
//                     h01 = -2t^3 + 3t^2, h11 = t^3 - t^2 and d = s_{k+1} - s_k
//
// Image differences and forces are taken modulo a rigid translation of the atoms
// (atom-row means removed), the metric in which the band measures its tangent and
// springs.  The maximum of the interpolant is found from its nodes and the roots of
// its derivative in each interval.
#include "internal.h"

#include <cmath>
#include <vector>

namespace {

double dotv(const std::vector<double>& a, const std::vector<double>& b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// Hermite cubic of one interval at t in [0, 1].
double hermite(double H0, double H1, double m0, double m1, double d, double t)
{
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    const double h10 = t3 - 2.0 * t2 + t;
    const double h01 = -2.0 * t3 + 3.0 * t2;
    const double h11 = t3 - t2;
    return h00 * H0 + h10 * d * m0 + h01 * H1 + h11 * d * m1;
}

}  // namespace

namespace orc {

// Arc length along the band: s_0 = 0, s_{k+1} = s_k + |X_{k+1} - X_k| with the rigid
// translation of the first natoms rows removed from each difference.
void arc_lengths(int M, int natoms, int dim, const double* X, double* s)
{
    std::vector<double> d(dim);
    s[0] = 0.0;
    for (int k = 0; k + 1 < M; ++k) {
        for (int i = 0; i < dim; ++i) d[i] = X[size_t(k + 1) * dim + i] - X[size_t(k) * dim + i];
        remove_translation(d, natoms);
        s[k + 1] = s[k] + std::sqrt(dotv(d, d));
    }
}

}  // namespace orc

// Normalized path coordinate xi_k = s_k / s_{M-1}: the axis against which the
// transitions of Sec. III are drawn, in the same metric as the profile's arc length.
extern "C" int orc_path_coord(int M, int natoms, int dim, const double* X, double* xi)
{
    if (M < 2 || dim <= 0 || natoms < 0 || 3 * natoms > dim) return ORC_EINVAL;
    orc::arc_lengths(M, natoms, dim, X, xi);
    const double S = xi[M - 1];
    for (int k = 0; k < M; ++k) xi[k] = S > 0.0 ? xi[k] / S : 0.0;
    return ORC_OK;
}

extern "C" int orc_profile(int M, int natoms, int dim, const double* X, const double* H, const double* Fg,
                           double* s, double* slope)
{
    if (M < 2 || dim <= 0 || natoms < 0 || 3 * natoms > dim) return ORC_EINVAL;
    std::vector<double> tp(dim), tm(dim), tau(dim), F(dim);
    auto row = [&](int k) { return X + size_t(k) * dim; };
    orc::arc_lengths(M, natoms, dim, X, s);
    for (int k = 0; k < M; ++k) {
        for (int i = 0; i < dim; ++i) {
            tp[i] = k + 1 < M ? row(k + 1)[i] - row(k)[i] : 0.0;
            tm[i] = k > 0 ? row(k)[i] - row(k - 1)[i] : 0.0;
            F[i] = Fg[size_t(k) * dim + i];
        }
        orc::remove_translation(tp, natoms);
        orc::remove_translation(tm, natoms);
        orc::remove_translation(F, natoms);
        double a, b;
        if (k == 0) {
            a = 1.0;
            b = 0.0;
        } else if (k == M - 1) {
            a = 0.0;
            b = 1.0;
        } else {
            orc_tangent_coeffs(H[k - 1], H[k], H[k + 1], &a, &b);
        }
        for (int i = 0; i < dim; ++i) tau[i] = a * tp[i] + b * tm[i];
        const double nt = std::sqrt(dotv(tau, tau));
        slope[k] = nt > 0.0 ? -dotv(F, tau) / nt : 0.0;
    }
    return ORC_OK;
}

extern "C" int orc_spline_eval(int M, const double* s, const double* H, const double* slope, int nq,
                               const double* sq, double* out)
{
    if (M < 2 || nq < 0) return ORC_EINVAL;
    for (int q = 0; q < nq; ++q) {
        // the last interval whose left node is at or before the query
        int k = 0;
        for (int j = 0; j <= M - 2; ++j)
            if (s[j] <= sq[q]) k = j;
        const double d = s[k + 1] - s[k];
        double t = d > 0.0 ? (sq[q] - s[k]) / d : 0.0;
        t = std::fmin(std::fmax(t, 0.0), 1.0);
        out[q] = hermite(H[k], H[k + 1], slope[k], slope[k + 1], d, t);
    }
    return ORC_OK;
}

extern "C" int orc_spline_max(int M, const double* s, const double* H, const double* slope, double* Hmax,
                              double* s_at)
{
    if (M < 2) return ORC_EINVAL;
    double best = H[0], where = s[0];
    auto consider = [&](double v, double at) {
        if (v > best) {
            best = v;
            where = at;
        }
    };
    for (int k = 0; k + 1 < M; ++k) {
        const double d = s[k + 1] - s[k];
        consider(H[k + 1], s[k + 1]);
        if (!(d > 0.0)) continue;
        const double m0 = d * slope[k], m1 = d * slope[k + 1];
        // derivative of the interval's cubic in t: A t^2 + B t + C
        const double A = 6.0 * H[k] + 3.0 * m0 - 6.0 * H[k + 1] + 3.0 * m1;
        const double B = -6.0 * H[k] - 4.0 * m0 + 6.0 * H[k + 1] - 2.0 * m1;
        const double C = m0;
        double roots[2];
        int nr = 0;
        if (A == 0.0) {
            if (B != 0.0) roots[nr++] = -C / B;
        } else {
            const double disc = B * B - 4.0 * A * C;
            if (disc >= 0.0) {
                const double r = std::sqrt(disc);
                roots[nr++] = (-B + r) / (2.0 * A);
                roots[nr++] = (-B - r) / (2.0 * A);
            }
        }
        for (int q = 0; q < nr; ++q)
            if (roots[q] > 0.0 && roots[q] < 1.0)
                consider(hermite(H[k], H[k + 1], slope[k], slope[k + 1], d, roots[q]), s[k] + roots[q] * d);
    }
    *Hmax = best;
    *s_at = where;
    return ORC_OK;
}
