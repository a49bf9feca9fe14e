// Oracle (test infrastructure only): the rotation-free cell filter (Sec. II.C).
//
// Generalized coordinates of one image (Eqs. (10), (11), (17)):
//     X = (R~_1 .. R~_n, c_f B),   R~ = R D^-1,   D = h0^-1 h,   B = D D^T
// The rotational gauge is fixed by D = symsqrt(B), so h = h0 D and R = R~ D.
// Generalized forces (Eqs. (12), (14), (16), (17)):
//     atoms:   F D^T
//     lattice: D^-T V_eff D^-1 / c_f     (V_eff = V - P Omega I, enthalpy H = U + P Omega)
// c_f is the cell factor (default: |det h0|^(1/3) n^(1/6), cell_factor_of).  The lattice force is the
// printed expression; the exact virtual-work conjugate of B is half of it, a
// factor that changes the path metric but no fixed point.
#include "internal.h"

#include <cmath>
#include <vector>

namespace {
constexpr double kEvPerA3InGPa = 160.21766208;
}

double orc::cell_factor_of(const orc_params* p, int n, const double* h0)
{
    if (p->cell_factor > 0.0) return p->cell_factor;
    return std::cbrt(std::fabs(orc_det3(h0))) * std::pow(double(n), 1.0 / 6.0);
}

int orc::cell_gauge(const orc_params* p, const double* C, double* D)
{
    if (p->cell_filter == 1) {
        for (int k = 0; k < 9; ++k) D[k] = C[k];
        const double det = orc_det3(D);
        return (det > 0.0 && std::isfinite(det)) ? ORC_OK : ORC_ECELL;
    }
    return orc_symsqrt(C, D);
}

extern "C" int orc_cf_eval(const orc_params* p, int n, const double* h0, const double* X,
                           double* H, double* E, double* Fg, double* V,
                           double* Fout, double* Rout, double* hout)
{
    const double cf = orc::cell_factor_of(p, n, h0);
    double B[9], D[9], h[9], Dinv[9], DinvT[9];
    for (int k = 0; k < 9; ++k) B[k] = X[3 * n + k] / cf;
    int rc = orc::cell_gauge(p, B, D);
    if (rc != ORC_OK) return rc;
    orc::matmul3(h0, D, h);
    std::vector<double> R(3 * size_t(n)), F(3 * size_t(n));
    orc::rows_times(n, X, D, R.data());

    std::vector<std::vector<orc::Nbr>> lists;
    rc = orc::build_lists(n, R.data(), h, orc::cutoff_of(p), n <= 16, lists);
    if (rc != ORC_OK) return rc;
    double e = 0.0, vir[9];
    rc = orc::eval_with_lists(p, n, R.data(), h, lists, &e, nullptr, F.data(), vir);
    if (rc != ORC_OK) return rc;

    const double P = p->pressure_GPa / kEvPerA3InGPa;
    const double omega = std::fabs(orc_det3(h));
    *E = e;
    *H = e + P * omega;
    for (int k = 0; k < 9; ++k) V[k] = vir[k];

    // Applied stress beyond the pressure: a second Piola-Kirchhoff stress S referred
    // to h0 does the work Omega0 S : E on the Green-Lagrange strain E = (D D^T - I)/2
    // (D maps reference rows to current rows, so lengths go with D D^T).  Its change
    // under dD is Omega0 tr(S D dD^T), the same as that of a virial Omega0 D^T S D
    // under the strain D^-1 dD, so it enters both filters through the virial.
    double S[9];
    const int voigt[9] = {0, 5, 4, 5, 1, 3, 4, 3, 2};
    for (int k = 0; k < 9; ++k) S[k] = p->stress_GPa[voigt[k]] / kEvPerA3InGPa;
    const double omega0 = std::fabs(orc_det3(h0));
    double DT0[9], DDT[9], SD[9], DTSD[9];
    orc::transpose3(D, DT0);
    orc::matmul3(D, DT0, DDT);
    orc::matmul3(S, D, SD);
    orc::matmul3(DT0, SD, DTSD);
    double SE = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) SE += S[3 * r + c] * 0.5 * (DDT[3 * r + c] - (r == c ? 1.0 : 0.0));
    *H -= omega0 * SE;
    double Vs[9];
    for (int k = 0; k < 9; ++k) Vs[k] = vir[k] + omega0 * DTSD[k];

    // atoms: F D^T
    double DT[9];
    orc::transpose3(D, DT);
    orc::rows_times(n, F.data(), DT, Fg);
    // lattice
    if (p->cell_filter == 2) {
        double Veff[9];
        for (int k = 0; k < 9; ++k) Veff[k] = Vs[k];
        for (int k = 0; k < 3; ++k) Veff[4 * k] -= P * omega;
        orc_inv3(D, Dinv);
        orc::transpose3(Dinv, DinvT);
        double T1[9], G[9];
        orc::matmul3(DinvT, Veff, T1);
        orc::matmul3(T1, Dinv, G);
        // B is symmetric (six coordinates), so its conjugate force is the symmetric
        // part of D^-T V D^-1; V itself is symmetric only up to rounding
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                Fg[3 * n + 3 * r + c] = p->b_force_scale * (0.5 * (G[3 * r + c] + G[3 * c + r])) / cf;
    } else if (p->cell_filter == 1) {
        // D-variant (Sec. II.C, Eq. (13)): coordinates D, conjugate force D^-T V
        double Veff[9];
        for (int k = 0; k < 9; ++k) Veff[k] = Vs[k];
        for (int k = 0; k < 3; ++k) Veff[4 * k] -= P * omega;
        orc_inv3(D, Dinv);
        orc::transpose3(Dinv, DinvT);
        double G[9];
        orc::matmul3(DinvT, Veff, G);
        for (int k = 0; k < 9; ++k) Fg[3 * n + k] = G[k] / cf;
    } else {
        for (int k = 0; k < 9; ++k) Fg[3 * n + k] = 0.0;
    }
    bool finite = std::isfinite(*H);
    for (int k = 0; k < 3 * (n + 3); ++k) finite = finite && std::isfinite(Fg[k]);
    if (Fout)
        for (int k = 0; k < 3 * n; ++k) Fout[k] = F[k];
    if (Rout)
        for (int k = 0; k < 3 * n; ++k) Rout[k] = R[k];
    if (hout)
        for (int k = 0; k < 9; ++k) hout[k] = h[k];
    return finite ? ORC_OK : ORC_ENONFINITE;
}

extern "C" int orc_build_endpoints(const orc_params* p, int n, const double* RA, const double* hA,
                                   const double* RB, const double* hB, double* XA, double* XB)
{
    const double* h0 = hA;
    const double cf = orc::cell_factor_of(p, n, h0);
    if (!(std::fabs(orc_det3(hA)) > 0.0) || !(std::fabs(orc_det3(hB)) > 0.0)) return ORC_ECELL;
    double h0inv[9], hBinv[9], Draw[9], DrawT[9], BB[9];
    orc_inv3(h0, h0inv);
    orc_inv3(hB, hBinv);
    orc::matmul3(h0inv, hB, Draw);
    orc::transpose3(Draw, DrawT);
    orc::matmul3(Draw, DrawT, BB);

    std::vector<double> sA(3 * size_t(n)), sB(3 * size_t(n));
    orc::rows_times(n, RA, h0inv, sA.data());
    orc::rows_times(n, RB, hBinv, sB.data());
    for (int i = 0; i < n; ++i) {
        double ds[3];
        for (int k = 0; k < 3; ++k) {
            ds[k] = sB[3 * i + k] - sA[3 * i + k];
            ds[k] -= std::nearbyint(ds[k]);
        }
        for (int c = 0; c < 3; ++c) {
            XA[3 * i + c] = RA[3 * i + c];
            XB[3 * i + c] = RA[3 * i + c] + (ds[0] * h0[c] + ds[1] * h0[3 + c] + ds[2] * h0[6 + c]);
        }
    }
    for (int k = 0; k < 9; ++k) {
        XA[3 * n + k] = (k % 4 == 0) ? cf : 0.0;
        // D-variant: the deformation gradient itself; rotation-free: B = D D^T
        XB[3 * n + k] = cf * (p->cell_filter == 1 ? Draw[k] : BB[k]);
    }
    return ORC_OK;
}
