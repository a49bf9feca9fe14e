// Oracle (test infrastructure only): short-range potentials, forces and virial in FP64.
//
// Both potentials are written as per-atom energies U_i of the displacements
// r^{ij} = R_j - R_i (+ lattice shift) to i's neighbours (Sec. II.B, Eq. (4)).
// For every neighbour entry e = (j, n) of atom i the oracle computes
//     P_e = dU_i / dr^{ij}
// and assembles
//     F_i  = sum_e P_e  - sum_{entries e' of other atoms that point at i} P_e'
//          = sum_j f^{ij},  f^{ij} = dU_i/dr^{ij} - dU_j/dr^{ji}
//            (the form used in the derivation of Eq. (6); the printed Eq. (5)
//             has the indices of the two terms swapped),
//     V_mn = - sum_e r^{ij}_m P_e,n  = -1/2 sum_{ij} r^{ij}_m f^{ij}_n   (Eqs. (6)-(8)).
#include "internal.h"

#include <cmath>

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Bond {
    double d[3];
    double r;
};

// Shifted Lennard-Jones: phi(r) = 4 eps [(s/r)^12 - (s/r)^6] - phi_rc (if shifted).
// U_i = 1/2 sum_j phi(r_ij), so P_e = 1/2 phi'(r) d / r.
void lj_atom(const orc_params* p, const std::vector<Bond>& b, double* ui, std::vector<double>& P)
{
    const double s2 = p->lj_sigma * p->lj_sigma;
    double shift = 0.0;
    if (p->lj_shift) {
        const double q = s2 / (p->lj_rc * p->lj_rc);
        const double q3 = q * q * q;
        shift = 4.0 * p->lj_eps * (q3 * q3 - q3);
    }
    double u = 0.0;
    P.assign(3 * b.size(), 0.0);
    for (size_t e = 0; e < b.size(); ++e) {
        const double r = b[e].r;
        const double q = s2 / (r * r);
        const double q3 = q * q * q;
        const double phi = 4.0 * p->lj_eps * (q3 * q3 - q3) - shift;
        const double dphi = 24.0 * p->lj_eps * (q3 - 2.0 * q3 * q3) / r;  // dphi/dr
        u += 0.5 * phi;
        for (int c = 0; c < 3; ++c) P[3 * e + c] = 0.5 * dphi * b[e].d[c] / r;
    }
    *ui = u;
}

// Tersoff bond-order form (lambda3 = 0):
//   U_i = 1/2 sum_j fc(r_ij) [A exp(-l1 r_ij) - b_ij B exp(-l2 r_ij)]
//   b_ij = (1 + beta^n zeta_ij^n)^(-1/(2n)),  zeta_ij = sum_{k != j} fc(r_ik) g(cos theta_ijk)
//   g(c) = 1 + c^2/d^2 - c^2/(d^2 + (h - cos)^2)
//   fc(r) = 1 (r < R), 1/2 + 1/2 cos(pi (r-R)/(S-R)) (R <= r < S), 0 (r >= S)
struct Tersoff {
    const orc_params* p;
    double fc(double r) const
    {
        if (r < p->ts_R) return 1.0;
        if (r >= p->ts_S) return 0.0;
        return 0.5 + 0.5 * std::cos(kPi * (r - p->ts_R) / (p->ts_S - p->ts_R));
    }
    double dfc(double r) const
    {
        if (r < p->ts_R || r >= p->ts_S) return 0.0;
        const double w = p->ts_S - p->ts_R;
        return -0.5 * kPi / w * std::sin(kPi * (r - p->ts_R) / w);
    }
    double g(double cs) const
    {
        const double c2 = p->ts_c * p->ts_c, d2 = p->ts_d * p->ts_d;
        const double t = p->ts_h - cs;
        return 1.0 + c2 / d2 - c2 / (d2 + t * t);
    }
    double dg(double cs) const  // dg / dcos
    {
        const double c2 = p->ts_c * p->ts_c, d2 = p->ts_d * p->ts_d;
        const double t = p->ts_h - cs;
        const double den = d2 + t * t;
        return -2.0 * c2 * t / (den * den);
    }
};

void tersoff_atom(const orc_params* p, const std::vector<Bond>& b, double* ui,
                  std::vector<double>& P)
{
    const Tersoff T{p};
    const size_t nb = b.size();
    std::vector<double> fc(nb), dfc(nb), fR(nb), fA(nb), cosm(nb * nb);
    for (size_t e = 0; e < nb; ++e) {
        fc[e] = T.fc(b[e].r);
        dfc[e] = T.dfc(b[e].r);
        fR[e] = p->ts_A * std::exp(-p->ts_lambda1 * b[e].r);
        fA[e] = p->ts_B * std::exp(-p->ts_lambda2 * b[e].r);
    }
    for (size_t e = 0; e < nb; ++e)
        for (size_t k = 0; k < nb; ++k) {
            const double dot = b[e].d[0] * b[k].d[0] + b[e].d[1] * b[k].d[1] + b[e].d[2] * b[k].d[2];
            cosm[e * nb + k] = dot / (b[e].r * b[k].r);
        }
    // zeta, b, db/dzeta per bond
    std::vector<double> bo(nb), dbo(nb);
    const double bn = std::pow(p->ts_beta, p->ts_n);
    for (size_t e = 0; e < nb; ++e) {
        double z = 0.0;
        for (size_t k = 0; k < nb; ++k)
            if (k != e) z += fc[k] * T.g(cosm[e * nb + k]);
        const double base = 1.0 + bn * std::pow(z, p->ts_n);
        bo[e] = std::pow(base, -1.0 / (2.0 * p->ts_n));
        dbo[e] = (z > 0.0)
                     ? -0.5 * bn * std::pow(z, p->ts_n - 1.0) * std::pow(base, -1.0 / (2.0 * p->ts_n) - 1.0)
                     : 0.0;
    }
    double u = 0.0;
    for (size_t e = 0; e < nb; ++e) u += 0.5 * fc[e] * (fR[e] - bo[e] * fA[e]);
    *ui = u;

    // P_e = dU_i/dd_e
    P.assign(3 * nb, 0.0);
    for (size_t e = 0; e < nb; ++e) {
        const double r = b[e].r;
        double hat[3];
        for (int c = 0; c < 3; ++c) hat[c] = b[e].d[c] / r;
        // direct radial term at fixed b_e
        const double dV = dfc[e] * (fR[e] - bo[e] * fA[e])
                        + fc[e] * (-p->ts_lambda1 * fR[e] + bo[e] * p->ts_lambda2 * fA[e]);
        double acc[3];
        for (int c = 0; c < 3; ++c) acc[c] = 0.5 * dV * hat[c];
        // bond-order terms: -1/2 sum_{e2} fc_e2 fA_e2 db_e2 dzeta_e2/dd_e
        const double pre_e = fc[e] * fA[e] * dbo[e];
        for (size_t k = 0; k < nb; ++k) {
            if (k == e) continue;
            const double cs = cosm[e * nb + k];
            double dcos[3];  // d cos(theta_{e,k}) / d d_e
            for (int c = 0; c < 3; ++c)
                dcos[c] = b[k].d[c] / (r * b[k].r) - cs * b[e].d[c] / (r * r);
            const double gk = T.g(cs), dgk = T.dg(cs);
            // zeta_e contains fc(r_k) g(cos_ek)
            for (int c = 0; c < 3; ++c) acc[c] -= 0.5 * pre_e * fc[k] * dgk * dcos[c];
            // zeta_k contains fc(r_e) g(cos_ke); cos_ke = cos_ek
            const double pre_k = fc[k] * fA[k] * dbo[k];
            for (int c = 0; c < 3; ++c)
                acc[c] -= 0.5 * pre_k * (dfc[e] * gk * hat[c] + fc[e] * dgk * dcos[c]);
        }
        for (int c = 0; c < 3; ++c) P[3 * e + c] = acc[c];
    }
}

}  // namespace

namespace orc {

double cutoff_of(const orc_params* p)
{
    return p->potential == ORC_LJ ? p->lj_rc : p->ts_S;
}

int eval_with_lists(const orc_params* p, int n, const double* R, const double* h,
                    const std::vector<std::vector<Nbr>>& lists,
                    double* E, double* u, double* F, double* V)
{
    if (p->potential != ORC_LJ && p->potential != ORC_TERSOFF) return ORC_EINVAL;
    for (int i = 0; i < 3 * n; ++i) F[i] = 0.0;
    for (int k = 0; k < 9; ++k) V[k] = 0.0;
    double etot = 0.0;
    std::vector<Bond> bonds;
    std::vector<double> P;
    for (int i = 0; i < n; ++i) {
        const auto& L = lists[i];
        bonds.resize(L.size());
        for (size_t e = 0; e < L.size(); ++e) {
            const int j = L[e].j;
            for (int c = 0; c < 3; ++c) {
                const double sh = (double(L[e].n[0]) * h[c] + double(L[e].n[1]) * h[3 + c])
                                + double(L[e].n[2]) * h[6 + c];
                bonds[e].d[c] = (R[3 * j + c] - R[3 * i + c]) + sh;
            }
            bonds[e].r = std::sqrt(bonds[e].d[0] * bonds[e].d[0] + bonds[e].d[1] * bonds[e].d[1]
                                   + bonds[e].d[2] * bonds[e].d[2]);
        }
        double ui = 0.0;
        if (p->potential == ORC_LJ)
            lj_atom(p, bonds, &ui, P);
        else
            tersoff_atom(p, bonds, &ui, P);
        if (u) u[i] = ui;
        etot += ui;
        for (size_t e = 0; e < L.size(); ++e) {
            const int j = L[e].j;
            for (int c = 0; c < 3; ++c) {
                F[3 * i + c] += P[3 * e + c];
                F[3 * j + c] -= P[3 * e + c];
            }
            for (int m = 0; m < 3; ++m)
                for (int c = 0; c < 3; ++c) V[3 * m + c] -= bonds[e].d[m] * P[3 * e + c];
        }
    }
    *E = etot;
    return ORC_OK;
}

}  // namespace orc

extern "C" int orc_eval(const orc_params* p, int n, const double* R, const double* h,
                        double* E, double* u, double* F, double* V)
{
    std::vector<std::vector<orc::Nbr>> lists;
    const int rc = orc::build_lists(n, R, h, orc::cutoff_of(p), n <= 64, lists);
    if (rc != ORC_OK) return rc;
    return orc::eval_with_lists(p, n, R, h, lists, E, u, F, V);
}
