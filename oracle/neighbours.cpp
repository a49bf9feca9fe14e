// Oracle (test infrastructure only): full neighbour sets under periodic boundaries.
//
// Definition: the neighbours of atom i are every (j, n), n in Z^3, (j, n) != (i, 0),
// whose displacement
//     r = (R_j - R_i) + ((n0 h_0 + n1 h_1) + n2 h_2)
// satisfies (r_x r_x + r_y r_y) + r_z r_z < rc*rc, every operation rounded on
// its own (compiled with -ffp-contract=off).  R is unwrapped.  This is the
// "n_i neighbours in i's local environment under PBC" of Sec. II.B, Eq. (4),
// with the cutoff of the short-range potential.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <tuple>

namespace {

bool within(const double* Ri, const double* Rj, const double* h, int n0, int n1, int n2,
            double rc2)
{
    double d[3];
    for (int c = 0; c < 3; ++c) {
        const double sh = (double(n0) * h[c] + double(n1) * h[3 + c]) + double(n2) * h[6 + c];
        d[c] = (Rj[c] - Ri[c]) + sh;
    }
    const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return r2 < rc2;
}

bool nbr_less(const orc::Nbr& a, const orc::Nbr& b)
{
    return std::tie(a.j, a.n[0], a.n[1], a.n[2]) < std::tie(b.j, b.n[0], b.n[1], b.n[2]);
}

void fractional(int n, const double* R, const double* h, std::vector<double>& s)
{
    double hinv[9];
    orc_inv3(h, hinv);
    s.resize(3 * size_t(n));
    orc::rows_times(n, R, hinv, s.data());
}

// O(N^2) brute force: every j, and every n in a box around the nearest image that
// is wide enough to hold all of |(ds + n) . w| < rc.
void brute(int n, const double* R, const double* h, double rc,
           std::vector<std::vector<orc::Nbr>>& lists)
{
    std::vector<double> s;
    fractional(n, R, h, s);
    double w[3];
    orc_widths(h, w);
    int m[3];
    for (int k = 0; k < 3; ++k) m[k] = int(std::ceil(rc / w[k])) + 1;
    const double rc2 = rc * rc;
    lists.assign(n, {});
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            int c0[3];
            for (int k = 0; k < 3; ++k) c0[k] = -int(std::nearbyint(s[3 * j + k] - s[3 * i + k]));
            for (int a = c0[0] - m[0]; a <= c0[0] + m[0]; ++a)
                for (int b = c0[1] - m[1]; b <= c0[1] + m[1]; ++b)
                    for (int c = c0[2] - m[2]; c <= c0[2] + m[2]; ++c) {
                        if (i == j && a == 0 && b == 0 && c == 0) continue;
                        if (within(R + 3 * i, R + 3 * j, h, a, b, c, rc2))
                            lists[i].push_back({j, {a, b, c}});
                    }
        }
        std::sort(lists[i].begin(), lists[i].end(), nbr_less);
    }
}

int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Linked bins on wrapped fractional coordinates.  Candidate (j, n) pairs are a
// superset of the true set; the inclusion test is the same as brute().
void cells(int n, const double* R, const double* h, double rc,
           std::vector<std::vector<orc::Nbr>>& lists)
{
    std::vector<double> s;
    fractional(n, R, h, s);
    double w[3];
    orc_widths(h, w);
    int nb[3], reach[3];
    for (int k = 0; k < 3; ++k) {
        nb[k] = std::max(1, int(std::floor(w[k] / rc)));
        nb[k] = std::min(nb[k], 256);
        reach[k] = int(std::ceil(rc * nb[k] / w[k])) + 1;
    }
    std::vector<int> img(3 * size_t(n));
    std::vector<std::vector<int>> bins(size_t(nb[0]) * nb[1] * nb[2]);
    std::vector<int> bin_of(n);
    for (int i = 0; i < n; ++i) {
        int b[3];
        for (int k = 0; k < 3; ++k) {
            const double fl = std::floor(s[3 * i + k]);
            img[3 * i + k] = int(fl);
            const double sw = s[3 * i + k] - fl;
            b[k] = std::min(nb[k] - 1, std::max(0, int(std::floor(sw * nb[k]))));
        }
        const int id = (b[0] * nb[1] + b[1]) * nb[2] + b[2];
        bin_of[i] = id;
        bins[id].push_back(i);
    }
    const double rc2 = rc * rc;
    lists.assign(n, {});
    for (int i = 0; i < n; ++i) {
        const int id = bin_of[i];
        const int bi[3] = {id / (nb[1] * nb[2]), (id / nb[2]) % nb[1], id % nb[2]};
        // Distinct offsets map to distinct (bin, lattice image) pairs and every atom
        // sits in one bin, so no (j, n) candidate is produced twice.
        for (int dx = -reach[0]; dx <= reach[0]; ++dx)
            for (int dy = -reach[1]; dy <= reach[1]; ++dy)
                for (int dz = -reach[2]; dz <= reach[2]; ++dz) {
                    const int v[3] = {bi[0] + dx, bi[1] + dy, bi[2] + dz};
                    int actual[3], mm[3];
                    for (int k = 0; k < 3; ++k) {
                        mm[k] = floordiv(v[k], nb[k]);
                        actual[k] = v[k] - mm[k] * nb[k];
                    }
                    const int bid = (actual[0] * nb[1] + actual[1]) * nb[2] + actual[2];
                    for (int j : bins[bid]) {
                        const int t0 = mm[0] + img[3 * i] - img[3 * j];
                        const int t1 = mm[1] + img[3 * i + 1] - img[3 * j + 1];
                        const int t2 = mm[2] + img[3 * i + 2] - img[3 * j + 2];
                        if (i == j && t0 == 0 && t1 == 0 && t2 == 0) continue;
                        if (within(R + 3 * i, R + 3 * j, h, t0, t1, t2, rc2))
                            lists[i].push_back({j, {t0, t1, t2}});
                    }
                }
        std::sort(lists[i].begin(), lists[i].end(), nbr_less);
    }
}

int64_t flatten(const std::vector<std::vector<orc::Nbr>>& lists, int32_t* cnt, int32_t* ent,
                int64_t cap_total)
{
    int64_t total = 0;
    for (size_t i = 0; i < lists.size(); ++i) {
        cnt[i] = int32_t(lists[i].size());
        for (const auto& e : lists[i]) {
            if (total < cap_total) {
                ent[4 * total + 0] = e.j;
                ent[4 * total + 1] = e.n[0];
                ent[4 * total + 2] = e.n[1];
                ent[4 * total + 3] = e.n[2];
            }
            ++total;
        }
    }
    return total > cap_total ? -total : total;
}

}  // namespace

namespace orc {

int build_lists(int n, const double* R, const double* h, double rc, bool use_brute,
                std::vector<std::vector<Nbr>>& lists)
{
    if (!(std::fabs(orc_det3(h)) > 0.0)) return ORC_ECELL;
    if (use_brute)
        brute(n, R, h, rc, lists);
    else
        cells(n, R, h, rc, lists);
    return ORC_OK;
}

}  // namespace orc

extern "C" int64_t orc_nlist_brute(int n, const double* R, const double* h, double rc,
                                   int32_t* cnt, int32_t* ent, int64_t cap_total)
{
    std::vector<std::vector<orc::Nbr>> lists;
    if (orc::build_lists(n, R, h, rc, true, lists) != ORC_OK) return ORC_ECELL;
    return flatten(lists, cnt, ent, cap_total);
}

extern "C" int64_t orc_nlist_cells(int n, const double* R, const double* h, double rc,
                                   int32_t* cnt, int32_t* ent, int64_t cap_total)
{
    std::vector<std::vector<orc::Nbr>> lists;
    if (orc::build_lists(n, R, h, rc, false, lists) != ORC_OK) return ORC_ECELL;
    return flatten(lists, cnt, ent, cap_total);
}
