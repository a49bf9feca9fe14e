// Oracle (test infrastructure only): 3x3 cell geometry in FP64.
// Lattice vectors are the rows of h (Sec. II.B, text after Eq. (2)).
#include "oracle.h"
#include "internal.h"

#include <cmath>

extern "C" double orc_det3(const double* A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Inverse by the adjugate divided by the determinant.
extern "C" void orc_inv3(const double* A, double* Ainv)
{
    const double det = orc_det3(A);
    double adj[9];
    adj[0] = A[4] * A[8] - A[5] * A[7];
    adj[1] = A[2] * A[7] - A[1] * A[8];
    adj[2] = A[1] * A[5] - A[2] * A[4];
    adj[3] = A[5] * A[6] - A[3] * A[8];
    adj[4] = A[0] * A[8] - A[2] * A[6];
    adj[5] = A[2] * A[3] - A[0] * A[5];
    adj[6] = A[3] * A[7] - A[4] * A[6];
    adj[7] = A[1] * A[6] - A[0] * A[7];
    adj[8] = A[0] * A[4] - A[1] * A[3];
    for (int i = 0; i < 9; ++i) Ainv[i] = adj[i] / det;
}

// Symmetric square root by cyclic Jacobi diagonalisation:
// sym(B) = Q diag(lambda) Q^T, D = Q diag(sqrt(lambda)) Q^T.
extern "C" int orc_symsqrt(const double* B, double* D)
{
    double a[3][3], q[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = 0.5 * (B[3 * i + j] + B[3 * j + i]);
            q[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-36 * diag) break;
        const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (const auto& pq : pairs) {
            const int p = pq[0], r = pq[1];
            if (a[p][r] == 0.0) continue;
            // rotation angle that zeroes a[p][r]
            const double theta = (a[r][r] - a[p][p]) / (2.0 * a[p][r]);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
            const double c = 1.0 / std::sqrt(t * t + 1.0);
            const double s = t * c;
            // A <- J^T A J with J the Givens rotation in the (p, r) plane
            for (int k = 0; k < 3; ++k) {
                const double akp = a[k][p], akr = a[k][r];
                a[k][p] = c * akp - s * akr;
                a[k][r] = s * akp + c * akr;
            }
            for (int k = 0; k < 3; ++k) {
                const double apk = a[p][k], ark = a[r][k];
                a[p][k] = c * apk - s * ark;
                a[r][k] = s * apk + c * ark;
            }
            for (int k = 0; k < 3; ++k) {
                const double qkp = q[k][p], qkr = q[k][r];
                q[k][p] = c * qkp - s * qkr;
                q[k][r] = s * qkp + c * qkr;
            }
        }
    }
    double sl[3];
    for (int i = 0; i < 3; ++i) {
        if (!(a[i][i] > 0.0)) return ORC_ECELL;
        sl[i] = std::sqrt(a[i][i]);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += q[i][k] * sl[k] * q[j][k];
            D[3 * i + j] = s;
        }
    return ORC_OK;
}

// w_k = Omega / |h_{k+1} x h_{k+2}|: distance between the two cell faces
// spanned by the other two lattice vectors.
extern "C" void orc_widths(const double* h, double* w)
{
    const double vol = std::fabs(orc_det3(h));
    for (int k = 0; k < 3; ++k) {
        const double* a = h + 3 * ((k + 1) % 3);
        const double* b = h + 3 * ((k + 2) % 3);
        const double cx = a[1] * b[2] - a[2] * b[1];
        const double cy = a[2] * b[0] - a[0] * b[2];
        const double cz = a[0] * b[1] - a[1] * b[0];
        w[k] = vol / std::sqrt(cx * cx + cy * cy + cz * cz);
    }
}

namespace orc {

void matmul3(const double* A, const double* B, double* C)
{
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    for (int i = 0; i < 9; ++i) C[i] = t[i];
}

void transpose3(const double* A, double* T)
{
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = A[3 * j + i];
    for (int i = 0; i < 9; ++i) T[i] = t[i];
}

// rows of P (n x 3) times M (3 x 3)
void rows_times(int n, const double* P, const double* M, double* out)
{
    for (int i = 0; i < n; ++i) {
        const double x = P[3 * i], y = P[3 * i + 1], z = P[3 * i + 2];
        for (int c = 0; c < 3; ++c) out[3 * i + c] = x * M[c] + y * M[3 + c] + z * M[6 + c];
    }
}

}  // namespace orc
