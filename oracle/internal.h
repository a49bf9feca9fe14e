// Oracle (test infrastructure only): helpers shared between the oracle's own files.
#ifndef CFNEB_ORACLE_INTERNAL_H
#define CFNEB_ORACLE_INTERNAL_H

#include <cstdint>
#include <vector>

#include "oracle.h"

namespace orc {

void matmul3(const double* A, const double* B, double* C);
void transpose3(const double* A, double* T);
void rows_times(int n, const double* P, const double* M, double* out);

// One neighbour entry (j, n) of atom i.
struct Nbr {
    int j;
    int n[3];
};

// Full neighbour lists, one vector per atom, sorted by (j, n).
int build_lists(int n, const double* R, const double* h, double rc, bool brute,
                std::vector<std::vector<Nbr>>& lists);

// Bond-wise evaluation: u_i and P_e = dU_i/dr^{ij} for every entry of i's list,
// then forces and virial are assembled from P.
int eval_with_lists(const orc_params* p, int n, const double* R, const double* h,
                    const std::vector<std::vector<Nbr>>& lists,
                    double* E, double* u, double* F, double* V);

double cutoff_of(const orc_params* p);

// Cell factor c_f of the generalized cell coordinate c_f B.  Default (cell_factor <= 0):
// |det h0|^(1/3) n^(1/6), the size-consistent Jacobian of the generalized solid-state
// NEB, so that a uniform strain of the cell and a uniform displacement of all n atoms
// have comparable lengths in the band's metric and comparable stiffness.
double cell_factor_of(const orc_params* p, int n, const double* h0);

// Deformation gradient D of an image from its cell coordinates C = (cell rows of X)/c_f:
// the rotation-free filter stores C = B = D D^T and takes D = symsqrt(B); the D-variant
// stores C = D itself (det D > 0 required).  ECELL otherwise.
int cell_gauge(const orc_params* p, const double* C, double* D);

// Subtract from each of the three components of the first natoms rows of a its mean
// over those rows (removes a rigid translation of the atoms; later rows untouched).
void remove_translation(std::vector<double>& a, int natoms);

// Arc lengths s_k of a band of M images (row-major M x dim) in the band's metric:
// Euclidean lengths of consecutive differences with the atoms' rigid translation removed.
void arc_lengths(int M, int natoms, int dim, const double* X, double* s);

}  // namespace orc

#endif
