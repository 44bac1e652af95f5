// Host-side set-up mathematics of the DG-BGK library: discrete velocity sets,
// the 1-D Gauss-Lobatto-Legendre reference element and its operators.
// Everything the device kernels consume as tables is built here once per
// solver; none of it runs per time step.
#pragma once

#include <vector>

namespace dgbgk {

// Eigen-decomposition of a symmetric n x n matrix (row-major) by cyclic
// Jacobi rotations: A = V diag(evals) V^T, eigenvalues ascending, eigenvector i
// in column i of V.
void symmetric_eigen(int n, std::vector<double> A, std::vector<double> &evals,
                     std::vector<double> &V);

// 1-D n-point Gauss-Hermite rule for the standard normal density (RT = 1),
// weights summing to one (Golub-Welsch nodes, Newton-polished; Christoffel
// weights).  Returns false on bad n.
bool gauss_hermite_rule(int n, std::vector<double> &x, std::vector<double> &w);

// 1-D m-point composite Newton-Cotes (trapezoid) rule on [-vmax, vmax] with
// Maxwellian weighting, normalised to sum one.
bool newton_cotes_rule(int m, double vmax, std::vector<double> &x, std::vector<double> &w);

// p+1 Gauss-Lobatto-Legendre nodes on [-1, 1], ascending.
bool gll_points(int p, std::vector<double> &r);

// n-point Gauss-Legendre rule on [-1, 1].
bool gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w);

// Values of the Lagrange basis on nodes r at point t (barycentric form).
void lagrange_values(const std::vector<double> &r, double t, std::vector<double> &out);

// Nodal differentiation matrix D[i][j] = l_j'(r_i) (barycentric formula).
void differentiation_matrix(const std::vector<double> &r, std::vector<double> &D);

// Exact 1-D mass matrix M[i][j] = int_{-1}^{1} l_i l_j by Gauss-Legendre.
void mass_matrix(const std::vector<double> &r, std::vector<double> &M);

// Solve M x = b for symmetric positive definite M (Cholesky).
bool spd_solve(int n, const std::vector<double> &M, const std::vector<double> &b,
               std::vector<double> &x);

}  // namespace dgbgk
