// Host-side (create-time) finite element and screen ingredients, float64.
//
// Element units throughout: one element is [-1/2, 1/2].  These small dense
// objects feed the device kernels as constants; nothing here runs per call.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace fep3m {

using Vec = std::vector<double>;

// Row-major dense matrix.
struct Mat {
  int r = 0, c = 0;
  Vec a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a(size_t(r_) * c_, 0.0) {}
  double &operator()(int i, int j) { return a[size_t(i) * c + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * c + j]; }
};

// Gauss-Legendre rule with m points on [-1/2, 1/2].
void gauss_legendre(int m, Vec &x, Vec &w);
// p+1 Gauss-Lobatto-Legendre nodes on [-1/2, 1/2].
Vec gll_nodes(int p);
// Lagrange basis on `nodes` at x: out[k] = l_k(x); dout[k] = l_k'(x) (may be null).
void lagrange(const Vec &nodes, double x, double *out, double *dout);
// Element stiffness ke[a][b] = int l_a' l_b' and mass me[a][b] = int l_a l_b.
void element_matrices(int p, Mat &ke, Mat &me);

// Symmetric eigen-decomposition by cyclic Jacobi rotations: A = V diag(w) V^T,
// eigenvalues ascending, V columns the eigenvectors.
void sym_eig(const Mat &A, Vec &w, Mat &V);
// Generalised symmetric-definite problem K v = lambda M v with V^T M V = I.
void sym_gen_eig(const Mat &K, const Mat &M, Vec &w, Mat &V);
// Dense inverse by Gauss-Jordan with partial pivoting.
Mat inverse(const Mat &A);

// One-element polynomial screen of degree q (moment degree d = q - 2):
// dual functions r_l, l = 0..d, on the element, with int x^m r_l = [m == l].
// The interior order-q Lagrange functions span bubble * P_d with
// bubble = 1/4 - x^2, so r_l is represented in that basis.
struct Screen1D {
  int q = 3, d = 1;
  Mat coef;                  // coef(j, l): r_l = sum_j coef(j,l) * bubble * x^j
  double eval(int l, double x) const;
  // Monomial coefficients (ascending) of r_l on the element, degree d + 2.
  Vec monomial(int l) const;
};
Screen1D make_screen(int q);

// g(l, k) = int l_k^(p) r_l over the element (load weights), (d+1) x (p+1).
Mat load_weights(int p, const Screen1D &s);

// Assembled 1-D matrices of `ne` unit elements, order p.
// periodic: p*ne DOFs; otherwise p*ne + 1 DOFs (all nodes).
void assemble_1d(int p, int ne, bool periodic, Mat &K, Mat &M);

}  // namespace fep3m
