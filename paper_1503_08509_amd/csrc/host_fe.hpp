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

// Polynomial screens of degree q (Section 2.1): per axis the dual functions
// r_l, l = 0..d, of the screen space, with int x^m r_l = [m == l] for
// m <= d, so that the combined screen of an element's charges is
// sum_a C[E][a] r_ax (x) r_ay (x) r_az with C[E][a] = sum Q u^a.
//   support 0, one element (Section 5): the order-q functions interior to the
//     element, span bubble * P_{q-2}; d = q - 2, one piece.
//   support 1, 27 elements (Section 2.1): the order-q Lagrange functions of
//     the nodes of the closed element on equispaced order-q nodes; the face
//     functions reach one element further, so the support spans 3 elements
//     per axis; d = q, pieces on the elements at offsets -1, 0, 1.
// Each piece is a polynomial of degree q in the local coordinate t in
// [-1/2, 1/2] of its element.
struct Screen1D {
  int q = 3, d = 1, support = 0;
  int span = 1;              // elements per axis of the support
  Vec pc;                    // pc[(s (d + 1) + l) (q + 1) + k]: t^k coefficient of r_l on piece s
  const double *piece(int s, int l) const { return &pc[(size_t(s) * (d + 1) + l) * (q + 1)]; }
  // r_l at x, element units from the centre of the charge's element
  double eval(int l, double x) const;
  // r_l on piece s at local coordinate t
  double eval_piece(int s, int l, double t) const;
};
Screen1D make_screen(int q, int support = 0);

// g(l, j) = int phi_j r_l over the support (load weights), (d + 1) x
// (span p + 1): phi_j the order-p GLL Lagrange function of the support's
// node j, j = 0 at the lower end of the support.
Mat load_weights(int p, const Screen1D &s);

// Fourier blocks of the periodic order-p 1-D operators over n unit
// elements: for each frequency f < n the p x p Hermitian pencil
// K^(f) = B0 + B+ w^f + B- w^-f (w = exp(2 pi i / n), B+- the couplings of
// an element's owned nodes to the next / previous element) and M^(f)
// alike, and its generalized eigenvectors: W[f][k][i] (component k of mode
// i, real and imaginary parts) with W^H M^ W = I, eigenvalues lam[f][i]
// ascending.  The null mode (constants, f = 0) has lam exactly 0.
void periodic_fourier_eigen(int p, int n, Vec &Wre, Vec &Wim, Vec &lam);

// Assembled 1-D matrices of `ne` unit elements, order p.
// periodic: p*ne DOFs; otherwise p*ne + 1 DOFs (all nodes).
void assemble_1d(int p, int ne, bool periodic, Mat &K, Mat &M);

}  // namespace fep3m
