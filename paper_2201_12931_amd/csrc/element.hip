// Unit hex8 element stiffness from the modal energy of a trilinear field.
//
// The paper uses the solid element stiffness K0 of the 8-node brick (Sec. 2,
// Eq. 2).  Here it is derived in closed form rather than by quadrature: a
// trilinear displacement component on the unit cube is written in the
// tensor-product basis Psi_m = prod_axis psi_{m_axis} with psi_s(t) = 1 and
// psi_d(t) = 2t - 1 (m in {s,d}^3, encoded as a 3-bit mask of the "d" axes).
// Nodal values v_a map to modal coefficients w_m = (1/8) sum_a H[m][a] v_a with
// H[m][a] = prod over the d-axes of m of (a_axis ? +1 : -1).  Because
// d/dt psi_d = 2 psi_s, a derivative of a mode is again a mode, and the 1-D
// integrals int psi_s^2 = 1, int psi_d^2 = 1/3, int psi_s psi_d = 0 make the
// strain energy
//     u^T K0 u = int lambda (div u)^2 + 2 mu eps:eps
//              = int lambda (sum_c d_c u_c)^2 + mu sum_{c,j} (d_j u_c)^2 + d_j u_c d_c u_j
// an exact, sparse quadratic form Q in the modal coefficients.  Then
// K0 = H^T Q H / 64 (node-major local DOF 3a + c).
#include "hexmg_impl.h"

namespace hexmg {

static double third_pow(int k) {
  double w = 1.0;
  for (int i = 0; i < k; ++i) w /= 3.0;
  return w;
}

// int (d_j u_c)(d_j2 u_c2) over the cube, as coefficients of w[c][m] w[c2][m2].
static void add_gradient_product(double Q[24][24], int c, int j, int c2, int j2, double kappa) {
  for (int m = 0; m < 8; ++m) {
    if (!((m >> j) & 1)) continue;
    for (int m2 = 0; m2 < 8; ++m2) {
      if (!((m2 >> j2) & 1)) continue;
      const int n = m & ~(1 << j);
      if (n != (m2 & ~(1 << j2))) continue;
      // d_j Psi_m = 2 Psi_n, so the product integrates to 4 * int Psi_n^2.
      const double v = kappa * 4.0 * third_pow(__builtin_popcount(n));
      Q[3 * m + c][3 * m2 + c2] += 0.5 * v;
      Q[3 * m2 + c2][3 * m + c] += 0.5 * v;
    }
  }
}

void modal_quadratic_form(double nu, double Q[24][24]) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  for (int r = 0; r < 24; ++r)
    for (int s = 0; s < 24; ++s) Q[r][s] = 0.0;
  for (int c = 0; c < 3; ++c)
    for (int c2 = 0; c2 < 3; ++c2) add_gradient_product(Q, c, c, c2, c2, lam);
  for (int c = 0; c < 3; ++c)
    for (int j = 0; j < 3; ++j) {
      add_gradient_product(Q, c, j, c, j, mu);
      add_gradient_product(Q, c, j, j, c, mu);
    }
}

static int haar_sign(int m, int a) {
  int s = 1;
  for (int ax = 0; ax < 3; ++ax)
    if (((m >> ax) & 1) && !((a >> ax) & 1)) s = -s;
  return s;
}

void element_matrix(double nu, double Ke[576]) {
  double Q[24][24];
  modal_quadratic_form(nu, Q);
  for (int a = 0; a < 8; ++a)
    for (int c = 0; c < 3; ++c)
      for (int b = 0; b < 8; ++b)
        for (int d = 0; d < 3; ++d) {
          double s = 0.0;
          for (int m = 0; m < 8; ++m)
            for (int m2 = 0; m2 < 8; ++m2)
              s += haar_sign(m, a) * Q[3 * m + c][3 * m2 + d] * haar_sign(m2, b);
          Ke[(3 * a + c) * 24 + 3 * b + d] = s / 64.0;
        }
}

}  // namespace hexmg
