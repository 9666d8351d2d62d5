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
#include <cmath>

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

bool haar_coefficients(double nu, HaarCoef<double>* q) {
  double Q[24][24];
  modal_quadratic_form(nu, Q);
  auto at = [&](int m, int c, int m2, int c2) { return Q[3 * m + c][3 * m2 + c2]; };
  const double a1 = at(1, 0, 1, 0), b1 = at(1, 0, 2, 1), g = at(1, 1, 1, 1);
  const double a2 = at(3, 0, 3, 0), b2 = at(3, 0, 6, 2), a3 = at(3, 2, 3, 2), b3 = at(3, 2, 5, 1);
  const double a4 = at(7, 0, 7, 0);
  // Rebuild Q from the 14-block pattern and compare.
  double P[24][24];
  for (int r = 0; r < 24; ++r)
    for (int s = 0; s < 24; ++s) P[r][s] = 0.0;
  auto set = [&](int m, int c, int m2, int c2, double v) {
    P[3 * m + c][3 * m2 + c2] = v;
    P[3 * m2 + c2][3 * m + c] = v;
  };
  const int normal[3][2] = {{1, 0}, {2, 1}, {4, 2}};
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) set(normal[x][0], normal[x][1], normal[y][0], normal[y][1], x == y ? a1 : b1);
  const int shear[3][4] = {{1, 1, 2, 0}, {1, 2, 4, 0}, {2, 2, 4, 1}};
  for (auto& sh : shear) {
    set(sh[0], sh[1], sh[0], sh[1], g);
    set(sh[2], sh[3], sh[2], sh[3], g);
    set(sh[0], sh[1], sh[2], sh[3], g);
  }
  const int bil[3][4] = {{3, 0, 6, 2}, {3, 1, 5, 2}, {5, 0, 6, 1}};
  for (auto& b : bil) {
    set(b[0], b[1], b[0], b[1], a2);
    set(b[2], b[3], b[2], b[3], a2);
    set(b[0], b[1], b[2], b[3], b2);
  }
  const int tri3[3][2] = {{3, 2}, {5, 1}, {6, 0}};
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) set(tri3[x][0], tri3[x][1], tri3[y][0], tri3[y][1], x == y ? a3 : b3);
  for (int c = 0; c < 3; ++c) set(7, c, 7, c, a4);
  double scale = 0.0, err = 0.0;
  for (int r = 0; r < 24; ++r)
    for (int s = 0; s < 24; ++s) {
      scale = std::fmax(scale, std::fabs(Q[r][s]));
      err = std::fmax(err, std::fabs(Q[r][s] - P[r][s]));
    }
  if (!(err <= 1e-13 * scale)) return false;
  q->d1 = (a1 - b1) / 64.0;
  q->b1 = b1 / 64.0;
  q->g = g / 64.0;
  q->a2 = a2 / 64.0;
  q->b2 = b2 / 64.0;
  q->d3 = (a3 - b3) / 64.0;
  q->b3 = b3 / 64.0;
  q->a4 = a4 / 64.0;
  return true;
}

}  // namespace hexmg
