// Lambda-adaptive weight table of the 27-point stencil, fitted on the host.
//
// Paper sec. 2.3 (FDFD): the stiffness and consistent-mass parts are mixed
// over rotated coordinate systems with weights chosen per G = lambda / h by
// least-squares minimisation of the phase-velocity dispersion; each row of
// A then uses the weights of its local G.
//
// Parametrisation.  Stiffness families F1 (axis differences), F2 (in-plane
// rotated), F3 (3D rotated) have plane-wave symbols, with c_a = cos(xi_a),
//   L1 = 2 (3 - S1), L2 = 3 - S2, L3 = (3 + S1 - S2 - 3 S3) / 2,
//   S1 = sum c_a, S2 = sum_{a<b} c_a c_b, S3 = c_x c_y c_z,
// and the mass symbol is mu = 1 + wf (2 S1 - 6) + we (4 S2 - 12) + wc (8 S3 - 8)
// after eliminating the centre weight (wm0 = 1 - 6 wf - 12 we - 8 wc).
// To first order the dispersion residual Lambda - k^2 mu lies in
// span{1, S1, S2, S3} with its constant fixed by consistency, so only three
// weight combinations are identifiable; the stiffness mix is therefore fixed
// at the fourth-order isotropic choice (1/2, 1/3, 1/6) and the three mass
// weights are fitted per G.  Objective (linearised relative phase-velocity
// error over 128 directions, theta = i (pi/2)/15, phi = j (pi/4)/7):
//   min_p  sum_d ((Lambda_d - k^2 mu_d) / (2 k^2))^2 + 1e-8 |p|^2,  k = 2 pi / G,
// a linear least-squares problem solved here by Householder QR of the
// stacked system [J; 1e-4 I] p = [y; 0].
#include <cmath>
#include <vector>

namespace oras {

namespace {

constexpr int NTH = 16, NPH = 8, NDIR = NTH * NPH, NP = 3;
constexpr double W1 = 0.5, W2 = 1.0 / 3.0, W3 = 1.0 / 6.0;
constexpr double RIDGE_SQRT = 1e-4;   // sqrt(1e-8)

// Solve min |M p - y| for an (m x 3) dense M (column major) by Householder QR.
void qr_solve(std::vector<double>& M, std::vector<double>& y, int m, double p[NP]) {
  for (int j = 0; j < NP; ++j) {
    double* col = &M[(size_t)j * m];
    double norm = 0.0;
    for (int i = j; i < m; ++i) norm += col[i] * col[i];
    norm = std::sqrt(norm);
    const double alpha = (col[j] > 0.0) ? -norm : norm;
    std::vector<double> v(m, 0.0);
    for (int i = j; i < m; ++i) v[i] = col[i];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int jj = j; jj < NP; ++jj) {
      double* cj = &M[(size_t)jj * m];
      double d = 0.0;
      for (int i = j; i < m; ++i) d += v[i] * cj[i];
      const double f = 2.0 * d / vv;
      for (int i = j; i < m; ++i) cj[i] -= f * v[i];
    }
    double d = 0.0;
    for (int i = j; i < m; ++i) d += v[i] * y[i];
    const double f = 2.0 * d / vv;
    for (int i = j; i < m; ++i) y[i] -= f * v[i];
  }
  for (int j = NP - 1; j >= 0; --j) {
    double acc = y[j];
    for (int jj = j + 1; jj < NP; ++jj) acc -= M[(size_t)jj * m + j] * p[jj];
    p[j] = acc / M[(size_t)j * m + j];
  }
}

}  // namespace

// Weights (w1, w2, w3, wm0, wmf, wme, wmc) at one G.
void fit_weights_at(double G, double out[7]) {
  const double k = 2.0 * M_PI / G;
  const int m = NDIR + NP;
  std::vector<double> M((size_t)m * NP, 0.0), y(m, 0.0);
  int row = 0;
  for (int it = 0; it < NTH; ++it) {
    const double th = it * (M_PI / 2.0) / (NTH - 1);
    for (int ip = 0; ip < NPH; ++ip, ++row) {
      const double ph = ip * (M_PI / 4.0) / (NPH - 1);
      const double nxv = std::sin(th) * std::cos(ph);
      const double nyv = std::sin(th) * std::sin(ph);
      const double nzv = std::cos(th);
      const double cx = std::cos(k * nxv), cy = std::cos(k * nyv), cz = std::cos(k * nzv);
      const double S1 = cx + cy + cz;
      const double S2 = cx * cy + cx * cz + cy * cz;
      const double S3 = cx * cy * cz;
      const double lam = W1 * 2.0 * (3.0 - S1) + W2 * (3.0 - S2) + W3 * 0.5 * (3.0 + S1 - S2 - 3.0 * S3);
      // residual = (lam - k^2) / (2k^2) - [ (S1-3) wf + (2S2-6) we + (4S3-4) wc ]
      y[row] = (lam - k * k) / (2.0 * k * k);
      M[0 * (size_t)m + row] = S1 - 3.0;
      M[1 * (size_t)m + row] = 2.0 * S2 - 6.0;
      M[2 * (size_t)m + row] = 4.0 * S3 - 4.0;
    }
  }
  for (int j = 0; j < NP; ++j) {
    M[(size_t)j * m + NDIR + j] = RIDGE_SQRT;
    y[NDIR + j] = 0.0;
  }
  double p[NP];
  qr_solve(M, y, m, p);
  out[0] = W1;
  out[1] = W2;
  out[2] = W3;
  out[4] = p[0];
  out[5] = p[1];
  out[6] = p[2];
  out[3] = 1.0 - 6.0 * p[0] - 12.0 * p[1] - 8.0 * p[2];
}

// Table on G = 3, 3.25, ..., 48.
void fit_table(std::vector<double>& tab, double& g0, double& dg, int& count) {
  g0 = 3.0;
  dg = 0.25;
  count = 181;
  tab.assign((size_t)count * 7, 0.0);
  for (int r = 0; r < count; ++r) fit_weights_at(g0 + dg * r, &tab[(size_t)r * 7]);
}

}  // namespace oras
