// Host-side FP64 tables uploaded once per RVE: FFT twiddles, per-axis wave
// vectors of the projection operators, and per-label material tables
// (sample-frame slip systems and rotated cubic stiffness).
#include "tables.hpp"

#include <cmath>
#include <stdexcept>

namespace rve {

std::vector<double> twiddles(int n) {
  // tw[m] = exp(-2 pi i m / n), interleaved (re, im)
  std::vector<double> t(2 * n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    t[2 * m] = std::cos(a);
    t[2 * m + 1] = std::sin(a);
  }
  return t;
}

std::vector<double> wave_vectors(int n, const double L[3], int projection) {
  // Sec. 2.2, Eq. 18: integer frequency k in {-n/2, ..., n/2 - 1} at DFT
  // index k mod n, q = 2 pi k / n.  Continuous operator (Eq. 19): v = q n/L;
  // discrete operator (Eqs. 20-21): v = tan(q/2) n/L.  The Nyquist entry is
  // never used (the operator is zero there) and is set to 0.
  std::vector<double> v(3 * n, 0.0);
  for (int d = 0; d < 3; ++d) {
    for (int idx = 0; idx < n; ++idx) {
      const int k = (idx < (n + 1) / 2) ? idx : idx - n;
      if (n % 2 == 0 && k == -n / 2) continue;
      const double q = 2.0 * M_PI * (double)k / (double)n;
      const double scale = (double)n / L[d];
      v[d * n + idx] = (projection == 0) ? q * scale : std::tan(0.5 * q) * scale;
    }
  }
  return v;
}

namespace {

// FCC {111}<110>: plane normals in this order; for each, the directions of
// the list below orthogonal to it, in list order.
const int kNormals[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
const int kDirs[6][3] = {{1, -1, 0}, {1, 0, -1}, {0, 1, -1},
                         {1, 1, 0},  {1, 0, 1},  {0, 1, 1}};

void slip_systems(double s[12][3], double m[12][3]) {
  int a = 0;
  for (int p = 0; p < 4; ++p) {
    for (int d = 0; d < 6; ++d) {
      const int dot = kNormals[p][0] * kDirs[d][0] +
                      kNormals[p][1] * kDirs[d][1] +
                      kNormals[p][2] * kDirs[d][2];
      if (dot != 0) continue;
      for (int i = 0; i < 3; ++i) {
        s[a][i] = kDirs[d][i] / std::sqrt(2.0);
        m[a][i] = kNormals[p][i] / std::sqrt(3.0);
      }
      ++a;
    }
  }
  if (a != 12) throw std::logic_error("slip system construction");
}

void quat_rotation(const double* q, double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z);
  R[0][1] = 2 * (x * y - w * z);
  R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);
  R[1][1] = 1 - 2 * (x * x + z * z);
  R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);
  R[2][1] = 2 * (y * z + w * x);
  R[2][2] = 1 - 2 * (x * x + y * y);
}

const int kVoigt[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};

}  // namespace

std::vector<double> label_table(int G, const double* quat, const int32_t* law,
                                const double* params) {
  std::vector<double> tab((size_t)G * kTableStride, 0.0);
  double s0[12][3], m0[12][3];
  slip_systems(s0, m0);
  const double C11 = params[0], C12 = params[1], C44 = params[2];
  const double E = params[8], nu = params[9];
  // lattice-frame cubic stiffness
  double Cl[3][3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double v = 0.0;
          if (a == b && c == d) v += C12;
          if (a == c && b == d) v += C44;
          if (a == d && b == c) v += C44;
          if (a == b && b == c && c == d) v += C11 - C12 - 2.0 * C44;
          Cl[a][b][c][d] = v;
        }
  for (int g = 0; g < G; ++g) {
    double* t = &tab[(size_t)g * kTableStride];
    t[0] = (double)law[g];
    if (law[g] == 1) {
      t[kTabLam] = E * nu / ((1 + nu) * (1 - 2 * nu));
      t[kTabMu] = E / (2 * (1 + nu));
      continue;
    }
    double qn[4];
    const double nrm = std::sqrt(quat[4 * g] * quat[4 * g] +
                                 quat[4 * g + 1] * quat[4 * g + 1] +
                                 quat[4 * g + 2] * quat[4 * g + 2] +
                                 quat[4 * g + 3] * quat[4 * g + 3]);
    for (int i = 0; i < 4; ++i) qn[i] = quat[4 * g + i] / nrm;
    double R[3][3];
    quat_rotation(qn, R);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) t[kTabR + 3 * i + j] = R[i][j];
    double s[12][3], m[12][3];
    for (int a = 0; a < 12; ++a)
      for (int i = 0; i < 3; ++i) {
        s[a][i] = R[i][0] * s0[a][0] + R[i][1] * s0[a][1] + R[i][2] * s0[a][2];
        m[a][i] = R[i][0] * m0[a][0] + R[i][1] * m0[a][1] + R[i][2] * m0[a][2];
        t[kTabS + 3 * a + i] = s[a][i];
        t[kTabM + 3 * a + i] = m[a][i];
      }
    // sample-frame stiffness C_ijkl = R_ia R_jb R_kc R_ld Cl_abcd
    double Cs[3][3][3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c)
                  for (int d = 0; d < 3; ++d)
                    acc += R[i][a] * R[j][b] * R[k][c] * R[l][d] * Cl[a][b][c][d];
            Cs[i][j][k][l] = acc;
          }
    for (int I = 0; I < 6; ++I)
      for (int J = 0; J < 6; ++J)
        t[kTabC + 6 * I + J] =
            Cs[kVoigt[I][0]][kVoigt[I][1]][kVoigt[J][0]][kVoigt[J][1]];
    // N_a = C : sym(s_a (x) m_a), Voigt
    for (int a = 0; a < 12; ++a)
      for (int I = 0; I < 6; ++I) {
        const int i = kVoigt[I][0], j = kVoigt[I][1];
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l)
            acc += Cs[i][j][k][l] * 0.5 * (s[a][k] * m[a][l] + s[a][l] * m[a][k]);
        t[kTabN + 6 * a + I] = acc;
      }
  }
  return tab;
}

}  // namespace rve
