// Host-side construction of the noisy circuit of a Trotterised time-independent Lindbladian
// (Sec. "Time-independent Lindbladian systems"; appendix "Exact decomposition of Trotterized
// Lindbladian evolutions").  Matrices here are at most 4 x 4, built once per circuit:
//   * the gate of a pair term, exp(-i H dt);
//   * the Kraus operators of a single-site jump process exp(L_jump tau): the vectorised jump
//     superoperator, its exponential, the reshuffle into the Choi matrix and that matrix's
//     eigendecomposition (K_i = sqrt(lambda_i) reshape(v_i)).
// Vectorisation |rho>> = (rho (x) I)|Omega>: (A (x) B)|rho>> = |A rho B^T>>, row-major indices.
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <utility>

#include "mpsb.h"

namespace mpsb {
int report_error(int code, const std::string& msg);
}

namespace {

using cd = std::complex<double>;

void matmul(int d, const cd* a, const cd* b, cd* c) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      cd s = 0.0;
      for (int k = 0; k < d; ++k) s += a[i * d + k] * b[k * d + j];
      c[i * d + j] = s;
    }
}

// exp(A), d <= 4: A / 2^s with ||A / 2^s||_1 <= 1/2, Taylor series to degree 18 (remainder
// below 2^-19 / 19! relative), then s squarings.
void expm(int d, const cd* a, cd* e) {
  double nrm = 0.0;
  for (int j = 0; j < d; ++j) {
    double col = 0.0;
    for (int i = 0; i < d; ++i) col += std::abs(a[i * d + j]);
    nrm = std::fmax(nrm, col);
  }
  int s = 0;
  while (nrm > 0.5 && s < 60) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = std::ldexp(1.0, -s);
  cd x[16], term[16], tmp[16];
  for (int i = 0; i < d * d; ++i) {
    x[i] = a[i] * sc;
    e[i] = (i % (d + 1) == 0) ? 1.0 : 0.0;
    term[i] = e[i];
  }
  for (int k = 1; k <= 18; ++k) {
    matmul(d, term, x, tmp);
    for (int i = 0; i < d * d; ++i) {
      term[i] = tmp[i] / (double)k;
      e[i] += term[i];
    }
  }
  for (int r = 0; r < s; ++r) {
    matmul(d, e, e, tmp);
    std::memcpy(e, tmp, sizeof(cd) * d * d);
  }
}

// Eigen-decomposition of a d x d Hermitian matrix (d <= 4) by cyclic Jacobi rotations: each
// pair (p, q) is made real by the phase of a_pq and then rotated to zero (a real symmetric
// Jacobi rotation).  w ascending is NOT imposed; V columns are the eigenvectors.
void heig(int d, cd* a, double* w, cd* v) {
  for (int i = 0; i < d * d; ++i) v[i] = (i % (d + 1) == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) (i == j ? dia : off) += std::norm(a[i * d + j]);
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < d - 1; ++p)
      for (int q = p + 1; q < d; ++q) {
        const cd apq = a[p * d + q];
        const double b = std::abs(apq);
        if (b == 0.0) continue;
        const cd ph = apq / b;   // e^{i phi}
        const double app = a[p * d + p].real(), aqq = a[q * d + q].real();
        const double tau = (aqq - app) / (2.0 * b);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // G = diag(1, e^{-i phi}) [[c, s], [-s, c]] on (p, q): columns p and q of G
        const cd gpp = c, gqp = -s * std::conj(ph), gpq = s, gqq = c * std::conj(ph);
        // A <- A G (columns), then A <- G^dag A (rows)
        for (int r = 0; r < d; ++r) {
          const cd xp = a[r * d + p], xq = a[r * d + q];
          a[r * d + p] = xp * gpp + xq * gqp;
          a[r * d + q] = xp * gpq + xq * gqq;
          const cd vp = v[r * d + p], vq = v[r * d + q];
          v[r * d + p] = vp * gpp + vq * gqp;
          v[r * d + q] = vp * gpq + vq * gqq;
        }
        for (int col = 0; col < d; ++col) {
          const cd xp = a[p * d + col], xq = a[q * d + col];
          a[p * d + col] = std::conj(gpp) * xp + std::conj(gqp) * xq;
          a[q * d + col] = std::conj(gpq) * xp + std::conj(gqq) * xq;
        }
        a[p * d + q] = 0.0;
        a[q * d + p] = 0.0;
      }
  }
  for (int i = 0; i < d; ++i) w[i] = a[i * d + i].real();
}

bool finite(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

extern "C" {

int mps_trotter_gate(const double* h, double dt, double* gate) {
  const auto fail = mpsb::report_error;
  if (!h || !gate) return fail(MPSB_EINVAL, "null argument");
  if (!finite(h, 32) || !std::isfinite(dt)) return fail(MPSB_ENUM, "non-finite Hamiltonian or time step");
  cd a[16], e[16];
  double scale = 0.0;
  for (int i = 0; i < 16; ++i) scale = std::fmax(scale, std::abs(cd(h[2 * i], h[2 * i + 1])));
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const cd hij(h[2 * (4 * i + j)], h[2 * (4 * i + j) + 1]), hji(h[2 * (4 * j + i)], h[2 * (4 * j + i) + 1]);
      if (std::abs(hij - std::conj(hji)) > 1e-12 * std::fmax(scale, 1.0)) return fail(MPSB_EINVAL, "Hamiltonian term is not Hermitian");
      a[4 * i + j] = cd(0.0, -dt) * hij;
    }
  expm(4, a, e);
  for (int i = 0; i < 16; ++i) {
    gate[2 * i] = e[i].real();
    gate[2 * i + 1] = e[i].imag();
  }
  return MPSB_OK;
}

int mps_jump_channel(int n_jumps, const double* c, const double* gamma, double tau, double* kraus, int* n_kraus) {
  const auto fail = mpsb::report_error;
  if (n_jumps < 1 || !c || !gamma || !kraus || !n_kraus) return fail(MPSB_EINVAL, "bad arguments");
  if (!finite(c, 8 * n_jumps) || !finite(gamma, n_jumps) || !std::isfinite(tau)) return fail(MPSB_ENUM, "non-finite input");
  if (tau < 0.0) return fail(MPSB_EINVAL, "tau < 0");
  for (int j = 0; j < n_jumps; ++j)
    if (gamma[j] < 0.0) return fail(MPSB_EINVAL, "negative jump rate");
  // L = sum_j gamma_j (c (x) c^* - 1/2 c^dag c (x) I - 1/2 I (x) c^T c^*), 4 x 4 on (a, b)
  cd L[16] = {};
  for (int j = 0; j < n_jumps; ++j) {
    cd m[2][2], cdc[2][2], ctc[2][2];
    for (int x = 0; x < 4; ++x) m[x >> 1][x & 1] = cd(c[8 * j + 2 * x], c[8 * j + 2 * x + 1]);
    for (int i = 0; i < 2; ++i)
      for (int k = 0; k < 2; ++k) {
        cdc[i][k] = std::conj(m[0][i]) * m[0][k] + std::conj(m[1][i]) * m[1][k];   // (c^dag c)_ik
        ctc[i][k] = m[0][i] * std::conj(m[0][k]) + m[1][i] * std::conj(m[1][k]);   // (c^T c^*)_ik
      }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int cc = 0; cc < 2; ++cc)
          for (int d = 0; d < 2; ++d) {
            cd v = m[a][cc] * std::conj(m[b][d]);
            if (b == d) v -= 0.5 * cdc[a][cc];
            if (a == cc) v -= 0.5 * ctc[b][d];
            L[(2 * a + b) * 4 + (2 * cc + d)] += gamma[j] * tau * v;
          }
  }
  cd S[16], J[16], V[16];
  expm(4, L, S);
  // Choi matrix J[(a,c),(b,d)] = S[(a,b),(c,d)], Hermitian part
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int cc = 0; cc < 2; ++cc)
        for (int d = 0; d < 2; ++d) J[(2 * a + cc) * 4 + (2 * b + d)] = S[(2 * a + b) * 4 + (2 * cc + d)];
  for (int i = 0; i < 4; ++i)
    for (int k = i; k < 4; ++k) {
      const cd x = 0.5 * (J[4 * i + k] + std::conj(J[4 * k + i]));
      J[4 * i + k] = x;
      J[4 * k + i] = std::conj(x);
    }
  double w[4];
  heig(4, J, w, V);
  // descending eigenvalues (ties by index), zero ones (below 1e-14 of the largest) dropped;
  // each operator's phase is fixed so that its largest-modulus entry (first on ties) is real
  // positive
  int ord[4] = {0, 1, 2, 3};
  for (int i = 0; i < 4; ++i)
    for (int k = i + 1; k < 4; ++k)
      if (w[ord[k]] > w[ord[i]] || (w[ord[k]] == w[ord[i]] && ord[k] < ord[i])) std::swap(ord[i], ord[k]);
  const double wmax = w[ord[0]];
  if (!(wmax > 0.0)) return fail(MPSB_ENUM, "jump channel has no positive Choi eigenvalue");
  std::memset(kraus, 0, sizeof(double) * 32);
  int r = 0;
  for (int i = 0; i < 4; ++i) {
    const int e = ord[i];
    if (!(w[e] > 1e-14 * wmax)) continue;
    const double sq = std::sqrt(w[e]);
    int big = 0;
    for (int x = 1; x < 4; ++x)
      if (std::abs(V[4 * x + e]) > std::abs(V[4 * big + e]) * (1.0 + 1e-12)) big = x;
    const cd ph = std::conj(V[4 * big + e]) / std::abs(V[4 * big + e]);
    for (int x = 0; x < 4; ++x) {
      const cd k = sq * ph * V[4 * x + e];   // K[x / 2][x % 2] = v_(a, c), x = 2 a + c
      kraus[8 * r + 2 * x] = k.real();
      kraus[8 * r + 2 * x + 1] = k.imag();
    }
    ++r;
  }
  *n_kraus = r;
  return MPSB_OK;
}

}  // extern "C"
