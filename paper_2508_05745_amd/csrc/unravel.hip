// Locally entanglement-optimal unravelling of single-qubit noise (FP64, one thread per
// noise event), the counter-based branch sampler, the per-gate event kernel of the
// trajectory sweep, the batched unravel_opt entry, and the differentiable unravelling cost
// with its hand-written adjoint.
//
// Steps of the optimal mixing (Sec. "Locally entanglement-optimal unraveling", appendix
// "Practical/closed-form version"):
//   Psi_eff = sqrt(rho_q)                     effective two-qubit state (Thm. 2 reduction)
//   phi     = [vec(K_i Psi_eff)]_i (4 x r)     induced decomposition
//   phi V   = v  (one-sided Jacobi SVD)        v = U_phi Sigma, V = V_phi
//   tau     = v^dag (Y x Y) v*                 Step 1, Takagi tau = U_T S U_T^T through the
//                                              real symmetric embedding [[A,B],[B,-A]]
//   x = v U_T, lambda_R = S (descending), C = max(0, l1 - l2 - l3 - l4)
//   C > 0:  y = x diag(1,-i,-i,-i) (Step 2), M = y^dag y~ - C y^dag y, Q_R = eig(Re M)
//           (Step 3), E = diag(1,-i,-i,-i) Q_R H4
//   C = 0:  E = diag(e^{i theta_j}) H4 with the trapezoid angles (separable case)
//   W = V[:, :rank] U_T E[:rank, :] + V[:, rank:r] E[rank:r, :]   (K'_j = sum_i W_ij K_i)
#include <float.h>

#include "common.h"
#include "kernels.h"

namespace mpsb {

using cd = c64d;

// ------------------------------------------------------------------ small helpers
__device__ inline cd cz() { return cd{0.0, 0.0}; }
__device__ inline double cabs_(cd a) { return sqrt(norm2(a)); }

// cyclic Jacobi eigen-decomposition of a real symmetric n x n matrix (n <= NMAX), in place:
// on exit a holds the eigenvalues on its diagonal, v the eigenvectors (columns).  The sweeps run
// on local copies with every index fixed at compile time (pairs and rows unrolled over NMAX,
// n as a guard), so that the matrices stay in registers rather than in per-lane scratch.  A
// pair is rotated only while its off-diagonal entry is not negligible against its diagonal
// entries (|a_pq| > eps (|a_pp| + |a_qq|) / 2), and the iteration stops after a sweep without a
// rotation (a test on the summed off-diagonal mass alone can stall above its threshold at
// rounding level and run every sweep).
template <int NMAX>
__device__ void jacobi_sym(int n, double (&a_io)[NMAX][NMAX], double (&v_io)[NMAX][NMAX]) {
  double a[NMAX][NMAX], v[NMAX][NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      a[i][j] = (i < n && j < n) ? a_io[i][j] : 0.0;
      v[i][j] = (i == j) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
#pragma unroll
      for (int j = 0; j < NMAX; ++j) {
        tot += a[i][j] * a[i][j];
        if (i != j) off += a[i][j] * a[i][j];
      }
    if (off <= 1e-34 * tot || off == 0.0) break;
    bool rotated = false;
#pragma unroll
    for (int p = 0; p < NMAX - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < NMAX; ++q) {
        const double apq = a[p][q];
        if (q < n && fabs(apq) > DBL_EPSILON * 0.5 * (fabs(a[p][p]) + fabs(a[q][q])) && fabs(apq) > 1e-300) {
          rotated = true;
          double zeta = (a[q][q] - a[p][p]) / (2.0 * apq);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
          for (int k = 0; k < NMAX; ++k) {
            double akp = a[k][p], akq = a[k][q];
            a[k][p] = c * akp - s * akq;
            a[k][q] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < NMAX; ++k) {
            double apk = a[p][k], aqk = a[q][k];
            a[p][k] = c * apk - s * aqk;
            a[q][k] = s * apk + c * aqk;
          }
#pragma unroll
          for (int k = 0; k < NMAX; ++k) {
            double vkp = v[k][p], vkq = v[k][q];
            v[k][p] = c * vkp - s * vkq;
            v[k][q] = s * vkp + c * vkq;
          }
        }
      }
    if (!rotated) break;
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (i < n && j < n) {
        a_io[i][j] = a[i][j];
        v_io[i][j] = v[i][j];
      }
}

__device__ inline cd yy_flip(const cd (&v)[4], int i) {
  // (Y x Y) v*:  [ -v3*, v2*, v1*, -v0* ]
  switch (i) {
    case 0: return cd{-v[3].re, v[3].im};
    case 1: return cd{v[2].re, -v[2].im};
    case 2: return cd{v[1].re, -v[1].im};
    default: return cd{-v[0].re, v[0].im};
  }
}

struct UnravelOut {
  cd W[4][4];     // [i][j], i < r: K'_j = sum_i W[i][j] K_i
  double p[4];
  double conc;
  int separable;
};

// ------------------------------------------------------------------ the optimal mixing
__device__ void optimal_mixing(const cd (&rho)[2][2], const cd (&K)[4][2][2], int r, UnravelOut& out) {
  // Psi_eff = sqrt(rho) for a 2x2 PSD matrix: (rho + sqrt(det) I) / sqrt(tr + 2 sqrt(det))
  double tr = rho[0][0].re + rho[1][1].re;
  double det = rho[0][0].re * rho[1][1].re - norm2(rho[0][1]);
  double sd = sqrt(fmax(det, 0.0));
  double den = sqrt(fmax(tr + 2.0 * sd, 0.0));
  cd psi[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      cd v = rho[a][b];
      if (a == b) v.re += sd;
      psi[a][b] = den > 0 ? cd{v.re / den, v.im / den} : cz();
    }
  // phi columns
  cd ph[4][4];   // [component][i]
  for (int i = 0; i < 4; ++i)
    for (int s = 0; s < 2; ++s)
      for (int e = 0; e < 2; ++e) {
        cd acc = cz();
        if (i < r)
          for (int m = 0; m < 2; ++m) cfma(acc, K[i][s][m], psi[m][e]);
        ph[2 * s + e][i] = acc;
      }
  // one-sided Jacobi: columns of ph made orthogonal, V accumulated
  cd V[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? cd{1.0, 0.0} : cz();
  // (pairs unrolled with r as a guard, so that ph and V keep compile-time indices)
  for (int sweep = 0; sweep < 30; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i + 1; j < 4; ++j) {
        if (j >= r) continue;
        double al = 0, be = 0;
        cd ga = cz();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          al += norm2(ph[c][i]);
          be += norm2(ph[c][j]);
          ga = ga + cmulc(ph[c][i], ph[c][j]);
        }
        // columns orthogonal to working precision: no rotation (a relative 1e-17 test below the
        // rounding level of the products would keep every sweep rotating)
        double g = cabs_(ga);
        if (g <= 2.0 * DBL_EPSILON * sqrt(al * be) || g == 0.0) continue;
        rotated = true;
        cd eph = {ga.re / g, -ga.im / g};   // e^{-i phi}
        double zeta = (be - al) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cd ai = ph[k][i], aj = eph * ph[k][j];
          ph[k][i] = c * ai - s * aj;
          ph[k][j] = s * ai + c * aj;
          cd vi = V[k][i], vj = eph * V[k][j];
          V[k][i] = c * vi - s * vj;
          V[k][j] = s * vi + c * vj;
        }
      }
    if (!rotated) break;
  }
  // singular values in descending order: the exchange sort of the indices, on register copies
  double sv[4];
  int ord[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s2 = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s2 += norm2(ph[c][i]);
    sv[i] = (i < r) ? sqrt(s2) : -1.0;
    ord[i] = i;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j)
      if (sv[j] > sv[i]) {
        const double tv = sv[i];
        sv[i] = sv[j];
        sv[j] = tv;
        const int ti = ord[i];
        ord[i] = ord[j];
        ord[j] = ti;
      }
  const double smax = sv[0];
  int rank = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i < r && sv[i] > 1e-12 * smax) rank++;
  cd v[4][4];    // [component][k], k < rank
  cd Vs[4][4];   // sorted V columns
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cd pv = cz(), vv = cz();
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (ord[k] == t) {
          pv = ph[c][t];
          vv = V[c][t];
        }
      v[c][k] = (k < rank) ? pv : cz();
      Vs[c][k] = vv;
    }
  // From here on every array index is fixed at compile time (loops over the padded size 4
  // or 8 with the rank as a guard, gathers by selects), so that the arrays stay in registers
  // instead of per-lane scratch memory.
  // tau = v^dag v~ (zero outside its rank x rank block)
  cd tau[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      cd vb[4] = {v[0][b], v[1][b], v[2][b], v[3][b]};
      cd acc = cz();
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = acc + cmulc(v[c][a], yy_flip(vb, c));
      tau[a][b] = (a < rank && b < rank) ? acc : cz();
    }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b) {
      cd m = {0.5 * (tau[a][b].re + tau[b][a].re), 0.5 * (tau[a][b].im + tau[b][a].im)};
      tau[a][b] = m;
      tau[b][a] = m;
    }
  // Takagi via the real embedding [[A, B], [B, -A]] of tau = A + iB in fixed blocks of 4 (the
  // rows and columns of the padding beyond the rank are zero and never rotated, so the
  // embedding of the rank block keeps its eigenpairs and the padding adds exact unit vectors)
  double E[8][8], Q[8][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      E[a][b] = tau[a][b].re;
      E[a][4 + b] = tau[a][b].im;
      E[4 + a][b] = tau[a][b].im;
      E[4 + a][4 + b] = -tau[a][b].re;
    }
  jacobi_sym<8>(8, E, Q);
  double ev8[8];
  double emax = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ev8[i] = E[i][i];
    emax = fmax(emax, fabs(ev8[i]));
  }
  // columns of U_T: the positive eigenvalues in descending order (ties: lower index), at most
  // rank of them, each eigenvector [a; b] giving the Takagi vector a + ib (unit norm)
  cd UT[4][4];
  double lam[4] = {0, 0, 0, 0};
  int kpos = 0;
  unsigned taken = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int idx = -1;
    double best = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (!((taken >> i) & 1u) && (idx < 0 || ev8[i] > best)) {
        idx = i;
        best = ev8[i];
      }
    const bool use = kpos == k && k < rank && best > 1e-12 * emax;
    double qr[4], qi[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) qr[a] = qi[a] = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i == idx) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          qr[a] = Q[a][i];
          qi[a] = Q[4 + a][i];
        }
      }
    double nn = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (a < rank) nn += qr[a] * qr[a] + qi[a] * qi[a];
    nn = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) UT[a][k] = (use && a < rank) ? cd{qr[a] * nn, qi[a] * nn} : cz();
    lam[k] = use ? best : 0.0;
    if (use) {
      kpos = k + 1;
      taken |= 1u << idx;
    }
  }
  // null directions (tau singular on the rank block): eigenvectors of the embedding with ~0
  // eigenvalue, complex Gram-Schmidt against the chosen columns, the largest residual taken
  bool nostop = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!(nostop && k == kpos && k < rank)) continue;
    double best = -1;
    cd cand[4] = {cz(), cz(), cz(), cz()};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (ev8[i] > 1e-12 * emax || ev8[i] < -1e-12 * emax) continue;
      cd u[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) u[a] = a < rank ? cd{Q[a][i], Q[4 + a][i]} : cz();
#pragma unroll
      for (int kk = 0; kk < k; ++kk) {
        cd pr = cz();
#pragma unroll
        for (int a = 0; a < 4; ++a) pr = pr + cmulc(UT[a][kk], u[a]);
#pragma unroll
        for (int a = 0; a < 4; ++a) u[a] = u[a] - pr * UT[a][kk];
      }
      double nn = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) nn += norm2(u[a]);
      if (nn > best) {
        best = nn;
#pragma unroll
        for (int a = 0; a < 4; ++a) cand[a] = u[a];
      }
    }
    if (best <= 1e-20) {
      nostop = false;
      continue;
    }
    const double inv = 1.0 / sqrt(best);
#pragma unroll
    for (int a = 0; a < 4; ++a) UT[a][k] = inv * cand[a];
    lam[k] = 0.0;
    kpos = k + 1;
  }
  // x = v U_T with the sign / phase pins: the first entry of largest modulus of column k made
  // real positive (sigma > 0: sign only; sigma = 0: its phase)
  cd x[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cd acc = cz();
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a < rank) cfma(acc, v[c][a], UT[a][k]);
      x[c][k] = k < kpos ? acc : cz();
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= kpos) continue;
    double mx = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) mx = fmax(mx, cabs_(x[c][k]));
    int i = -1;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (i < 0 && cabs_(x[c][k]) >= mx * (1.0 - 1e-12)) i = c;
    cd e = x[0][k];
#pragma unroll
    for (int c = 1; c < 4; ++c)
      if (c == i) e = x[c][k];
    const double ae = cabs_(e);
    if (ae == 0.0) continue;
    cd f;
    if (lam[k] > 0.0) f = (e.re < 0.0 || (e.re == 0.0 && e.im < 0.0)) ? cd{-1.0, 0.0} : cd{1.0, 0.0};
    else f = cd{e.re / ae, -e.im / ae};
#pragma unroll
    for (int a = 0; a < 4; ++a) UT[a][k] = UT[a][k] * f;
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c][k] = x[c][k] * f;
  }
  const double cdiff = lam[0] - lam[1] - lam[2] - lam[3];
  const double conc = fmax(0.0, cdiff);
  cd Em[4][4];   // E[a][col]
  const double h = 0.5;
  const double H4[4][4] = {{h, h, h, h}, {h, h, -h, -h}, {h, -h, h, -h}, {h, -h, -h, h}};
  if (cdiff > 0.0) {
    const cd u2[4] = {{1, 0}, {0, -1}, {0, -1}, {0, -1}};
    cd y[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) y[c][k] = x[c][k] * u2[k];
    double MR[4][4], QR[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cd yb[4] = {y[0][b], y[1][b], y[2][b], y[3][b]};
        cd s1 = cz(), s2 = cz();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s1 = s1 + cmulc(y[c][a], yy_flip(yb, c));
          s2 = s2 + cmulc(y[c][a], y[c][b]);
        }
        MR[a][b] = s1.re - conc * s2.re;
      }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a + 1; b < 4; ++b) {
        double m = 0.5 * (MR[a][b] + MR[b][a]);
        MR[a][b] = MR[b][a] = m;
      }
    jacobi_sym<4>(4, MR, QR);
    // eigenvalues ascending: the exchange sort of the indices, on register copies
    double qv[4];
    int qo[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      qv[i] = MR[i][i];
      qo[i] = i;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i + 1; j < 4; ++j)
        if (qv[j] < qv[i]) {
          const double tv = qv[i];
          qv[i] = qv[j];
          qv[j] = tv;
          const int ti = qo[i];
          qo[i] = qo[j];
          qo[j] = ti;
        }
    double Qs[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double col[4] = {0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (qo[k] == t) {
#pragma unroll
          for (int a = 0; a < 4; ++a) col[a] = QR[a][t];
        }
      double mx = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) mx = fmax(mx, fabs(col[a]));
      double lead = col[0];
      bool found = false;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (!found && fabs(col[a]) >= mx * (1.0 - 1e-12)) {
          lead = col[a];
          found = true;
        }
      const double sg = lead < 0 ? -1.0 : 1.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) Qs[a][k] = sg * col[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        double sum = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) sum += Qs[a][b] * H4[cc][b];
        Em[a][cc] = u2[a] * cd{sum, 0.0};
      }
  } else {
    double l1 = lam[0], l2 = lam[1], l3 = lam[2], l4 = lam[3];
    double th[4];
    if (l1 - l4 <= 1e-15 * fmax(l1, 1e-300)) {
      th[0] = 0; th[1] = M_PI / 4; th[2] = M_PI / 2; th[3] = 3 * M_PI / 4;
    } else {
      double base = l1 - l4, sp = 0.5 * (base + l2 + l3);
      double area2 = fmax(0.0, sp * (sp - base) * (sp - l2) * (sp - l3));
      double hh = 2.0 / base * sqrt(area2);
      double t2 = (l2 > 0) ? M_PI - asin(fmin(1.0, hh / l2)) : M_PI;
      double cr = (l4 - l1) - l2 * cos(t2), ci = -l2 * sin(t2);
      double t3 = (cr != 0.0 || ci != 0.0) ? atan2(ci, cr) : 0.0;
      th[0] = 0; th[1] = 0.5 * t2; th[2] = 0.5 * t3; th[3] = M_PI / 2;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) Em[a][cc] = cd{cos(th[a]) * H4[a][cc], sin(th[a]) * H4[a][cc]};
  }
  // W = Vs[:, :rank] U_T E[:rank] + Vs[:, rank:r] E[rank:r]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cd acc = cz();
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a < rank) {
          cd ue = cz();
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < rank) cfma(ue, UT[a][k], Em[k][j]);
          cfma(acc, Vs[i][a], ue);
        } else if (a < r) {
          cfma(acc, Vs[i][a], Em[a][j]);
        }
      }
      out.W[i][j] = i < r ? acc : cz();
    }
  out.conc = conc;
  out.separable = cdiff > 0.0 ? 0 : 1;
}

// K'_j, p_j = Tr(K'_j rho K'_j^dag)
__device__ void mixed_ops(const cd (&K)[4][2][2], int r, const cd (&W)[4][4], const cd (&rho)[2][2],
                          cd (&Kp)[4][2][2], double (&p)[4]) {
  for (int j = 0; j < 4; ++j) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        cd acc = cz();
        for (int i = 0; i < r; ++i) cfma(acc, W[i][j], K[i][a][b]);
        Kp[j][a][b] = acc;
      }
    double s = 0;
    for (int a = 0; a < 2; ++a) {
      // (K rho K^dag)[a][a] = sum_{m,n} K[a][m] rho[m][n] conj(K[a][n])
      cd acc = cz();
      for (int m = 0; m < 2; ++m)
        for (int nn = 0; nn < 2; ++nn) acc = acc + Kp[j][a][m] * rho[m][nn] * conj(Kp[j][a][nn]);
      s += acc.re;
    }
    p[j] = fmax(s, 0.0);
  }
}

__device__ void choose_mixing(int mode, const cd (&rho)[2][2], const cd (&K)[4][2][2], int r, const cd (&Ufix)[4][4],
                              cd (&W)[4][4], double& conc) {
  conc = -1.0;
  if (mode == 3) {
    UnravelOut o;
    optimal_mixing(rho, K, r, o);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) W[i][j] = o.W[i][j];
    conc = o.conc;
  } else if (mode == 1) {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) W[i][j] = (i < r) ? Ufix[j][i] : cz();
  } else {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) W[i][j] = (i == j && i < r) ? cd{1.0, 0.0} : cz();
  }
}

// ------------------------------------------------------------------ sampler
__device__ inline uint64_t splitmix64_kth(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ inline double event_uniform(uint64_t seed, uint32_t traj, uint32_t layer, uint32_t qubit) {
  uint64_t key = ((uint64_t)traj << 32) | ((uint64_t)(layer & 0xFFFF) << 16) | (uint64_t)(qubit & 0xFFFF);
  return (double)(splitmix64_kth(seed, key + 1) >> 11) * (1.0 / 9007199254740992.0);
}
__device__ inline int sample_branch(const double (&p)[4], double u) {
  double total = 0;
  for (int j = 0; j < 4; ++j) total += p[j];
  double acc = 0;
  int last = -1;
  for (int j = 0; j < 4; ++j) {
    acc += p[j];
    if (p[j] > 0.0) {
      last = j;
      if (u < acc / total) return j;
    }
  }
  return last;
}

// ------------------------------------------------------------------ event plumbing


// Channel of an event: table entry `id` when the launch reads the circuit tables, else the
// by-value slot `slot` (0: lower / single qubit, 1: upper qubit of a gate).
__device__ void load_channel(const EventArgs& ea, int slot, int id, cd (&K)[4][2][2], int& r, cd (&Uf)[4][4]) {
  const double* kd = ea.ev_ids ? ea.kraus_tab + 32LL * id : ea.kraus[slot];
  const double* ud = ea.ev_ids ? (ea.fixed_tab ? ea.fixed_tab + 32LL * id : nullptr) : ea.fixed_u[slot];
  r = ea.ev_ids ? ea.nk_tab[id] : ea.n_kraus[slot];
  for (int i = 0; i < 4; ++i)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        int o = 2 * (4 * i + 2 * a + b);
        K[i][a][b] = cd{kd[o], kd[o + 1]};
      }
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      int o = 2 * (4 * j + i);
      Uf[j][i] = ud ? cd{ud[o], ud[o + 1]} : cz();
    }
}

__device__ inline int current_layer(const EventArgs& ea) { return ea.layer_ptr ? *ea.layer_ptr : ea.layer; }

// channel id of the event on qubit x of trajectory traj in the current layer (tables), or the
// by-value slot's presence flag
__device__ inline int event_channel(const EventArgs& ea, int traj, int layer, int x, int slot_present) {
  if (ea.ev_ids) return ea.ev_ids[traj * ea.ev_traj_stride + (long long)layer * ea.ev_layer_stride + x];
  return slot_present ? 0 : -1;
}

// One noise event on a normalised single-qubit reduced state: choose W, p, draw, return the
// selected operator.  Returns -1 on a forced zero-probability branch.
__device__ int one_event(const EventArgs& ea, int slot, int id, const cd (&rho)[2][2], uint32_t traj, uint32_t layer,
                         uint32_t qubit, int forced, cd (&Ksel)[2][2], double (&p)[4], cd (&W)[4][4]) {
  cd K[4][2][2], Uf[4][4], Kp[4][2][2];
  int r;
  load_channel(ea, slot, id, K, r, Uf);
  const long long ridx = (long long)traj * ea.rec_stride + ((int)qubit - ea.rec_qbase);
  if (ea.w_in) {   // replayed mixing: W[i][j] = U[j][i]
    const double* w = ea.w_in + ridx * 32;
    for (int jj = 0; jj < 4; ++jj)
      for (int i = 0; i < 4; ++i) W[i][jj] = cd{w[2 * (4 * jj + i)], w[2 * (4 * jj + i) + 1]};
  } else {
    double conc;
    choose_mixing(ea.mode, rho, K, r, Uf, W, conc);
  }
  mixed_ops(K, r, W, rho, Kp, p);
  if (ea.branch_in && forced < 0) forced = ea.branch_in[ridx];
  int j;
  if (forced >= 0) {
    j = forced;
    if (j > 3 || !(p[j] > 0.0)) return -1;
  } else {
    j = sample_branch(p, event_uniform(ea.seed, (uint32_t)(ea.traj_base + (long long)traj), layer, qubit));
    // no branch of positive weight (a zero or non-finite state): nothing is selected
    if (j < 0) {
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) Ksel[a][b] = cz();
      return -2;
    }
  }
  double inv = 1.0 / sqrt(p[j]);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) Ksel[a][b] = inv * Kp[j][a][b];
  return j;
}

__device__ void write_record(const EventArgs& ea, int traj, int qubit, int j, const cd (&W)[4][4]) {
  const long long idx = (long long)traj * ea.rec_stride + (qubit - ea.rec_qbase);
  if (ea.branch_out) ea.branch_out[idx] = j;
  if (ea.w_out) {
    double* w = ea.w_out + idx * 32;
    // U[j][i] = W[i][j]
    for (int jj = 0; jj < 4; ++jj)
      for (int i = 0; i < 4; ++i) {
        w[2 * (4 * jj + i)] = W[i][jj].re;
        w[2 * (4 * jj + i) + 1] = W[i][jj].im;
      }
  }
}

// Gate events: reduce the theta tiles' RDM partials (fixed order), then the events of the
// lower and upper qubit; writes kops[traj] = {Ks, Kt} (normalised by 1/sqrt(p)).
constexpr int EV_SPREAD = 8;
__global__ __launch_bounds__(64) void k_gate_events(EventArgs ea, const double* __restrict__ partial, int n_tiles, int q, int has_s, int has_t,
                              double* __restrict__ kops, int* __restrict__ status) {
  // EV_SPREAD trajectories per wave (one lane each, the other lanes idle): the per-lane work
  // is a long dependent chain (the small eigensolvers of two noise events) with a large
  // register footprint, so spreading the waves over all CUs shortens the launch; 8 per wave
  // measured fastest (16 leaves half the CUs idle, 4 and 2 add waves without gain)
  if (threadIdx.x % (64 / EV_SPREAD)) return;
  int traj = blockIdx.x * EV_SPREAD + threadIdx.x / (64 / EV_SPREAD);
  if (traj >= ea.n_traj) return;
  const int layer = current_layer(ea);
  const int ch_s = event_channel(ea, traj, layer, q, has_s), ch_t = event_channel(ea, traj, layer, q + 1, has_t);
  cd rho[4][4];
  for (int x = 0; x < 16; ++x) rho[x >> 2][x & 3] = cz();
  const double* pp = partial + (long long)traj * n_tiles * 32;
  for (int t = 0; t < n_tiles; ++t)
    for (int x = 0; x < 16; ++x) {
      rho[x >> 2][x & 3].re += pp[t * 32 + 2 * x];
      rho[x >> 2][x & 3].im += pp[t * 32 + 2 * x + 1];
    }
  double tr = rho[0][0].re + rho[1][1].re + rho[2][2].re + rho[3][3].re;
  if (!(tr > 0.0) || !isfinite(tr)) { atomicOr(status, 1); tr = 1.0; }
  for (int x = 0; x < 16; ++x) rho[x >> 2][x & 3] = (1.0 / tr) * rho[x >> 2][x & 3];
  cd Ks[2][2] = {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}}, Kt[2][2] = {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}};
  double p[4];
  cd W[4][4];
  if (ch_s >= 0) {
    cd rs[2][2];
    for (int s = 0; s < 2; ++s)
      for (int s2 = 0; s2 < 2; ++s2) rs[s][s2] = rho[2 * s][2 * s2] + rho[2 * s + 1][2 * s2 + 1];
    int j = one_event(ea, 0, ch_s, rs, traj, layer, q, -1, Ks, p, W);
    if (j < 0) { atomicOr(status, j == -1 ? 2 : 1); j = 0; }
    write_record(ea, traj, q, j, W);
    // rho <- (Ks x I) rho (Ks x I)^dag  (Ks already carries 1/sqrt(p))
    cd t1[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        cd acc = cz();
        for (int s0 = 0; s0 < 2; ++s0) cfma(acc, Ks[a >> 1][s0], rho[2 * s0 + (a & 1)][b]);
        t1[a][b] = acc;
      }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        cd acc = cz();
        for (int s0 = 0; s0 < 2; ++s0) cfma_conj(acc, t1[a][2 * s0 + (b & 1)], Ks[b >> 1][s0]);
        rho[a][b] = acc;
      }
  }
  if (ch_t >= 0) {
    cd rt[2][2];
    for (int t = 0; t < 2; ++t)
      for (int t2 = 0; t2 < 2; ++t2) rt[t][t2] = rho[t][t2] + rho[2 + t][2 + t2];
    double tt = rt[0][0].re + rt[1][1].re;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) rt[a][b] = (1.0 / tt) * rt[a][b];
    int j = one_event(ea, 1, ch_t, rt, traj, layer, q + 1, -1, Kt, p, W);
    if (j < 0) { atomicOr(status, j == -1 ? 2 : 1); j = 0; }
    write_record(ea, traj, q + 1, j, W);
  }
  double* ko = kops + (long long)traj * 16;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      ko[2 * (2 * a + b)] = Ks[a][b].re;
      ko[2 * (2 * a + b) + 1] = Ks[a][b].im;
      ko[8 + 2 * (2 * a + b)] = Kt[a][b].re;
      ko[8 + 2 * (2 * a + b) + 1] = Kt[a][b].im;
    }
}

// Single-site event on the centre tensor: rho1 [traj][2][2] c128 (unnormalised) -> kops
// (first 2x2 block = selected operator, second = identity).
__global__ __launch_bounds__(64) void k_site_event(EventArgs ea, const double* __restrict__ rho1, int q, int ch /* slot */, const int* __restrict__ forced,
                             double* __restrict__ kops, double* __restrict__ p_out, int* __restrict__ status) {
  int traj = blockIdx.x * blockDim.x + threadIdx.x;
  if (traj >= ea.n_traj) return;
  const int layer = current_layer(ea);
  const int id = event_channel(ea, traj, layer, q, 1);
  double* ko = kops + (long long)traj * 16;
  if (id < 0) {   // no event on this trajectory: identity
    for (int x = 0; x < 16; ++x) ko[x] = (x == 0 || x == 6 || x == 8 || x == 14) ? 1.0 : 0.0;
    return;
  }
  cd rho[2][2];
  const double* r = rho1 + traj * 8;
  for (int x = 0; x < 4; ++x) rho[x >> 1][x & 1] = cd{r[2 * x], r[2 * x + 1]};
  double tr = rho[0][0].re + rho[1][1].re;
  if (!(tr > 0.0) || !isfinite(tr)) { atomicOr(status, 1); tr = 1.0; }
  for (int x = 0; x < 4; ++x) rho[x >> 1][x & 1] = (1.0 / tr) * rho[x >> 1][x & 1];
  cd Ks[2][2];
  double p[4];
  cd W[4][4];
  int f = forced ? forced[traj] : -1;
  int j = one_event(ea, ch, id, rho, traj, layer, q, f, Ks, p, W);
  if (j < 0) {
    atomicOr(status, j == -1 ? 2 : 1);
    Ks[0][0] = cd{1, 0}; Ks[0][1] = cz(); Ks[1][0] = cz(); Ks[1][1] = cd{1, 0};
    j = 0;
  }
  write_record(ea, traj, q, j, W);
  if (p_out)
    for (int jj = 0; jj < 4; ++jj) p_out[traj * 4 + jj] = p[jj];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      ko[2 * (2 * a + b)] = Ks[a][b].re;
      ko[2 * (2 * a + b) + 1] = Ks[a][b].im;
      ko[8 + 2 * (2 * a + b)] = (a == b) ? 1.0 : 0.0;
      ko[8 + 2 * (2 * a + b) + 1] = 0.0;
    }
}

// Forced-branch feasibility check (run before any state change): flags status bit 2 when
// a forced branch has zero probability.
__global__ __launch_bounds__(64) void k_site_event_check(EventArgs ea, const double* __restrict__ rho1, int ch, const int* __restrict__ forced,
                                   int* __restrict__ status) {
  int traj = blockIdx.x * blockDim.x + threadIdx.x;
  if (traj >= ea.n_traj || !forced || forced[traj] < 0) return;
  cd rho[2][2];
  const double* r = rho1 + traj * 8;
  for (int x = 0; x < 4; ++x) rho[x >> 1][x & 1] = cd{r[2 * x], r[2 * x + 1]};
  double tr = rho[0][0].re + rho[1][1].re;
  if (!(tr > 0.0)) { atomicOr(status, 1); return; }
  for (int x = 0; x < 4; ++x) rho[x >> 1][x & 1] = (1.0 / tr) * rho[x >> 1][x & 1];
  cd K[4][2][2], Uf[4][4], Kp[4][2][2], W[4][4];
  int rr;
  load_channel(ea, ch, 0, K, rr, Uf);
  double conc, p[4];
  choose_mixing(ea.mode, rho, K, rr, Uf, W, conc);
  mixed_ops(K, rr, W, rho, Kp, p);
  if (!(p[forced[traj]] > 0.0)) atomicOr(status, 2);
}

// ------------------------------------------------------------------ unravel_opt
// An item whose channel id lies outside 0..n_k-1 reads no channel: its U, p and eof are NaN.
__global__ __launch_bounds__(64) void k_unravel_opt(int batch, const double* __restrict__ rho_q, const double* __restrict__ kraus,
                              int n_k, const int* __restrict__ kraus_id, int r, double* __restrict__ U,
                              double* __restrict__ p_out, double* __restrict__ eof) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int kid = kraus_id ? kraus_id[b] : 0;
  if (kid < 0 || kid >= n_k) {
    const double nan = __builtin_nan("");
    for (int j = 0; j < 4; ++j) {
      p_out[b * 4 + j] = nan;
      for (int i = 0; i < 2 * r; ++i) U[((long long)b * 4 + j) * r * 2 + i] = nan;
    }
    eof[b] = nan;
    return;
  }
  cd rho[2][2];
  for (int x = 0; x < 4; ++x) rho[x >> 1][x & 1] = cd{rho_q[b * 8 + 2 * x], rho_q[b * 8 + 2 * x + 1]};
  cd K[4][2][2];
  for (int i = 0; i < 4; ++i)
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        if (i < r) {
          const double* kp = kraus + ((long long)kid * r + i) * 8 + 2 * (2 * a + c);
          K[i][a][c] = cd{kp[0], kp[1]};
        } else K[i][a][c] = cz();
      }
  UnravelOut o;
  optimal_mixing(rho, K, r, o);
  cd Kp[4][2][2];
  double p[4];
  mixed_ops(K, r, o.W, rho, Kp, p);
  for (int j = 0; j < 4; ++j) {
    p_out[b * 4 + j] = p[j];
    for (int i = 0; i < r; ++i) {
      U[((long long)b * 4 + j) * r * 2 + 2 * i] = o.W[i][j].re;
      U[((long long)b * 4 + j) * r * 2 + 2 * i + 1] = o.W[i][j].im;
    }
  }
  double c = fmin(fmax(o.conc, 0.0), 1.0);
  double x = 0.5 * (1.0 + sqrt(fmax(0.0, 1.0 - c * c)));
  double h = 0;
  if (x > 0 && x < 1) h = -x * log2(x) - (1 - x) * log2(1 - x);
  eof[b] = h;
}

hipError_t launch_unravel_opt(int batch, const double* rho_q, const double* kraus, int n_k, const int* kraus_id, int r,
                              double* U, double* p, double* eof, hipStream_t st) {
  hipLaunchKernelGGL(k_unravel_opt, dim3((batch + 63) / 64), dim3(64), 0, st, batch, rho_q, kraus, n_k, kraus_id, r, U, p,
                     eof);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Born sampling
// Sampling of computational-basis outcomes from each trajectory's state, site by site, with
// the centre at site 0 (the rest right-orthonormal): W = V A_k holds, for every sample, the
// left vector of its drawn prefix times the site tensor, [S][s][b] per trajectory; the
// conditional probability of s_k = s is ||W_s||^2 / (||W_0||^2 + ||W_1||^2) (FP64 sums in
// index order); the draw is the counter uniform keyed by (trajectory, sample, site) of the
// sampling seed; V <- W_s / ||W_s||.  One thread per (trajectory, sample).
template <typename T>
__global__ void k_born_init(cplx<T>* V, long long sV, int S, int n_traj) {
  const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (g >= (long long)n_traj * S) return;
  V[(g / S) * sV + g % S] = cplx<T>{(T)1, (T)0};
}

template <typename T>
__global__ void k_born_step(const cplx<T>* __restrict__ W, long long sW, int S, int dr, cplx<T>* __restrict__ V,
                            long long sV, uint8_t* __restrict__ bits, int n, int k, uint64_t seed, long long traj_base,
                            int n_traj) {
  const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (g >= (long long)n_traj * S) return;
  const long long t = g / S;
  const int i = (int)(g % S);
  const cplx<T>* w = W + t * sW + (long long)i * 2 * dr;
  double p0 = 0.0, p1 = 0.0;
  for (int b = 0; b < dr; ++b) p0 += (double)w[b].re * w[b].re + (double)w[b].im * w[b].im;
  for (int b = 0; b < dr; ++b) p1 += (double)w[dr + b].re * w[dr + b].re + (double)w[dr + b].im * w[dr + b].im;
  const double tot = p0 + p1;
  const double u = event_uniform(seed, (uint32_t)(traj_base + t), (uint32_t)i, (uint32_t)k);
  const int s = (tot > 0.0 && !(u < p0 / tot)) ? 1 : 0;
  const double ps = s ? p1 : p0;
  const double sc = ps > 0.0 ? 1.0 / sqrt(ps) : 0.0;
  bits[g * n + k] = (uint8_t)s;
  cplx<T>* v = V + t * sV + (long long)i * dr;
  for (int b = 0; b < dr; ++b) v[b] = cplx<T>{(T)(sc * w[s * dr + b].re), (T)(sc * w[s * dr + b].im)};
}

hipError_t born_init(int prec, void* V, long long sV, int S, int n_traj, hipStream_t st) {
  const int nb = (int)(((long long)n_traj * S + 255) / 256);
  if (prec == 0) hipLaunchKernelGGL(k_born_init<float>, dim3(nb), dim3(256), 0, st, (c32*)V, sV, S, n_traj);
  else hipLaunchKernelGGL(k_born_init<double>, dim3(nb), dim3(256), 0, st, (c64d*)V, sV, S, n_traj);
  return hipGetLastError();
}

hipError_t born_step(int prec, const void* W, long long sW, int S, int dr, void* V, long long sV, uint8_t* bits, int n,
                     int k, uint64_t seed, long long traj_base, int n_traj, hipStream_t st) {
  const int nb = (int)(((long long)n_traj * S + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_born_step<float>, dim3(nb), dim3(256), 0, st, (const c32*)W, sW, S, dr, (c32*)V, sV, bits, n, k,
                       seed, traj_base, n_traj);
  else
    hipLaunchKernelGGL(k_born_step<double>, dim3(nb), dim3(256), 0, st, (const c64d*)W, sW, S, dr, (c64d*)V, sV, bits,
                       n, k, seed, traj_base, n_traj);
  return hipGetLastError();
}

hipError_t launch_gate_events(const EventArgs& ea, const double* partial, int n_tiles, int q, int has_s, int has_t,
                              double* kops, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_gate_events, dim3((ea.n_traj + EV_SPREAD - 1) / EV_SPREAD), dim3(64), 0, st, ea, partial, n_tiles, q, has_s, has_t,
                     kops, status);
  return hipGetLastError();
}

hipError_t launch_site_event(const EventArgs& ea, const double* rho1, int q, int ch, const int* forced, double* kops,
                             double* p_out, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_site_event, dim3((ea.n_traj + 63) / 64), dim3(64), 0, st, ea, rho1, q, ch, forced, kops, p_out,
                     status);
  return hipGetLastError();
}

hipError_t launch_site_event_check(const EventArgs& ea, const double* rho1, int ch, const int* forced, int* status,
                                   hipStream_t st) {
  hipLaunchKernelGGL(k_site_event_check, dim3((ea.n_traj + 63) / 64), dim3(64), 0, st, ea, rho1, ch, forced, status);
  return hipGetLastError();
}

}  // namespace mpsb
