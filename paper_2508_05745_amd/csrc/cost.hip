// Expected entanglement of an unravelling as a differentiable function of the Kraus mixing,
// and its hand-written adjoint.
//
// Forward (per state): rho_q[s][s'] = sum_{a,t,b} theta[a,s,t,b] conj(theta[a,s',t,b])
// (HBM-bound reduction, FP64 accumulation), U = exp(iH) U_ref with H = sum_k params_k L_k,
// K'_j = sum_i U_ji K_i, sigma~_j = K'_j rho K'_j^dag, p_j = Tr sigma~_j, P_j = Tr sigma~_j^2,
//   f_lin = sum_j (p_j - P_j / p_j),   f_R2 = sum_j -p_j log2(P_j / p_j^2).
// Adjoint: G[j][i] = df/dU_ji (holomorphic part), M = U_ref G^T, and with the Frechet
// derivative L of the matrix exponential, df/dparams_k = 2 Re Tr(L(X^dag, M^dag)^dag i L_k),
// X = iH; L(X^dag, M^dag) is the upper-right block of exp([[X^dag, M^dag], [0, X^dag]]).
#include "common.h"
#include "kernels.h"

namespace mpsb {

using cd = c64d;

// ------------------------------------------------------------------ rho_q reduction
// One workgroup per state.  Thread e takes elements 2e, 2e + 1 of a row (t, b) run (two
// complex values per vector load, 2 chi_r even), at rows a and a + ... of both s planes; the
// row / column position advances by a fixed step, so the loop divides nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_cost_rho(int chi_l, int chi_r, const cplx<T>* __restrict__ theta, double* rho) {
  __shared__ double red[4][4];
  const long long per = (long long)chi_l * 4 * chi_r;
  const cplx<T>* th = theta + blockIdx.x * per;
  const int w = 2 * chi_r;        // (t,b) run length
  const int w2 = chi_r;           // pairs per run
  const int tot = chi_l * w2;     // pairs per s plane
  const int da = 256 / w2, dr = 256 % w2;
  int a = threadIdx.x / w2, r = threadIdx.x % w2;
  double r00 = 0, r11 = 0, r01r = 0, r01i = 0;
  for (int e = threadIdx.x; e < tot; e += 256) {
    const cplx<T>* p0 = th + (long long)a * 2 * w + 2 * r;
    const cplx<T> x0 = p0[0], y0 = p0[1], x1 = p0[w], y1 = p0[w + 1];
    const double a0 = x0.re, b0 = x0.im, a1 = x1.re, b1 = x1.im;
    const double c0 = y0.re, d0 = y0.im, c1 = y1.re, d1 = y1.im;
    r00 += (a0 * a0 + b0 * b0) + (c0 * c0 + d0 * d0);
    r11 += (a1 * a1 + b1 * b1) + (c1 * c1 + d1 * d1);
    r01r += (a0 * a1 + b0 * b1) + (c0 * c1 + d0 * d1);   // x0 conj(x1)
    r01i += (b0 * a1 - a0 * b1) + (d0 * c1 - c0 * d1);
    a += da;
    r += dr;
    if (r >= w2) {
      r -= w2;
      ++a;
    }
  }
  double v[4] = {r00, r11, r01r, r01i};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int x = 0; x < 4; ++x) {
    double s = v[x];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wv][x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[4];
    for (int x = 0; x < 4; ++x) s[x] = red[0][x] + red[1][x] + red[2][x] + red[3][x];
    double* o = rho + blockIdx.x * 8;
    o[0] = s[0]; o[1] = 0;
    o[2] = s[2]; o[3] = s[3];
    o[4] = s[2]; o[5] = -s[3];
    o[6] = s[1]; o[7] = 0;
  }
}

hipError_t cost_rho(int batch, const void* theta, int chi_l, int chi_r, int prec, double* rho, hipStream_t st) {
  if (prec == 0) hipLaunchKernelGGL(k_cost_rho<float>, dim3(batch), dim3(256), 0, st, chi_l, chi_r, (const c32*)theta, rho);
  else hipLaunchKernelGGL(k_cost_rho<double>, dim3(batch), dim3(256), 0, st, chi_l, chi_r, (const c64d*)theta, rho);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small complex matrices
template <int N>
__device__ void mm(const cd (&a)[N][N], const cd (&b)[N][N], cd (&c)[N][N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cd s = {0, 0};
      for (int k = 0; k < N; ++k) cfma(s, a[i][k], b[k][j]);
      c[i][j] = s;
    }
}

// exp(A) by scaling and squaring with a degree-18 Taylor polynomial (||A/2^s||_1 <= 1/4).
template <int N>
__device__ void expm(const cd (&a)[N][N], cd (&out)[N][N]) {
  double nrm = 0;
  for (int j = 0; j < N; ++j) {
    double c = 0;
    for (int i = 0; i < N; ++i) c += sqrt(norm2(a[i][j]));
    nrm = fmax(nrm, c);
  }
  int s = 0;
  while (nrm > 0.25 && s < 60) { nrm *= 0.5; ++s; }
  const double sc = ldexp(1.0, -s);
  cd x[N][N], term[N][N], tmp[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      x[i][j] = sc * a[i][j];
      term[i][j] = (i == j) ? cd{1, 0} : cd{0, 0};
      out[i][j] = term[i][j];
    }
  for (int k = 1; k <= 18; ++k) {
    mm<N>(term, x, tmp);
    const double f = 1.0 / k;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        term[i][j] = f * tmp[i][j];
        out[i][j] = out[i][j] + term[i][j];
      }
  }
  for (int k = 0; k < s; ++k) {
    mm<N>(out, out, tmp);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) out[i][j] = tmp[i][j];
  }
}

__device__ void generator(int k, cd (&g)[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) g[i][j] = cd{0, 0};
  const int pj[6] = {0, 0, 0, 1, 1, 2}, pk[6] = {1, 2, 3, 2, 3, 3};
  if (k < 4) g[k][k] = cd{1, 0};
  else if (k < 10) { int a = pj[k - 4], b = pk[k - 4]; g[a][b] = cd{1, 0}; g[b][a] = cd{1, 0}; }
  else { int a = pj[k - 10], b = pk[k - 10]; g[b][a] = cd{0, 1}; g[a][b] = cd{0, -1}; }
}

struct CostState {
  cd U[4][4], Kp[4][2][2], K[4][2][2], rho[2][2], sig[4][2][2];
  double p[4], P[4];
};

__device__ void cost_setup(const double* rho_in, const double* kraus, const double* params, const double* uref,
                           CostState& cs, cd (&Xh)[4][4]) {
  for (int x = 0; x < 4; ++x) cs.rho[x >> 1][x & 1] = cd{rho_in[2 * x], rho_in[2 * x + 1]};
  // normalise rho (the reduction of an unnormalised theta is allowed)
  double tr = cs.rho[0][0].re + cs.rho[1][1].re;
  for (int x = 0; x < 4; ++x) cs.rho[x >> 1][x & 1] = (1.0 / tr) * cs.rho[x >> 1][x & 1];
  for (int i = 0; i < 4; ++i)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) cs.K[i][a][b] = cd{kraus[2 * (4 * i + 2 * a + b)], kraus[2 * (4 * i + 2 * a + b) + 1]};
  cd H[4][4], X[4][4], E[4][4], Ur[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      H[i][j] = cd{0, 0};
      Ur[i][j] = cd{uref[2 * (4 * i + j)], uref[2 * (4 * i + j) + 1]};
    }
  for (int k = 0; k < 16; ++k) {
    cd g[4][4];
    generator(k, g);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) H[i][j] = H[i][j] + params[k] * g[i][j];
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) X[i][j] = cd{-H[i][j].im, H[i][j].re};   // iH
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Xh[i][j] = conj(X[j][i]);                // (iH)^dag
  expm<4>(X, E);
  mm<4>(E, Ur, cs.U);
  for (int j = 0; j < 4; ++j) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        cd s = {0, 0};
        for (int i = 0; i < 4; ++i) cfma(s, cs.U[j][i], cs.K[i][a][b]);
        cs.Kp[j][a][b] = s;
      }
    // sigma~ = K' rho K'^dag
    cd t[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        cd s = {0, 0};
        for (int m = 0; m < 2; ++m) cfma(s, cs.Kp[j][a][m], cs.rho[m][b]);
        t[a][b] = s;
      }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        cd s = {0, 0};
        for (int m = 0; m < 2; ++m) cfma_conj(s, t[a][m], cs.Kp[j][b][m]);
        cs.sig[j][a][b] = s;
      }
    cs.p[j] = cs.sig[j][0][0].re + cs.sig[j][1][1].re;
    double P = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) P += (cs.sig[j][a][b] * cs.sig[j][b][a]).re;
    cs.P[j] = P;
  }
}

constexpr double P_TINY = 1e-300;
constexpr double LN2 = 0.69314718055994530942;

__global__ void k_cost_eval(int batch, const double* rho, const double* kraus, const double* params, const double* uref,
                            int kind, double* f) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  CostState cs;
  cd Xh[4][4];
  cost_setup(rho + b * 8, kraus, params + b * 16, uref + b * 32, cs, Xh);
  double acc = 0;
  for (int j = 0; j < 4; ++j) {
    double p = cs.p[j], P = cs.P[j];
    if (!(p > P_TINY)) continue;
    if (kind == 0) acc += p - P / p;
    else acc += -p * log(P / (p * p)) / LN2;
  }
  f[b] = acc;
}

__global__ void k_cost_grad(int batch, const double* rho, const double* kraus, const double* params, const double* uref,
                            int kind, const double* grad_f, double* grad) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  CostState cs;
  cd Xh[4][4];
  cost_setup(rho + b * 8, kraus, params + b * 16, uref + b * 32, cs, Xh);
  // G[j][i] = g_p Tr(K_i rho K'_j^dag) + g_P 2 Tr(sigma~_j K_i rho K'_j^dag)
  cd G[4][4];
  for (int j = 0; j < 4; ++j) {
    double p = cs.p[j], P = cs.P[j];
    double gp = 0, gP = 0;
    if (p > P_TINY) {
      if (kind == 0) { gp = 1.0 + P / (p * p); gP = -1.0 / p; }
      else { gp = -log(P / (p * p)) / LN2 + 2.0 / LN2; gP = -p / (P * LN2); }
    }
    for (int i = 0; i < 4; ++i) {
      // B = K_i rho K'_j^dag
      cd t[2][2], B[2][2];
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
          cd s = {0, 0};
          for (int m = 0; m < 2; ++m) cfma(s, cs.K[i][a][m], cs.rho[m][c]);
          t[a][c] = s;
        }
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
          cd s = {0, 0};
          for (int m = 0; m < 2; ++m) cfma_conj(s, t[a][m], cs.Kp[j][c][m]);
          B[a][c] = s;
        }
      cd trB = B[0][0] + B[1][1];
      cd trSB = {0, 0};
      for (int a = 0; a < 2; ++a)
        for (int m = 0; m < 2; ++m) trSB = trSB + cs.sig[j][a][m] * B[m][a];
      G[j][i] = gp * trB + (2.0 * gP) * trSB;
    }
  }
  // M = U_ref G^T ; block exponential for L(X^dag, M^dag)
  cd Ur[4][4], Mt[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Ur[i][j] = cd{uref[b * 32 + 2 * (4 * i + j)], uref[b * 32 + 2 * (4 * i + j) + 1]};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd s = {0, 0};
      for (int k = 0; k < 4; ++k) cfma(s, Ur[i][k], G[j][k]);
      Mt[i][j] = s;
    }
  cd Bk[8][8], Eb[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) Bk[i][j] = cd{0, 0};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      Bk[i][j] = Xh[i][j];
      Bk[4 + i][4 + j] = Xh[i][j];
      Bk[i][4 + j] = conj(Mt[j][i]);   // M^dag
    }
  expm<8>(Bk, Eb);
  const double gf = grad_f ? grad_f[b] : 1.0;
  for (int k = 0; k < 16; ++k) {
    cd g[4][4];
    generator(k, g);
    // Tr(Y^dag i g) = sum_{a,c} conj(Y[a][c]) (i g[a][c])
    cd s = {0, 0};
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) s = s + cmulc(Eb[a][4 + c], cd{-g[a][c].im, g[a][c].re});
    grad[b * 16 + k] = gf * 2.0 * s.re;
  }
}

hipError_t cost_eval(int batch, const double* rho, const double* kraus, const double* params, const double* u_ref,
                     int kind, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_cost_eval, dim3((batch + 63) / 64), dim3(64), 0, st, batch, rho, kraus, params, u_ref, kind, f);
  return hipGetLastError();
}

hipError_t cost_grad(int batch, const double* rho, const double* kraus, const double* params, const double* u_ref,
                     int kind, const double* grad_f, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_cost_grad, dim3((batch + 63) / 64), dim3(64), 0, st, batch, rho, kraus, params, u_ref, kind,
                     grad_f, grad);
  return hipGetLastError();
}

}  // namespace mpsb
