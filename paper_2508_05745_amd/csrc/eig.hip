// Batched FP64 Hermitian eigensolver for the truncation Gram matrices and the centre hops.
//
// For each matrix (one workgroup per matrix and phase):
//   E1  Householder reduction to tridiagonal form, A = Q T Q^dag, Q = H_0 H_1 ... H_{n-3},
//       H_j = I - 2 u_j u_j^dag; the reflector vectors overwrite the strict upper triangle;
//   E2  a diagonal phase similarity makes T real symmetric; the `keep` largest
//       eigenvalues by Sturm-count bisection (one thread per eigenvalue); eigenvectors of
//       the real tridiagonal by inverse iteration with partial-pivoting LU (one thread
//       per eigenvalue); eigenvalues <= zero_tol * lambda_max are dropped (value 0, vector
//       0: such directions carry no weight of the state);
//   E3  CholeskyQR2 orthonormalisation of the kept vectors (restores orthogonality inside
//       clusters of close eigenvalues);
//   E4  back-transformation evec = Q diag(omega) X with blocked compact-WY reflectors.
// Outputs: eigenvalues (descending), eigenvectors n x keep (row-major, ld keep) c128,
// the trace of the input and the sum of the kept eigenvalues.
#include <float.h>

#include "common.h"
#include "kernels.h"

namespace mpsb {

constexpr int ET = 256;           // threads per workgroup
constexpr int EMAX = 512;         // largest matrix dimension

__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < ET / 64; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------- E1
__global__ __launch_bounds__(ET) void k_tridiag(int n, c64d* __restrict__ Ag, long long sA, double* __restrict__ ws,
                                                long long sW) {
  __shared__ c64d su[EMAX], sp[EMAX];
  __shared__ double red[ET / 64];
  __shared__ double s_scal[4];
  c64d* A = Ag + blockIdx.x * sA;
  double* W = ws + blockIdx.x * sW;
  double* d = W;                          // [n]
  c64d* ec = (c64d*)(W + n);              // [n]   subdiagonal T[j+1][j] (complex)
  double* tr = W + 3 * n;                 // [1]   trace
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // trace of the input
  double t = 0;
  for (int i = tid; i < n; i += ET) t += A[(long long)i * n + i].re;
  t = block_sum(t, red);
  if (tid == 0) tr[0] = t;

  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const c64d* row = A + (long long)j * n + (j + 1);
    // alpha = ||x||, x_i = conj(A[j][j+1+i])
    double s2 = 0;
    for (int i = tid; i < m; i += ET) s2 += norm2(row[i]);
    s2 = block_sum(s2, red);
    const double alpha = sqrt(s2);
    const c64d x0 = conj(row[0]);
    const double ax0 = sqrt(norm2(x0));
    if (alpha <= 1e-300) {
      // nothing to annihilate: H = I
      for (int i = tid; i < m; i += ET) A[(long long)j * n + j + 1 + i] = c64d{0, 0};
      if (tid == 0) ec[j] = x0;
      __syncthreads();
      continue;
    }
    const c64d ph = ax0 > 0 ? c64d{x0.re / ax0, x0.im / ax0} : c64d{1.0, 0.0};
    const double vn = sqrt(2.0 * alpha * (alpha + ax0));
    __syncthreads();
    for (int i = tid; i < m; i += ET) {
      c64d xi = conj(row[i]);
      if (i == 0) xi = xi + alpha * ph;
      su[i] = c64d{xi.re / vn, xi.im / vn};
    }
    __syncthreads();
    // p = A22 u, one wave per row
    for (int i = wv; i < m; i += ET / 64) {
      const c64d* r = A + (long long)(j + 1 + i) * n + (j + 1);
      double pr = 0, pi = 0;
      for (int k = lane; k < m; k += 64) {
        c64d a = r[k], u = su[k];
        pr += a.re * u.re - a.im * u.im;
        pi += a.re * u.im + a.im * u.re;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        pr += __shfl_down(pr, off, 64);
        pi += __shfl_down(pi, off, 64);
      }
      if (lane == 0) sp[i] = c64d{pr, pi};
    }
    __syncthreads();
    // K = Re(u^dag p); w = p - K u (kept in sp)
    double kk = 0;
    for (int i = tid; i < m; i += ET) kk += su[i].re * sp[i].re + su[i].im * sp[i].im;
    kk = block_sum(kk, red);
    for (int i = tid; i < m; i += ET) sp[i] = sp[i] - kk * su[i];
    __syncthreads();
    // A22 -= 2 (u w^dag + w u^dag)
    for (int i = wv; i < m; i += ET / 64) {
      const c64d ui = su[i], wi = sp[i];
      c64d* r = A + (long long)(j + 1 + i) * n + (j + 1);
      for (int k = lane; k < m; k += 64) {
        c64d uk = su[k], wk = sp[k];
        c64d upd = ui * conj(wk) + wi * conj(uk);
        r[k] = r[k] - 2.0 * upd;
      }
    }
    // keep u in row j, the subdiagonal element in ec
    for (int i = tid; i < m; i += ET) A[(long long)j * n + j + 1 + i] = su[i];
    if (tid == 0) ec[j] = c64d{-ph.re * alpha, -ph.im * alpha};
    __syncthreads();
  }
  if (n >= 2 && tid == 0) ec[n - 2] = conj(A[(long long)(n - 2) * n + (n - 1)]);
  if (tid == 0 && n >= 2) {
    // the last reflector slot (row n-2) holds no reflector
    A[(long long)(n - 2) * n + (n - 1)] = c64d{0, 0};
  }
  __syncthreads();
  for (int i = tid; i < n; i += ET) d[i] = A[(long long)i * n + i].re;
}

// ---------------------------------------------------------------------------- E2
// Sturm count: number of eigenvalues of the real symmetric tridiagonal (d, e) below x.
__device__ inline int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
}

__device__ inline uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(ET) void k_tri_eig(int n, int keep, double zero_tol, double* __restrict__ ws, long long sW,
                                                double* __restrict__ evals, long long sE, double* __restrict__ kept_sum) {
  __shared__ double sd[EMAX], se[EMAX], se2[EMAX];
  __shared__ double red[ET / 64];
  __shared__ double s_bounds[2];
  double* W = ws + blockIdx.x * sW;
  double* d = W;
  c64d* ec = (c64d*)(W + n);
  c64d* om = (c64d*)(W + 4 * n);            // [n] phases omega
  double* X = W + 6 * n;                    // [n][keep]   vectors (component-major)
  double* U0 = X + (long long)n * keep;     // [n][keep]   LU factors
  double* U1 = U0 + (long long)n * keep;
  double* U2 = U1 + (long long)n * keep;
  double* L = U2 + (long long)n * keep;
  double* PV = L + (long long)n * keep;
  double* ev = evals + blockIdx.x * sE;
  const int tid = threadIdx.x;

  for (int i = tid; i < n; i += ET) {
    sd[i] = d[i];
    double a = (i + 1 < n) ? sqrt(norm2(ec[i])) : 0.0;
    se[i] = a;
    se2[i] = a * a;
  }
  __syncthreads();
  if (tid == 0) {
    c64d w = {1.0, 0.0};
    om[0] = w;
    for (int i = 0; i + 1 < n; ++i) {
      double a = se[i];
      if (a > 0) {
        c64d ph = {ec[i].re / a, ec[i].im / a};
        w = w * ph;
      }
      om[i + 1] = w;
    }
    double lo = 1e300, hi = -1e300, emax2 = 0;
    for (int i = 0; i < n; ++i) {
      double r = (i > 0 ? se[i - 1] : 0.0) + (i + 1 < n ? se[i] : 0.0);
      lo = fmin(lo, sd[i] - r);
      hi = fmax(hi, sd[i] + r);
      if (i + 1 < n) emax2 = fmax(emax2, se2[i]);
    }
    double nrm = fmax(fabs(lo), fabs(hi));
    lo -= 2 * DBL_EPSILON * nrm + 1e-300;
    hi += 2 * DBL_EPSILON * nrm + 1e-300;
    s_bounds[0] = lo;
    s_bounds[1] = hi;
  }
  __syncthreads();
  const double glo = s_bounds[0], ghi = s_bounds[1];
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  double emax2 = 0;
  for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, se2[i]);
  const double pivmin = DBL_MIN * fmax(1.0, emax2);

  // ---- bisection for the keep largest eigenvalues
  for (int k = tid; k < keep; k += ET) {
    const int idx = n - 1 - k;   // ascending index
    double lo = glo, hi = ghi;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin || mid <= lo || mid >= hi) break;
      if (sturm_count(n, sd, se2, mid, pivmin) <= idx) lo = mid; else hi = mid;
    }
    ev[k] = 0.5 * (lo + hi);
  }
  __syncthreads();
  const double lmax = ev[0];
  const double cut = fmax(zero_tol * fmax(lmax, 0.0), 1e-300);

  // ---- inverse iteration, one thread per kept eigenvalue
  for (int k = tid; k < keep; k += ET) {
    const double lam = ev[k];
    const bool drop = !(lam > cut);
    if (drop) {
      for (int i = 0; i < n; ++i) X[(long long)i * keep + k] = 0.0;
      continue;
    }
    // perturb the shift by a relative eps so that the factorisation is never exactly singular
    const double sig = lam + 4.0 * DBL_EPSILON * tnorm * (1.0 + 0.37 * (k & 7));
    const double tiny = DBL_EPSILON * tnorm + 1e-300;
    // LU with partial pivoting of T - sig I
    double cd = sd[0] - sig, cs = (n > 1) ? se[0] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = se[i], nd = sd[i + 1] - sig, ns = (i + 2 < n) ? se[i + 1] : 0.0;
      const long long o = (long long)i * keep + k;
      if (fabs(cd) >= fabs(sub)) {
        double l = (cd != 0.0) ? sub / cd : 0.0;
        U0[o] = (cd != 0.0) ? cd : tiny;
        U1[o] = cs;
        U2[o] = 0.0;
        L[o] = l;
        PV[o] = 0.0;
        cd = nd - l * cs;
        cs = ns;
      } else {
        double l = cd / sub;
        U0[o] = sub;
        U1[o] = nd;
        U2[o] = ns;
        L[o] = l;
        PV[o] = 1.0;
        cd = cs - l * nd;
        cs = -l * ns;
      }
    }
    U0[(long long)(n - 1) * keep + k] = (cd != 0.0) ? cd : tiny;
    // start vector: deterministic pseudo-random in [0.5, 1.5)
    for (int i = 0; i < n; ++i)
      X[(long long)i * keep + k] = 0.5 + (hash32((uint32_t)(i * 7919 + k * 104729 + 17)) >> 8) * (1.0 / 16777216.0);
    for (int itr = 0; itr < 3; ++itr) {
      if (itr > 0) {
        // apply P and L^{-1}
        for (int i = 0; i + 1 < n; ++i) {
          const long long o = (long long)i * keep + k;
          double xi = X[o], xn = X[o + keep];
          if (PV[o] != 0.0) { double tmp = xi; xi = xn; xn = tmp; }
          xn -= L[o] * xi;
          X[o] = xi;
          X[o + keep] = xn;
        }
      }
      // U^{-1}
      double y1 = 0.0, y2 = 0.0, mx = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        const long long o = (long long)i * keep + k;
        double y = (X[o] - U1[o] * y1 - U2[o] * y2) / U0[o];
        if (i == n - 1) y = X[o] / U0[o];
        else if (i == n - 2) y = (X[o] - U1[o] * y1) / U0[o];
        X[o] = y;
        y2 = y1;
        y1 = y;
        mx = fmax(mx, fabs(y));
      }
      double sc = (mx > 0) ? 1.0 / mx : 1.0;
      double nn = 0;
      for (int i = 0; i < n; ++i) {
        const long long o = (long long)i * keep + k;
        double y = X[o] * sc;
        X[o] = y;
        nn += y * y;
      }
      double inv = 1.0 / sqrt(nn);
      for (int i = 0; i < n; ++i) X[(long long)i * keep + k] *= inv;
    }
  }
  __syncthreads();
  // zero the dropped eigenvalues, kept sum
  double s = 0;
  for (int k = tid; k < keep; k += ET) {
    double lam = ev[k];
    if (!(lam > cut)) { lam = 0.0; ev[k] = 0.0; }
    s += lam;
  }
  s = block_sum(s, red);
  if (tid == 0 && kept_sum) kept_sum[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------- E3
// CholeskyQR2 of the n x keep real matrix X (component-major), zero columns left alone.
__global__ __launch_bounds__(ET) void k_cholqr(int n, int keep, double* __restrict__ ws, long long sW,
                                               double* __restrict__ gws, long long sG) {
  double* W = ws + blockIdx.x * sW;
  double* X = W + 6 * n;
  double* G = gws + blockIdx.x * sG;     // keep x keep
  const int tid = threadIdx.x;
  __shared__ double piv[EMAX];
  for (int pass = 0; pass < 2; ++pass) {
    // G = X^T X (lower + diag)
    const int kk = keep * keep;
    for (int e = tid; e < kk; e += ET) {
      int a = e / keep, b = e % keep;
      if (b > a) continue;
      double s = 0;
      for (int i = 0; i < n; ++i) s += X[(long long)i * keep + a] * X[(long long)i * keep + b];
      G[(long long)a * keep + b] = s;
    }
    __syncthreads();
    // right-looking Cholesky of the lower triangle; zero / dependent pivots -> column dropped
    for (int c = 0; c < keep; ++c) {
      double g = G[(long long)c * keep + c];
      __syncthreads();
      bool ok = g > 1e-28;
      double r = ok ? sqrt(g) : 0.0;
      if (tid == 0) piv[c] = r;
      for (int i = c + 1 + tid; i < keep; i += ET) G[(long long)i * keep + c] = ok ? G[(long long)i * keep + c] / r : 0.0;
      __syncthreads();
      const int m = keep - c - 1;
      const int mm = m * m;
      for (int e = tid; e < mm; e += ET) {
        int i = c + 1 + e / m, l = c + 1 + e % m;
        if (l > i) continue;
        G[(long long)i * keep + l] -= G[(long long)i * keep + c] * G[(long long)l * keep + c];
      }
      __syncthreads();
    }
    // X <- X R^{-1}, R = L^T, one thread per row of X
    for (int i = tid; i < n; i += ET) {
      double* xr = X + (long long)i * keep;
      for (int c = 0; c < keep; ++c) {
        double v = xr[c];
        for (int l = 0; l < c; ++l) v -= xr[l] * G[(long long)c * keep + l];
        xr[c] = (piv[c] > 0) ? v / piv[c] : 0.0;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- E4
// evec = Q diag(omega) X, Q = H_0 ... H_{n-3}; reflectors applied in blocks of NB from the
// last block to the first as (I - V T V^dag).
constexpr int NB = 16;
__global__ __launch_bounds__(ET) void k_backtransform(int n, int keep, const c64d* __restrict__ Ag, long long sA,
                                                      double* __restrict__ ws, long long sW,
                                                      c64d* __restrict__ Zg, long long sZ) {
  __shared__ c64d Tm[NB][NB];
  __shared__ c64d Sv[NB][NB];
  __shared__ c64d Wt[NB][EMAX / 2];        // NB x keep (keep <= 256)
  const c64d* A = Ag + blockIdx.x * sA;
  double* W = ws + blockIdx.x * sW;
  const c64d* om = (const c64d*)(W + 4 * n);
  const double* X = W + 6 * n;
  c64d* Z = Zg + blockIdx.x * sZ;
  const int tid = threadIdx.x;
  // Z = diag(omega) X
  for (int i = 0; i < n; ++i)
    for (int c = tid; c < keep; c += ET) {
      double x = X[(long long)i * keep + c];
      Z[(long long)i * keep + c] = c64d{om[i].re * x, om[i].im * x};
    }
  __syncthreads();
  const int nref = n - 2;   // reflectors j = 0 .. n-3
  if (nref <= 0) return;
  const int nblk = (nref + NB - 1) / NB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = blk * NB, nb = min(NB, nref - j0);
    // u_j (column jj of V) lives in row j of A at columns j+1..n-1; V[i][jj] = A[j][i] for i > j
    // S = V^dag V
    for (int e = tid; e < nb * nb; e += ET) {
      int a = e / nb, b = e % nb;
      int ja = j0 + a, jb = j0 + b;
      int start = max(ja, jb) + 1;
      c64d s = {0, 0};
      for (int i = start; i < n; ++i) s = s + cmulc(A[(long long)ja * n + i], A[(long long)jb * n + i]);
      Sv[a][b] = s;
    }
    __syncthreads();
    if (tid == 0) {
      // T upper triangular: T_jj = 2, T[0:j, j] = -2 T[0:j, 0:j] S[0:j, j]
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) Tm[a][b] = c64d{0, 0};
      for (int jj = 0; jj < nb; ++jj) {
        for (int a = 0; a < jj; ++a) {
          c64d s = {0, 0};
          for (int b = a; b < jj; ++b) s = s + Tm[a][b] * Sv[b][jj];
          Tm[a][jj] = -2.0 * s;
        }
        Tm[jj][jj] = c64d{2.0, 0.0};
      }
    }
    __syncthreads();
    // Wt = V^dag Z  (nb x keep)
    for (int e = tid; e < nb * keep; e += ET) {
      int a = e / keep, c = e % keep;
      int ja = j0 + a;
      c64d s = {0, 0};
      for (int i = ja + 1; i < n; ++i) s = s + cmulc(A[(long long)ja * n + i], Z[(long long)i * keep + c]);
      Wt[a][c] = s;
    }
    __syncthreads();
    // Wt = T Wt (upper triangular, in place top-down)
    for (int c = tid; c < keep; c += ET) {
      c64d tmp[NB];
      for (int a = 0; a < nb; ++a) {
        c64d s = {0, 0};
        for (int b = a; b < nb; ++b) s = s + Tm[a][b] * Wt[b][c];
        tmp[a] = s;
      }
      for (int a = 0; a < nb; ++a) Wt[a][c] = tmp[a];
    }
    __syncthreads();
    // Z -= V Wt
    for (int i = j0 + 1; i < n; ++i) {
      const int amax = min(nb, i - j0);   // V[i][a] nonzero only if i > j0 + a
      for (int c = tid; c < keep; c += ET) {
        c64d s = {0, 0};
        for (int a = 0; a < amax; ++a) s = s + A[(long long)(j0 + a) * n + i] * Wt[a][c];
        Z[(long long)i * keep + c] = Z[(long long)i * keep + c] - s;
      }
    }
    __syncthreads();
  }
}

size_t heev_ws_doubles(int n, int keep) { return (size_t)6 * n + (size_t)6 * n * keep + 64; }
size_t heev_gws_doubles(int keep) { return (size_t)keep * keep + 64; }

hipError_t heev_phase(int phase, int n, int keep, double zero_tol, void* A, long long sA, double* ws, long long sW,
                      double* gws, long long sG, double* evals, long long sE, double* kept_sum, void* Z, long long sZ,
                      int batch, hipStream_t st) {
  if (n > EMAX || keep > n || keep > EMAX / 2) return hipErrorInvalidValue;
  switch (phase) {
    case 0: hipLaunchKernelGGL(k_tridiag, dim3(batch), dim3(ET), 0, st, n, (c64d*)A, sA, ws, sW); break;
    case 1: hipLaunchKernelGGL(k_tri_eig, dim3(batch), dim3(ET), 0, st, n, keep, zero_tol, ws, sW, evals, sE, kept_sum); break;
    case 2: hipLaunchKernelGGL(k_cholqr, dim3(batch), dim3(ET), 0, st, n, keep, ws, sW, gws, sG); break;
    default: hipLaunchKernelGGL(k_backtransform, dim3(batch), dim3(ET), 0, st, n, keep, (const c64d*)A, sA, ws, sW, (c64d*)Z, sZ); break;
  }
  return hipGetLastError();
}

// trace of the input is kept at ws[3n] by E1
}  // namespace mpsb
