// Centre hop by Cholesky factorisation of the Gram matrix (LDS-resident, FP64).
//
// Left-to-right hop of the orthogonality centre from site j to j+1: C_j (rows (a,s), n = chi_R
// columns) = Q R with E = C^dag C = R^dag R (upper-triangular R); R is written out for
// C_{j+1} = R B_{j+1}, inverted in place in LDS, and Q = C R^{-1} replaces C_j in place.
// Right-to-left hop from j to j-1: C_j (n = chi_L rows, 2 chi_R columns) = R^dag Q with
// E = C C^dag = R^dag R; R is written out for C_{j-1} = A_{j-1} R^dag and Q = R^{-dag} C
// replaces C_j.  The products with R^{-1} run on f64 MFMA over its nonzero triangle (a
// triangular solve per vector spent most of its time moving broadcasts, not computing).
// Pivots below tol * max(diag E) are dropped (the row of R and the row and column of R^{-1}
// become zero): such directions carry no weight of the state.
#include "common.h"
#include "kernels.h"

namespace mpsb {

constexpr int HT = 512;

// a double from another lane of the same quad (DPP quad_perm: 0xB1 = lane ^ 1, 0x4E = lane ^ 2)
template <int CTRL>
__device__ inline double quad_xor(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

typedef double v4d_t __attribute__((ext_vector_type(4)));
__device__ inline v4d_t mfma64(double a, double b, v4d_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

__device__ inline int pk(int i, int k, int n) { return i * n - (i * (i - 1)) / 2 + (k - i); }   // packed upper

template <typename T, int NMAX>
__global__ __launch_bounds__(HT) void k_hop_chol(int n, int left_to_right, int other, const c64d* __restrict__ Eg,
                                                 long long sE, cplx<T>* __restrict__ C, long long sC,
                                                 cplx<T>* __restrict__ Rout, long long sR, double tol) {
  __shared__ c64d R[NMAX * (NMAX + 1) / 2];
  __shared__ double piv[NMAX], ipiv[NMAX];   // pivots R[c][c] and their inverses (0 if dropped)
  __shared__ c64d tcol[NMAX];                 // a column of each diagonal block of R while it is inverted
  __shared__ double red[HT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const c64d* E = Eg + blockIdx.x * sE;
  cplx<T>* Cj = C + blockIdx.x * sC;
  cplx<T>* Ro = Rout + blockIdx.x * sR;
  // load the upper triangle, find max diagonal
  double dm = 0;
  for (int i = wv; i < n; i += HT / 64)
    for (int k = i + lane; k < n; k += 64) {
      c64d v = E[(long long)i * n + k];
      R[pk(i, k, n)] = v;
      if (k == i) dm = fmax(dm, v.re);
    }
  for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_down(dm, off, 64));
  if (lane == 0) red[wv] = dm;
  __syncthreads();
  double dmax = 0;
  for (int w = 0; w < HT / 64; ++w) dmax = fmax(dmax, red[w]);
  const double cut = tol * dmax;
  // blocked right-looking Cholesky E = R^dag R: panels of CB rows are factored column by
  // column (updates confined to the panel), then the trailing upper triangle takes the
  // rank-CB update in 4 x 4 register tiles
  constexpr int CB = 8;
  for (int c0 = 0; c0 < n; c0 += CB) {
    const int cb = min(CB, n - c0);
    for (int c = c0; c < c0 + cb; ++c) {
      __syncthreads();   // previous updates complete
      const double p = R[pk(c, c, n)].re;
      const bool keep = p > cut && p > 0.0;
      const double r = keep ? sqrt(p) : 0.0;
      // row c past the diagonal; the pivot itself is overwritten after the next barrier, once
      // every thread has read it (nothing below reads it)
      for (int k = c + 1 + tid; k < n; k += HT) {
        c64d v = R[pk(c, k, n)];
        R[pk(c, k, n)] = keep ? c64d{v.re / r, v.im / r} : c64d{0, 0};
      }
      if (tid == 0) {
        piv[c] = r;
        ipiv[c] = keep ? 1.0 / r : 0.0;
      }
      __syncthreads();
      if (tid == 0) R[pk(c, c, n)] = c64d{r, 0.0};
      // rows c+1 .. c0+cb-1 of the panel, a wave per row: E[i][k] -= conj(R[c][i]) R[c][k], k >= i
      if (keep) {
        for (int i = c + 1 + wv; i < c0 + cb; i += HT / 64)
          for (int k = i + lane; k < n; k += 64) R[pk(i, k, n)] = R[pk(i, k, n)] - cmulc(R[pk(c, i, n)], R[pk(c, k, n)]);
      }
    }
    __syncthreads();
    // trailing update, rows and columns >= t0 = c0 + cb, upper triangle in 4 x 4 tiles
    const int t0 = c0 + cb, m = n - t0;
    if (m <= 0) continue;
    const int nt = (m + 3) / 4, ntiles = nt * (nt + 1) / 2;
    for (int t = tid; t < ntiles; t += HT) {
      // tile (ti, tk), tk >= ti, linear index t = tk (tk + 1) / 2 + ti
      int tk = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      while (tk * (tk + 1) / 2 > t) --tk;
      while ((tk + 1) * (tk + 2) / 2 <= t) ++tk;
      const int ti = t - tk * (tk + 1) / 2;
      const int i0 = t0 + 4 * ti, k0 = t0 + 4 * tk;
      c64d acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = c64d{0, 0};
      for (int c = c0; c < t0; ++c) {
        if (!(piv[c] > 0.0)) continue;
        c64d ri[4], rk[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          ri[a] = (i0 + a < n) ? R[pk(c, i0 + a, n)] : c64d{0, 0};
          rk[a] = (k0 + a < n) ? R[pk(c, k0 + a, n)] : c64d{0, 0};
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = acc[a][b] + cmulc(ri[a], rk[b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, k = k0 + b;
          if (i < n && k < n && k >= i) R[pk(i, k, n)] = R[pk(i, k, n)] - acc[a][b];
        }
    }
  }
  __syncthreads();
  // R out (upper, zeros below), precision of the state
  for (int i = wv; i < n; i += HT / 64)
    for (int k = lane; k < n; k += 64) {
      c64d v = k >= i ? R[pk(i, k, n)] : c64d{0, 0};
      Ro[(long long)i * n + k] = cplx<T>{(T)v.re, (T)v.im};
    }
  // R^{-1} in place (upper triangle, packed), by 16 x 16 blocks.  For R = [[A, B], [0, C]] the
  // inverse is [[A^-1, -(A^-1 B) C^-1], [0, C^-1]]: the diagonal blocks are inverted together,
  // column by column (column jj of a block's inverse is -(1 / R[j][j]) X[., 0:jj] R[0:jj, jj]
  // within the block), then block column J above the diagonal becomes -(X[0:a, 0:a] R[0:a, J])
  // X_JJ with a = 16 J, for J = 1, 2, ... in turn.  A dropped pivot (1 / R[j][j] taken as 0)
  // gives a zero row and column, so the products below leave those directions out exactly as
  // the substitution would.
  __syncthreads();   // R has been written out
  const int nbk = (n + 15) / 16;
  static_assert(HT >= 16 * (NMAX / 16), "a thread per row of every diagonal block");
  {
    const int b = tid >> 4, ii = tid & 15, r0 = 16 * b;
    const int bs = b < nbk ? min(16, n - r0) : 0;
    for (int jj = 0; jj < 16; ++jj) {
      if (ii < jj && jj < bs) tcol[r0 + ii] = R[pk(r0 + ii, r0 + jj, n)];
      __syncthreads();
      if (jj < bs) {
        const int i = r0 + ii, j = r0 + jj;
        const double dj = ipiv[j];
        if (ii < jj) {
          double yr0 = 0.0, yi0 = 0.0, yr1 = 0.0, yi1 = 0.0;
          int l = ii;
          for (; l + 1 < jj; l += 2) {
            const c64d a0 = R[pk(i, r0 + l, n)], x0 = tcol[r0 + l], a1 = R[pk(i, r0 + l + 1, n)], x1 = tcol[r0 + l + 1];
            yr0 = fma(a0.re, x0.re, yr0);
            yr0 = fma(-a0.im, x0.im, yr0);
            yi0 = fma(a0.re, x0.im, yi0);
            yi0 = fma(a0.im, x0.re, yi0);
            yr1 = fma(a1.re, x1.re, yr1);
            yr1 = fma(-a1.im, x1.im, yr1);
            yi1 = fma(a1.re, x1.im, yi1);
            yi1 = fma(a1.im, x1.re, yi1);
          }
          if (l < jj) {
            const c64d a0 = R[pk(i, r0 + l, n)], x0 = tcol[r0 + l];
            yr0 = fma(a0.re, x0.re, yr0);
            yr0 = fma(-a0.im, x0.im, yr0);
            yi0 = fma(a0.re, x0.im, yi0);
            yi0 = fma(a0.im, x0.re, yi0);
          }
          R[pk(i, j, n)] = c64d{-dj * (yr0 + yr1), -dj * (yi0 + yi1)};
        } else if (ii == jj) {
          R[pk(j, j, n)] = c64d{dj, 0.0};
        }
      }
      __syncthreads();
    }
  }
  // block columns J >= 1: element (i, jj) of the a x 16 block above the diagonal in thread
  // (16 i + jj) mod HT, at most four per thread (a <= NMAX - 16)
  constexpr int PER = ((NMAX - 16) * 16 + HT - 1) / HT;
  for (int J = 1; J < nbk; ++J) {
    const int a = 16 * J, cw = min(16, n - a);
    c64d yv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + HT * q, i = e >> 4, jj = e & 15;
      double yr0 = 0.0, yi0 = 0.0, yr1 = 0.0, yi1 = 0.0;
      if (i < a && jj < cw) {
        // Y[i][jj] = sum_{l = i}^{a-1} X[i][l] R[l][a + jj]
        const int base = pk(i, i, n) - i;   // X[i][l] = R[base + l], l >= i
        int l = i;
        for (; l + 1 < a; l += 2) {
          const c64d x0 = R[base + l], r0v = R[pk(l, a + jj, n)], x1 = R[base + l + 1], r1v = R[pk(l + 1, a + jj, n)];
          yr0 = fma(x0.re, r0v.re, yr0);
          yr0 = fma(-x0.im, r0v.im, yr0);
          yi0 = fma(x0.re, r0v.im, yi0);
          yi0 = fma(x0.im, r0v.re, yi0);
          yr1 = fma(x1.re, r1v.re, yr1);
          yr1 = fma(-x1.im, r1v.im, yr1);
          yi1 = fma(x1.re, r1v.im, yi1);
          yi1 = fma(x1.im, r1v.re, yi1);
        }
        if (l < a) {
          const c64d x0 = R[base + l], r0v = R[pk(l, a + jj, n)];
          yr0 = fma(x0.re, r0v.re, yr0);
          yr0 = fma(-x0.im, r0v.im, yr0);
          yi0 = fma(x0.re, r0v.im, yi0);
          yi0 = fma(x0.im, r0v.re, yi0);
        }
      }
      yv[q] = c64d{yr0 + yr1, yi0 + yi1};
    }
    __syncthreads();   // block column J of R has been read
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + HT * q, i = e >> 4, jj = e & 15;
      if (i < a && jj < cw) R[pk(i, a + jj, n)] = yv[q];
    }
    __syncthreads();
    // X[i][a + jj] = -sum_{m <= jj} Y[i][m] X_JJ[m][jj]
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + HT * q, i = e >> 4, jj = e & 15;
      double xr = 0.0, xi = 0.0;
      if (i < a && jj < cw) {
        for (int m = 0; m <= jj; ++m) {
          const c64d y = R[pk(i, a + m, n)], z = R[pk(a + m, a + jj, n)];
          xr = fma(y.re, z.re, xr);
          xr = fma(-y.im, z.im, xr);
          xi = fma(y.re, z.im, xi);
          xi = fma(y.im, z.re, xi);
        }
      }
      yv[q] = c64d{-xr, -xi};
    }
    __syncthreads();   // Y has been read
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + HT * q, i = e >> 4, jj = e & 15;
      if (i < a && jj < cw) R[pk(i, a + jj, n)] = yv[q];
    }
    __syncthreads();
  }
  // Q = C R^{-1} (L->R, C: other x n, row-major) or Q = R^{-dag} C (R->L, C: n x other), in
  // place, on f64 MFMA over the nonzero triangle of R^{-1}.  A wave owns 16 rows (L->R) or
  // 16 columns (R->L) of C with all their output tiles in registers, so it reads those rows /
  // columns completely before it writes them.  Lane layout (f64 16x16x4): A[i][k] in lane
  // i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), register i / 4.
  const int i16 = lane & 15, kq = lane >> 4;
  constexpr int NT16 = NMAX / 16;
  const int nt = (n + 15) / 16;
  if (left_to_right) {
    const int nvt = (other + 15) / 16;
    for (int vt = wv; vt < nvt; vt += HT / 64) {
      v4d_t ar[NT16], ai[NT16];
#pragma unroll
      for (int t = 0; t < NT16; ++t) ar[t] = ai[t] = v4d_t{0, 0, 0, 0};
      const int v = 16 * vt + i16;
      for (int l0 = 0; l0 < n; l0 += 4) {
        const int l = l0 + kq;
        cplx<T> cv = {0, 0};
        if (v < other && l < n) cv = Cj[(long long)v * n + l];
        const double cr = (double)cv.re, ci = (double)cv.im;
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
          if (t < nt && l0 <= 16 * t + 15) {   // Rinv[l][c] = 0 for l > c
            const int c = 16 * t + i16;
            const c64d b = (l < n && c < n && l <= c) ? R[pk(l, c, n)] : c64d{0, 0};
            ar[t] = mfma64(cr, b.re, ar[t]);
            ar[t] = mfma64(-ci, b.im, ar[t]);
            ai[t] = mfma64(cr, b.im, ai[t]);
            ai[t] = mfma64(ci, b.re, ai[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT16; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * vt + kq + 4 * q, c = 16 * t + i16;
          if (t < nt && row < other && c < n) Cj[(long long)row * n + c] = cplx<T>{(T)ar[t][q], (T)ai[t][q]};
        }
    }
  } else {
    const int nvt = (other + 15) / 16;
    for (int vt = wv; vt < nvt; vt += HT / 64) {
      v4d_t ar[NT16], ai[NT16];
#pragma unroll
      for (int t = 0; t < NT16; ++t) ar[t] = ai[t] = v4d_t{0, 0, 0, 0};
      const int v = 16 * vt + i16;
      for (int l0 = 0; l0 < n; l0 += 4) {
        const int l = l0 + kq;
        cplx<T> cv = {0, 0};
        if (v < other && l < n) cv = Cj[(long long)l * other + v];
        const double br = (double)cv.re, bi = (double)cv.im;
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
          if (t < nt && l0 <= 16 * t + 15) {   // conj(Rinv[l][r]) = 0 for l > r
            const int r = 16 * t + i16;
            const c64d a = (l < n && r < n && l <= r) ? R[pk(l, r, n)] : c64d{0, 0};
            // A[r][l] = conj(Rinv[l][r])
            ar[t] = mfma64(a.re, br, ar[t]);
            ar[t] = mfma64(a.im, bi, ar[t]);
            ai[t] = mfma64(a.re, bi, ai[t]);
            ai[t] = mfma64(-a.im, br, ai[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT16; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * t + kq + 4 * q, col = 16 * vt + i16;
          if (t < nt && r < n && col < other) Cj[(long long)r * other + col] = cplx<T>{(T)ar[t][q], (T)ai[t][q]};
        }
    }
  }
}

hipError_t hop_chol(int prec, int n, int left_to_right, int other, const void* E, long long sE, void* C, long long sC,
                    void* Rout, long long sR, double tol, int n_traj, hipStream_t st) {
  if (n > 128) return hipErrorInvalidValue;
  if (prec == 0)
    hipLaunchKernelGGL((k_hop_chol<float, 128>), dim3(n_traj), dim3(HT), 0, st, n, left_to_right, other,
                       (const c64d*)E, sE, (c32*)C, sC, (c32*)Rout, sR, tol);
  else
    hipLaunchKernelGGL((k_hop_chol<double, 128>), dim3(n_traj), dim3(HT), 0, st, n, left_to_right, other,
                       (const c64d*)E, sE, (c64d*)C, sC, (c64d*)Rout, sR, tol);
  return hipGetLastError();
}

}  // namespace mpsb
