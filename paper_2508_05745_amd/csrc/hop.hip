// Centre hop by Cholesky factorisation of the Gram matrix (LDS-resident, FP64).
//
// Left-to-right hop of the orthogonality centre from site j to j+1: C_j (rows (a,s), n = chi_R
// columns) = Q R with E = C^dag C = R^dag R (upper-triangular R); Q = C R^{-1} replaces C_j in
// place (row by row, a wave per row) and R is written out for C_{j+1} = R B_{j+1}.
// Right-to-left hop from j to j-1: C_j (n = chi_L rows, 2 chi_R columns) = R^dag Q with
// E = C C^dag = R^dag R; Q = R^{-dag} C replaces C_j (column by column) and R is written out
// for C_{j-1} = A_{j-1} R^dag.
// Pivots below tol * max(diag E) are dropped (the row of R and the column of R^{-1} become
// zero): such directions carry no weight of the state.
#include "common.h"
#include "kernels.h"

namespace mpsb {

constexpr int HT = 512;

__device__ inline int pk(int i, int k, int n) { return i * n - (i * (i - 1)) / 2 + (k - i); }   // packed upper

template <typename T, int NMAX>
__global__ __launch_bounds__(HT) void k_hop_chol(int n, int left_to_right, int other, const c64d* __restrict__ Eg,
                                                 long long sE, cplx<T>* __restrict__ C, long long sC,
                                                 cplx<T>* __restrict__ Rout, long long sR, double tol) {
  __shared__ c64d R[NMAX * (NMAX + 1) / 2];
  __shared__ double piv[NMAX];
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
      __syncthreads();   // everyone has read the pivot before row c is rewritten
      for (int k = c + tid; k < n; k += HT) {
        c64d v = R[pk(c, k, n)];
        R[pk(c, k, n)] = keep ? (k == c ? c64d{r, 0.0} : c64d{v.re / r, v.im / r}) : c64d{0, 0};
      }
      if (tid == 0) piv[c] = r;
      __syncthreads();
      // rows c+1 .. c0+cb-1 of the panel: E[i][k] -= conj(R[c][i]) R[c][k], i <= k
      if (keep) {
        const int rows = c0 + cb - (c + 1), m = n - (c + 1);
        for (int e = tid; e < rows * m; e += HT) {
          const int i = c + 1 + e / m, k = c + 1 + e % m;
          if (k >= i) R[pk(i, k, n)] = R[pk(i, k, n)] - cmulc(R[pk(c, i, n)], R[pk(c, k, n)]);
        }
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
  // triangular solves, one wave per group of VG vectors solved together (independent chains
  // share the broadcasts of R); lane owns entries lane + 64 s
  constexpr int SL = NMAX / 64, VG = 8;
  const int nvec = other;
  for (int v0 = VG * wv; v0 < nvec; v0 += VG * (HT / 64)) {
    c64d x[VG][SL];
    // load the vectors: L->R: row vidx of C (length n, contiguous); R->L: column vidx of C,
    // conjugated (C^dag row), stride `other`
#pragma unroll
    for (int g = 0; g < VG; ++g)
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int k = lane + 64 * s, vidx = v0 + g;
        cplx<T> v = {0, 0};
        if (k < n && vidx < nvec) v = left_to_right ? Cj[(long long)vidx * n + k] : Cj[(long long)k * other + vidx];
        x[g][s] = left_to_right ? c64d{(double)v.re, (double)v.im} : c64d{(double)v.re, -(double)v.im};
      }
    // solve q R = x: q_k = (x_k - sum_{i<k} q_i R[i][k]) / R[k][k], column-oriented updates
    for (int k = 0; k < n; ++k) {
      const int owner = k & 63, slot = k >> 6;
      const double rkk = piv[k];
      const double inv = rkk > 0 ? 1.0 / rkk : 0.0;
      c64d qk[VG];
#pragma unroll
      for (int g = 0; g < VG; ++g) {
        c64d xk = {0, 0};
#pragma unroll
        for (int s = 0; s < SL; ++s)
          if (s == slot) xk = x[g][s];
        xk.re = __shfl(xk.re, owner, 64);
        xk.im = __shfl(xk.im, owner, 64);
        qk[g] = c64d{xk.re * inv, xk.im * inv};
      }
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        if (64 * s + 63 < k) continue;   // slot already solved (wave-uniform)
        const int j = lane + 64 * s;
        if (j == k) {
#pragma unroll
          for (int g = 0; g < VG; ++g) x[g][s] = qk[g];
        } else if (j > k && j < n && rkk > 0) {
          const c64d rkj = R[pk(k, j, n)];
#pragma unroll
          for (int g = 0; g < VG; ++g) x[g][s] = x[g][s] - qk[g] * rkj;
        }
      }
    }
#pragma unroll
    for (int g = 0; g < VG; ++g)
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int k = lane + 64 * s, vidx = v0 + g;
        if (k < n && vidx < nvec) {
          if (left_to_right) Cj[(long long)vidx * n + k] = cplx<T>{(T)x[g][s].re, (T)x[g][s].im};
          else Cj[(long long)k * other + vidx] = cplx<T>{(T)x[g][s].re, (T)(-x[g][s].im)};
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
