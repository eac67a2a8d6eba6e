// Small kernels of the sweep: single-site reduced states and operator application for idle-
// qubit events, truncation / hop scale factors, precision widening, and the observable
// traces and the fixed-order reduction over trajectories.
#include "common.h"
#include "kernels.h"

namespace mpsb {

static inline int nblocks(long long total, int bs = 256) {
  long long b = (total + bs - 1) / bs;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

// rho1[traj][s][s'] = sum_{a,b} A[a][s][b] conj(A[a][s'][b])  (one workgroup per trajectory)
template <typename T>
__global__ void k_site_rdm(int chi_l, int chi_r, const cplx<T>* __restrict__ site, long long s_traj, double* rho1) {
  __shared__ double red[4][8];
  const cplx<T>* A = site + blockIdx.x * s_traj;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long tot = (long long)chi_l * chi_r;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    int a = (int)(e / chi_r), b = (int)(e % chi_r);
    cplx<T> v0 = A[(long long)a * 2 * chi_r + b], v1 = A[(long long)a * 2 * chi_r + chi_r + b];
    double r0 = v0.re, i0 = v0.im, r1 = v1.re, i1 = v1.im;
    acc[0] += r0 * r0 + i0 * i0;          // [0][0]
    acc[2] += r0 * r1 + i0 * i1;          // [0][1] re
    acc[3] += i0 * r1 - r0 * i1;          // [0][1] im
    acc[6] += r1 * r1 + i1 * i1;          // [1][1]
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int x = 0; x < 8; ++x) {
    double v = acc[x];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[8];
    for (int x = 0; x < 8; ++x) s[x] = red[0][x] + red[1][x] + red[2][x] + red[3][x];
    double* o = rho1 + blockIdx.x * 8;
    o[0] = s[0]; o[1] = 0.0;
    o[2] = s[2]; o[3] = s[3];
    o[4] = s[2]; o[5] = -s[3];
    o[6] = s[6]; o[7] = 0.0;
  }
}

hipError_t site_rdm(int prec, int chi_l, int chi_r, const void* site, long long s_traj, double* rho1, int n_traj,
                    hipStream_t st) {
  if (prec == 0) hipLaunchKernelGGL(k_site_rdm<float>, dim3(n_traj), dim3(256), 0, st, chi_l, chi_r, (const c32*)site, s_traj, rho1);
  else hipLaunchKernelGGL(k_site_rdm<double>, dim3(n_traj), dim3(256), 0, st, chi_l, chi_r, (const c64d*)site, s_traj, rho1);
  return hipGetLastError();
}

// A[a][s][b] <- sum_s0 K[s][s0] A[a][s0][b]
template <typename T>
__global__ void k_site_apply(int chi_l, int chi_r, cplx<T>* site, long long s_traj, const double* __restrict__ kops,
                             int n_traj) {
  const long long per = (long long)chi_l * chi_r, total = per * n_traj;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    int traj = (int)(e / per);
    long long r = e % per;
    int a = (int)(r / chi_r), b = (int)(r % chi_r);
    cplx<T>* A = site + traj * s_traj;
    const double* k = kops + (long long)traj * 16;
    cplx<T> v0 = A[(long long)a * 2 * chi_r + b], v1 = A[(long long)a * 2 * chi_r + chi_r + b];
    double o[2][2];
    for (int s = 0; s < 2; ++s) {
      double k0r = k[2 * (2 * s)], k0i = k[2 * (2 * s) + 1], k1r = k[2 * (2 * s + 1)], k1i = k[2 * (2 * s + 1) + 1];
      o[s][0] = k0r * v0.re - k0i * v0.im + k1r * v1.re - k1i * v1.im;
      o[s][1] = k0r * v0.im + k0i * v0.re + k1r * v1.im + k1i * v1.re;
    }
    A[(long long)a * 2 * chi_r + b] = cplx<T>{(T)o[0][0], (T)o[0][1]};
    A[(long long)a * 2 * chi_r + chi_r + b] = cplx<T>{(T)o[1][0], (T)o[1][1]};
  }
}

hipError_t site_apply(int prec, int chi_l, int chi_r, void* site, long long s_traj, const double* kops, int n_traj,
                      hipStream_t st) {
  int nb = nblocks((long long)chi_l * chi_r * n_traj);
  if (prec == 0) hipLaunchKernelGGL(k_site_apply<float>, dim3(nb), dim3(256), 0, st, chi_l, chi_r, (c32*)site, s_traj, kops, n_traj);
  else hipLaunchKernelGGL(k_site_apply<double>, dim3(nb), dim3(256), 0, st, chi_l, chi_r, (c64d*)site, s_traj, kops, n_traj);
  return hipGetLastError();
}

// alpha = 1/sqrt(kept); discarded = (trace - kept) / trace (trace kept by the eigensolver at
// ws[3n] of each matrix)
__global__ void k_trunc_factors(const double* kept, const double* ws, long long sW, int n, double* alpha,
                                double* discarded, int disc_stride, int accumulate, int n_traj) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_traj) return;
  double k = kept[t], tr = ws[t * sW + 3 * n];
  alpha[t] = k > 0 ? 1.0 / sqrt(k) : 0.0;
  double eps = tr > 0 ? fmax(tr - k, 0.0) / tr : 0.0;
  if (discarded) {
    double* d = discarded + (long long)t * disc_stride;
    *d = accumulate ? *d + eps : eps;
  }
}

hipError_t trunc_factors(const double* kept, const double* ws, long long sW, int n, double* alpha, double* discarded,
                         int disc_stride, int accumulate, int n_traj, hipStream_t st) {
  hipLaunchKernelGGL(k_trunc_factors, dim3((n_traj + 255) / 256), dim3(256), 0, st, kept, ws, sW, n, alpha, discarded,
                     disc_stride, accumulate, n_traj);
  return hipGetLastError();
}

// Entanglement entropy (base 2) of a bond from the eigenvalues of its Gram matrix (the
// squared Schmidt coefficients up to normalisation): S = log2 N - (1/N) sum_k l_k log2 l_k,
// N = sum_k l_k, over the first `keep` values (dropped ones are 0); one thread per
// trajectory, sums in index order.
__global__ void k_bond_entropy(const double* __restrict__ ev, long long sE, int keep, double* __restrict__ out,
                               int stride, int n_traj) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_traj) return;
  const double* e = ev + t * sE;
  double nrm = 0.0, a = 0.0;
  for (int k = 0; k < keep; ++k) {
    const double l = e[k];
    if (l > 0.0) {
      nrm += l;
      a = fma(l, log2(l), a);
    }
  }
  out[(long long)t * stride] = nrm > 0.0 ? fmax(log2(nrm) - a / nrm, 0.0) : 0.0;
}

hipError_t bond_entropy(const double* ev, long long sE, int keep, double* out, int stride, int n_traj, hipStream_t st) {
  hipLaunchKernelGGL(k_bond_entropy, dim3((n_traj + 255) / 256), dim3(256), 0, st, ev, sE, keep, out, stride, n_traj);
  return hipGetLastError();
}

// zero columns [c0, c0+w) of rows x ld matrices (prec)
template <typename T>
__global__ void k_zero_cols(cplx<T>* X, long long sX, int rows, int ld, int c0, int w, int n_traj) {
  long long per = (long long)rows * w, total = per * n_traj;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    int t = (int)(e / per);
    long long r = e % per;
    int i = (int)(r / w), j = (int)(r % w);
    X[t * sX + (long long)i * ld + c0 + j] = cplx<T>{(T)0, (T)0};
  }
}

hipError_t zero_cols(int prec, void* X, long long sX, int rows, int ld, int c0, int w, int n_traj, hipStream_t st) {
  int nb = nblocks((long long)rows * w * n_traj);
  if (prec == 0) hipLaunchKernelGGL(k_zero_cols<float>, dim3(nb), dim3(256), 0, st, (c32*)X, sX, rows, ld, c0, w, n_traj);
  else hipLaunchKernelGGL(k_zero_cols<double>, dim3(nb), dim3(256), 0, st, (c64d*)X, sX, rows, ld, c0, w, n_traj);
  return hipGetLastError();
}

__global__ void k_hop_scales(const double* evals, long long sE, int n, double* inv_sqrt, double* sqrt_, int n_traj) {
  long long total = (long long)n * n_traj;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    int t = (int)(e / n), k = (int)(e % n);
    double l = evals[t * sE + k];
    inv_sqrt[e] = l > 0 ? 1.0 / sqrt(l) : 0.0;
    sqrt_[e] = l > 0 ? sqrt(l) : 0.0;
  }
}

hipError_t hop_scales(const double* evals, long long sE, int n, double* inv_sqrt, double* sqrt_, int n_traj,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_hop_scales, dim3(nblocks((long long)n * n_traj)), dim3(256), 0, st, evals, sE, n, inv_sqrt, sqrt_, n_traj);
  return hipGetLastError();
}


// Observables of a two-site step with the identity gate: the 4 x 4 two-site reduced state of
// sites (i, i+1) summed over the theta tiles' partials in a fixed order (FP64), then
// <Z_i>, <Z_i Z_(i+1)> (and <Z_(i+1)> for the last pair) normalised by its trace, into row
// traj of per_traj (stride doubles): <Z_k> at k, <Z_k Z_(k+1)> at n + k.
__global__ void k_obs_pair(const double* __restrict__ partial, int n_tiles, int i, int n, double* __restrict__ per_traj,
                           int stride, int n_traj) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_traj) return;
  const double* pp = partial + (long long)t * n_tiles * 32;
  double d[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < n_tiles; ++k)
    for (int x = 0; x < 4; ++x) d[x] += pp[k * 32 + 2 * (5 * x)];   // diagonal element (x, x)
  const double tr = (d[0] + d[1]) + (d[2] + d[3]);
  const double inv = tr > 0.0 ? 1.0 / tr : __builtin_nan("");
  double* o = per_traj + (long long)t * stride;
  o[i] = ((d[0] + d[1]) - (d[2] + d[3])) * inv;          // x = 2 s + t: s = 0 for x < 2
  o[n + i] = ((d[0] - d[1]) - (d[2] - d[3])) * inv;      // z_s z_t
  if (i == n - 2) o[n - 1] = ((d[0] - d[1]) + (d[2] - d[3])) * inv;
}

hipError_t obs_pair(const double* partial, int n_tiles, int i, int n, double* per_traj, int stride, int n_traj,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_obs_pair, dim3((n_traj + 127) / 128), dim3(128), 0, st, partial, n_tiles, i, n, per_traj, stride,
                     n_traj);
  return hipGetLastError();
}

__global__ void k_obs_reduce(const double* __restrict__ per_traj, int n_obs, int stride, int n_traj, double* mean,
                             double* m2) {
  __shared__ double sn[256], sm[256], sq[256];
  const int o = blockIdx.x, tid = threadIdx.x;
  double n = 0, mu = 0, q = 0;
  for (int t = tid; t < n_traj; t += 256) {
    double x = per_traj[(long long)t * stride + o];
    n += 1;
    double d = x - mu;
    mu += d / n;
    q += d * (x - mu);
  }
  sn[tid] = n; sm[tid] = mu; sq[tid] = q;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      double na = sn[tid], nb = sn[tid + s];
      double nn = na + nb;
      if (nb > 0) {
        double d = sm[tid + s] - sm[tid];
        sm[tid] = nn > 0 ? sm[tid] + d * nb / nn : 0.0;
        sq[tid] = sq[tid] + sq[tid + s] + d * d * na * nb / nn;
        sn[tid] = nn;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    mean[o] = sm[0];
    m2[o] = sq[0];
  }
}

hipError_t obs_reduce(const double* per_traj, int n_obs, int stride, int n_traj, double* mean, double* m2,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_obs_reduce, dim3(n_obs), dim3(256), 0, st, per_traj, n_obs, stride, n_traj, mean, m2);
  return hipGetLastError();
}

// ------------------------------------------------------------------ untruncated splits
// 1 / ||X||_F of each trajectory's two-site matrix (FP64 sums), and a zero discarded weight.
template <typename T>
__global__ __launch_bounds__(256) void k_split_norm(const cplx<T>* __restrict__ X, long long sX, long long len,
                                                    double* __restrict__ alpha, double* discarded, int disc_stride,
                                                    int accumulate) {
  __shared__ double red[4];
  const cplx<T>* x = X + blockIdx.x * sX;
  double a = 0.0;
  for (long long e = threadIdx.x; e < len; e += 256) {
    const double r = (double)x[e].re, i = (double)x[e].im;
    a = fma(r, r, fma(i, i, a));
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    alpha[blockIdx.x] = t > 0 ? 1.0 / sqrt(t) : 0.0;
    if (discarded && !accumulate) discarded[(long long)blockIdx.x * disc_stride] = 0.0;
  }
}

hipError_t split_norm(int prec, const void* X, long long sX, long long len, double* alpha, double* discarded,
                      int disc_stride, int accumulate, int n_traj, hipStream_t st) {
  if (prec == 0)
    hipLaunchKernelGGL(k_split_norm<float>, dim3(n_traj), dim3(256), 0, st, (const c32*)X, sX, len, alpha, discarded,
                       disc_stride, accumulate);
  else
    hipLaunchKernelGGL(k_split_norm<double>, dim3(n_traj), dim3(256), 0, st, (const c64d*)X, sX, len, alpha,
                       discarded, disc_stride, accumulate);
  return hipGetLastError();
}

// Block re-mapping between a trajectory's full-capacity matrices and the compact live blocks
// of an untruncated split.  dst[i][j] (i < drows, j < dcols) = alpha_t * S(i, j), where
// column j is read as (t, b) = (j / dh, j % dh) (dh = dcols: unsplit columns, t = 0), the
// element is live iff i < ri, t < 2 and b < bh, and then
//   S(i, j) = src[i][t * sh + b]   (conj_t: conj(src[t * sh + b][i]))
// or, with src == NULL, S(i, j) = 1 if i == t * bh + b (an identity on the live block);
// every other element is set to zero.
template <typename T>
__global__ void k_remap(cplx<T>* dst, long long sD, int ldd, int drows, int dcols, int dh, int ri, int bh,
                        const cplx<T>* __restrict__ src, long long sS, int lds, int sh, int conj_t,
                        const double* __restrict__ alpha) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int tr = blockIdx.y;
  if (e >= (long long)drows * dcols) return;
  const int i = (int)(e / dcols), j = (int)(e % dcols);
  const int t = j / dh, b = j % dh;
  cplx<T> v = {(T)0, (T)0};
  if (i < ri && t < 2 && b < bh) {
    if (!src) {
      v.re = (i == t * bh + b) ? (T)1 : (T)0;
    } else {
      const int c = t * sh + b;
      v = conj_t ? src[tr * sS + (long long)c * lds + i] : src[tr * sS + (long long)i * lds + c];
      if (conj_t) v.im = -v.im;
      if (alpha) {
        const double a = alpha[tr];
        v = cplx<T>{(T)(a * (double)v.re), (T)(a * (double)v.im)};
      }
    }
  }
  dst[tr * sD + (long long)i * ldd + j] = v;
}

hipError_t remap(int prec, void* dst, long long sD, int ldd, int drows, int dcols, int dh, int ri, int bh,
                 const void* src, long long sS, int lds, int sh, bool conj_t, const double* alpha, int n_traj,
                 hipStream_t st) {
  const long long len = (long long)drows * dcols;
  if (len <= 0) return hipSuccess;
  dim3 g((unsigned)((len + 255) / 256), (unsigned)n_traj);
  if (prec == 0)
    hipLaunchKernelGGL(k_remap<float>, g, dim3(256), 0, st, (c32*)dst, sD, ldd, drows, dcols, dh, ri, bh,
                       (const c32*)src, sS, lds, sh, (int)conj_t, alpha);
  else
    hipLaunchKernelGGL(k_remap<double>, g, dim3(256), 0, st, (c64d*)dst, sD, ldd, drows, dcols, dh, ri, bh,
                       (const c64d*)src, sS, lds, sh, (int)conj_t, alpha);
  return hipGetLastError();
}

// ------------------------------------------------------------------ second-level truncation
// A Gram matrix G = M M^dag resolves singular values only down to about sqrt(eps) of the
// largest (its eigenvectors carry an absolute error of eps * lambda_max), so when a truncation
// cut falls below that level the kept subspace is re-solved from the residual
// R = M - Z_r Z_r^dag M of the well-resolved directions Z_r (lambda > tau lambda_max), whose own
// Gram R R^dag resolves the rest.  l2_prep decides per trajectory (active iff the kept
// eigenvalue at the cut lies below tau lambda_max), counts r and masks Z to its first r
// columns; l2_merge places the top kept - r residual directions after them and updates the
// renormalisation and the discarded weight.
__global__ __launch_bounds__(256) void k_l2_prep(const double* __restrict__ evals, long long sE, const double* __restrict__ ws,
                                                 long long sW, const double* __restrict__ kept_l1, int n, int kk, double tau,
                                                 const c64d* __restrict__ Z, long long sZ, c64d* __restrict__ Zr,
                                                 long long sZr, int* __restrict__ act, int* __restrict__ rr,
                                                 double* __restrict__ info) {
  __shared__ int s_r;
  const int t = blockIdx.x, tid = threadIdx.x;
  const double* ev = evals + t * sE;
  const double thr = tau * ev[0];
  if (tid == 0) {
    int r = 0;
    double k1 = 0.0;
    while (r < kk && ev[r] >= thr && ev[r] > 0.0) k1 += ev[r++];
    const int a = (r < kk && ev[0] > 0.0) ? 1 : 0;
    act[t] = a;
    rr[t] = r;
    info[3 * t] = k1;                     // kept weight of the resolved directions
    info[3 * t + 1] = ws[t * sW + 3 * n]; // trace of the Gram
    info[3 * t + 2] = kept_l1[t];         // kept weight of the first-level truncation
    s_r = r;
  }
  __syncthreads();
  const int r = s_r;
  for (long long e = tid; e < (long long)n * kk; e += 256) {
    const int c = (int)(e % kk);
    Zr[t * sZr + e] = c < r ? Z[t * sZ + e] : c64d{0.0, 0.0};
  }
}

hipError_t l2_prep(const double* evals, long long sE, const double* ws, long long sW, const double* kept_l1, int n,
                   int kk, double tau, const double* Z, long long sZ, double* Zr, long long sZr, int* act, int* r,
                   double* info, int n_traj, hipStream_t st) {
  hipLaunchKernelGGL(k_l2_prep, dim3(n_traj), dim3(256), 0, st, evals, sE, ws, sW, kept_l1, n, kk, tau, (const c64d*)Z,
                     sZ, (c64d*)Zr, sZr, act, r, info);
  return hipGetLastError();
}

// out = a - b elementwise (len c128 per trajectory) for active trajectories (act NULL: all)
__global__ void k_l2_sub(c64d* out, long long sO, const c64d* __restrict__ a, long long sa, const c64d* __restrict__ b,
                         long long sb, long long len, const int* __restrict__ act) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (e >= len || (act && !act[t])) return;
  const c64d x = a[t * sa + e], y = b[t * sb + e];
  out[t * sO + e] = c64d{x.re - y.re, x.im - y.im};
}

hipError_t l2_sub(double* out, long long sO, const double* a, long long sa, const double* b, long long sb, long long len,
                  const int* act, int n_traj, hipStream_t st) {
  dim3 g((unsigned)((len + 255) / 256), (unsigned)n_traj);
  hipLaunchKernelGGL(k_l2_sub, g, dim3(256), 0, st, (c64d*)out, sO, (const c64d*)a, sa, (const c64d*)b, sb, len, act);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_l2_merge(const int* __restrict__ act, const int* __restrict__ rr, int n, int kk,
                                                  c64d* __restrict__ Z, long long sZ, const c64d* __restrict__ Z2,
                                                  long long sZ2, const double* __restrict__ ev2, long long sE,
                                                  const double* __restrict__ info, double* __restrict__ alpha,
                                                  double* discarded, int disc_stride, int accumulate) {
  __shared__ double red[4];
  __shared__ double s_inv;
  const int t = blockIdx.x, tid = threadIdx.x;
  if (!act[t]) return;
  const int r = rr[t];
  for (int j = 0; j + r < kk; ++j) {
    const c64d* z = Z2 + t * sZ2;
    double a = 0.0;
    for (int i = tid; i < n; i += 256) {
      const c64d v = z[(long long)i * kk + j];
      a = fma(v.re, v.re, fma(v.im, v.im, a));
    }
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = a;
    __syncthreads();
    if (tid == 0) {
      const double q = (red[0] + red[1]) + (red[2] + red[3]);
      // a residual direction of no weight (eigenvalue dropped) stays a zero vector
      s_inv = (q > 0.0 && ev2[t * sE + j] > 0.0) ? 1.0 / sqrt(q) : 0.0;
    }
    __syncthreads();
    const double inv = s_inv;
    for (int i = tid; i < n; i += 256) {
      const c64d v = z[(long long)i * kk + j];
      Z[t * sZ + (long long)i * kk + r + j] = c64d{v.re * inv, v.im * inv};
    }
    __syncthreads();
  }
  if (tid == 0) {
    double kept = info[3 * t];
    for (int j = 0; j + r < kk; ++j) kept += fmax(ev2[t * sE + j], 0.0);
    const double tr = info[3 * t + 1], k1 = info[3 * t + 2];
    alpha[t] = kept > 0.0 ? 1.0 / sqrt(kept) : 0.0;
    if (discarded) {
      const double e2 = tr > 0.0 ? fmax(tr - kept, 0.0) / tr : 0.0;
      const double e1 = tr > 0.0 ? fmax(tr - k1, 0.0) / tr : 0.0;
      double* d = discarded + (long long)t * disc_stride;
      *d = accumulate ? *d - e1 + e2 : e2;
    }
  }
}

hipError_t l2_merge(const int* act, const int* r, int n, int kk, double* Z, long long sZ, const double* Z2, long long sZ2,
                    const double* ev2, long long sE, const double* info, double* alpha, double* discarded,
                    int disc_stride, int accumulate, int n_traj, hipStream_t st) {
  hipLaunchKernelGGL(k_l2_merge, dim3(n_traj), dim3(256), 0, st, act, r, n, kk, (c64d*)Z, sZ, (const c64d*)Z2, sZ2, ev2,
                     sE, info, alpha, discarded, disc_stride, accumulate);
  return hipGetLastError();
}

// dst[r0 + i][c0 + j] = src[i][j] (c128, rows x cols), conj_t: conj(src[j][i]); the rest of dst
// is not touched
__global__ void k_put_block(c64d* dst, long long sD, int ldd, int r0, int c0, int rows, int cols,
                            const c64d* __restrict__ src, long long sS, int lds, int conj_t) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (e >= (long long)rows * cols) return;
  const int i = (int)(e / cols), j = (int)(e % cols);
  c64d v = conj_t ? src[t * sS + (long long)j * lds + i] : src[t * sS + (long long)i * lds + j];
  if (conj_t) v.im = -v.im;
  dst[t * sD + (long long)(r0 + i) * ldd + c0 + j] = v;
}

hipError_t put_block(double* dst, long long sD, int ldd, int r0, int c0, int rows, int cols, const double* src,
                     long long sS, int lds, bool conj_t, int n_traj, hipStream_t st) {
  const long long len = (long long)rows * cols;
  if (len <= 0) return hipSuccess;
  dim3 g((unsigned)((len + 255) / 256), (unsigned)n_traj);
  hipLaunchKernelGGL(k_put_block, g, dim3(256), 0, st, (c64d*)dst, sD, ldd, r0, c0, rows, cols, (const c64d*)src, sS, lds,
                     (int)conj_t);
  return hipGetLastError();
}

// acc += b (c128, len per trajectory)
__global__ void k_add(c64d* acc, long long sA, const c64d* __restrict__ b, long long sB, long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (e >= len) return;
  const c64d x = acc[t * sA + e], y = b[t * sB + e];
  acc[t * sA + e] = c64d{x.re + y.re, x.im + y.im};
}

hipError_t add_c128(double* acc, long long sA, const double* b, long long sB, long long len, int n_traj, hipStream_t st) {
  dim3 g((unsigned)((len + 255) / 256), (unsigned)n_traj);
  hipLaunchKernelGGL(k_add, g, dim3(256), 0, st, (c64d*)acc, sA, (const c64d*)b, sB, len);
  return hipGetLastError();
}

// per_traj[t][c] = NaN for c0 <= c < stride (rows of a mixed batch past a trajectory's width)
__global__ void k_fill_nan(double* per_traj, int stride, int c0, int n_traj) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = stride - c0;
  if (e >= (long long)w * n_traj) return;
  per_traj[(e / w) * stride + c0 + e % w] = __builtin_nan("");
}

hipError_t fill_nan(double* per_traj, int stride, int c0, int n_traj, hipStream_t st) {
  if (c0 >= stride) return hipSuccess;
  hipLaunchKernelGGL(k_fill_nan, dim3(nblocks((long long)(stride - c0) * n_traj)), dim3(256), 0, st, per_traj, stride, c0,
                     n_traj);
  return hipGetLastError();
}

// ------------------------------------------------------------------ certified error
// eps_tot[t] += weight * sum over the layer's truncation steps of their trace-norm change:
// 2 sqrt(eps) (kind 0, the exact value for one bond) or 4 sqrt(2 eps) (kind 1, the
// computable bound of the MPS-truncation section).
__global__ void k_err_acc(int n_traj, int slots, const double* __restrict__ disc, int kind, double weight,
                          double* __restrict__ eps_tot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_traj) return;
  double s = 0.0;
  for (int k = 0; k < slots; ++k) {
    const double e = fmax(disc[(long long)t * slots + k], 0.0);
    s += kind == 0 ? 2.0 * sqrt(e) : 4.0 * sqrt(2.0 * e);
  }
  eps_tot[t] += weight * s;
}

hipError_t err_accumulate(int n_traj, int slots, const double* disc, int kind, double weight, double* eps_tot,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_err_acc, dim3((n_traj + 255) / 256), dim3(256), 0, st, n_traj, slots, disc, kind, weight, eps_tot);
  return hipGetLastError();
}

// out = (mean of the capped errors, Hoeffding buffer, their sum): eps_bound = eps_tot when
// eps_tot <= eps_max - 2, else eps_max; one workgroup, fixed summation order.
__global__ __launch_bounds__(256) void k_err_est(int n_traj, const double* __restrict__ eps_tot, double eps_max,
                                                 double delta, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int t = threadIdx.x; t < n_traj; t += 256) {
    const double e = eps_tot[t];
    s += e <= eps_max - 2.0 ? e : eps_max;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double hat = red[0] / n_traj;
    const double buf = sqrt(eps_max * eps_max * log(1.0 / delta) / (2.0 * n_traj));
    out[0] = hat;
    out[1] = buf;
    out[2] = hat + buf;
  }
}

hipError_t err_estimate(int n_traj, const double* eps_tot, double eps_max, double delta, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_err_est, dim3(1), dim3(256), 0, st, n_traj, eps_tot, eps_max, delta, out);
  return hipGetLastError();
}

}  // namespace mpsb
