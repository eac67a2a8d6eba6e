// Batched complex contractions of the gate-step: the generic strided GEMM used for the
// Gram matrices, recomposition, centre hops and environments, the two-site theta
// contraction with the gate and two-site reduced density matrix fused in its epilogue, the
// in-place application of the sampled Kraus pair, and small cast/scale helpers.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace mpsb {

// ============================================================================ generic GEMM
// C[b] = alpha[b] * op(A[b]) * op(B[b]);  op = N (row-major M x K, ld) or
// C (conjugate transpose of a row-major K x M matrix).  64x64 tiles, BK = 16, 256 threads,
// LDS staging as separate re/im planes.
constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

template <typename T> struct Ld;
template <> struct Ld<float> { using C = c32; };
template <> struct Ld<double> { using C = c64d; };

typedef float v4f __attribute__((ext_vector_type(4)));

// the 4x4 gate of trajectory traj (uniform over the workgroup)
__device__ inline void load_gate(const Mat4& gate, const GateRef& gref, int traj, double (&gg)[32]) {
  if (gref.pool) {
    const int id = gref.ids[traj * gref.traj_stride + (long long)(*gref.layer) * gref.layer_stride + gref.pair];
    const double* g = gref.pool + 32LL * id;
#pragma unroll
    for (int x = 0; x < 32; ++x) gg[x] = g[x];
  } else {
#pragma unroll
    for (int x = 0; x < 32; ++x) gg[x] = gate.v[x];
  }
}

// The two-site RDM is Hermitian: per theta entry only its upper triangle is accumulated
// (Re v_x conj(v_y) for x <= y, Im for x < y; index o of (x, y) = 4 x - x (x - 1) / 2 + y - x),
// and the workgroup's sums (red[w][0..9] real, red[w][10..19] imaginary, one row per wave) are
// written out as the full 4 x 4 c128 by symmetry.
__device__ inline void rdm_upper_acc(double (&rr)[10], double (&ri)[10], const double (&vr)[4], const double (&vi)[4]) {
  int o = 0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = x; y < 4; ++y) {
      rr[o] += vr[x] * vr[y] + vi[x] * vi[y];
      if (y > x) ri[o] += vi[x] * vr[y] - vr[x] * vi[y];
      ++o;
    }
}

__device__ inline void rdm_reduce_write(const double (&rr)[10], const double (&ri)[10], double (&red)[4][32], double* p) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int x = 0; x < 20; ++x) {
    double v = (x < 10) ? rr[x] : ri[x - 10];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][x] = v;
  }
  __syncthreads();
  if (tid < 32) {
    const int x = (tid & 15) >> 2, y = tid & 3, lo = x < y ? x : y, hi = x < y ? y : x;
    const int o = lo * 4 - lo * (lo - 1) / 2 + (hi - lo);
    double v;
    if (tid < 16) v = red[0][o] + red[1][o] + red[2][o] + red[3][o];
    else v = x == y ? 0.0 : (x < y ? 1.0 : -1.0) * (red[0][10 + o] + red[1][10 + o] + red[2][10 + o] + red[3][10 + o]);
    if (tid < 16) p[2 * (tid & 15)] = v; else p[2 * (tid & 15) + 1] = v;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
  using V = v4f;
  static __device__ inline V mac(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane_hi, int reg) { return 4 * lane_hi + reg; }
};
template <> struct MfmaAcc<double> {
  using V = v4d;
  static __device__ inline V mac(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane_hi, int reg) { return lane_hi + 4 * reg; }
};

// MFMA form of the generic GEMM: the same 64 x 64 block tile and LDS staging; each of the
// 4 waves owns a 32 x 32 quadrant as 2 x 2 MFMA sub-tiles of 16 x 16, complex products as four
// real 16x16x4 MFMAs (f32 for FP32 inputs, f64 for FP64 inputs) per k-step of 4.
template <typename TA, typename TB, typename TACC, typename TC, bool CA, bool CB, int S = 2>
__global__ __launch_bounds__(256, S == 4 ? 2 : 1) void k_gemm_mfma(int M, int N, int K, const cplx<TA>* __restrict__ A,
                                                   int lda, long long sA, const cplx<TB>* __restrict__ B,
                                                   int ldb, long long sB, cplx<TC>* __restrict__ C, int ldc,
                                                   long long sC, const double* __restrict__ alpha, int lower,
                                                   const int* __restrict__ active) {
  using Mf = MfmaAcc<TACC>;
  using V = typename Mf::V;
  constexpr int TILE = 32 * S;   // workgroup tile TILE x TILE, wave tile 16 S x 16 S
  constexpr int LPT = 2 * S;     // elements of each operand slice per thread
  __shared__ TACC As_re[GB_K][TILE + 4], As_im[GB_K][TILE + 4];
  __shared__ TACC Bs_re[GB_K][TILE + 4], Bs_im[GB_K][TILE + 4];
  const int bz = blockIdx.z;
  if (active && !active[bz]) return;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  // lower: only the tiles holding elements on or below the diagonal are computed (the upper
  // triangle of a Hermitian product that is read from its lower triangle alone)
  if (lower && n0 >= m0 + TILE) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wa = wv >> 1, wb = wv & 1, r16 = lane & 15, kq = lane >> 4;
  V acc_re[S][S], acc_im[S][S];
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      acc_re[i][j] = V{0, 0, 0, 0};
      acc_im[i][j] = V{0, 0, 0, 0};
    }
  // the next k-slice is loaded into registers while the current one is multiplied from LDS
  cplx<TA> pa[LPT];
  cplx<TB> pb[LPT];
  auto load_slice = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (!CA) { kk = e & 15; mm = e >> 4; } else { mm = e % TILE; kk = e / TILE; }
      const int m = m0 + mm, k = k0 + kk;
      cplx<TA> v = {0, 0};
      if (m < M && k < K) {
        if (!CA) v = A[(long long)m * lda + k];
        else { v = A[(long long)k * lda + m]; v.im = -v.im; }
      }
      pa[r] = v;
    }
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      const int e = tid + 256 * r;
      int nn, kk;
      if (!CB) { nn = e % TILE; kk = e / TILE; } else { kk = e & 15; nn = e >> 4; }
      const int n = n0 + nn, k = k0 + kk;
      cplx<TB> v = {0, 0};
      if (n < N && k < K) {
        if (!CB) v = B[(long long)k * ldb + n];
        else { v = B[(long long)n * ldb + k]; v.im = -v.im; }
      }
      pb[r] = v;
    }
  };
  load_slice(0);
  for (int k0 = 0; k0 < K; k0 += GB_K) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (!CA) { kk = e & 15; mm = e >> 4; } else { mm = e % TILE; kk = e / TILE; }
      As_re[kk][mm] = (TACC)pa[r].re;
      As_im[kk][mm] = (TACC)pa[r].im;
    }
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      const int e = tid + 256 * r;
      int nn, kk;
      if (!CB) { nn = e % TILE; kk = e / TILE; } else { kk = e & 15; nn = e >> 4; }
      Bs_re[kk][nn] = (TACC)pb[r].re;
      Bs_im[kk][nn] = (TACC)pb[r].im;
    }
    __syncthreads();
    if (k0 + GB_K < K) load_slice(k0 + GB_K);
#pragma unroll
    for (int k4 = 0; k4 < GB_K / 4; ++k4) {
      const int kk = 4 * k4 + kq;
      TACC ar[S], ai[S], br[S], bi[S];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        ar[i] = As_re[kk][16 * S * wa + 16 * i + r16];
        ai[i] = As_im[kk][16 * S * wa + 16 * i + r16];
        br[i] = Bs_re[kk][16 * S * wb + 16 * i + r16];
        bi[i] = Bs_im[kk][16 * S * wb + 16 * i + r16];
      }
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) {
          acc_re[i][j] = Mf::mac(ar[i], br[j], acc_re[i][j]);
          acc_re[i][j] = Mf::mac(-ai[i], bi[j], acc_re[i][j]);
          acc_im[i][j] = Mf::mac(ar[i], bi[j], acc_im[i][j]);
          acc_im[i][j] = Mf::mac(ai[i], br[j], acc_im[i][j]);
        }
    }
    __syncthreads();
  }
  const double al = alpha ? alpha[bz] : 1.0;
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int n = n0 + 16 * S * wb + 16 * j + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * S * wa + 16 * i + Mf::row(kq, r);
        if (m >= M || n >= N) continue;
        cplx<TC> o;
        o.re = (TC)(al * (double)acc_re[i][j][r]);
        o.im = (TC)(al * (double)acc_im[i][j][r]);
        C[(long long)m * ldc + n] = o;
      }
    }
}

template <typename TA, typename TB, typename TACC, typename TC, int S>
static hipError_t gemm_launch(bool ca, bool cb, int M, int N, int K, const void* A, int lda,
                              long long sA, const void* B, int ldb, long long sB, void* C,
                              int ldc, long long sC, const double* alpha, int batch,
                              hipStream_t st, int lower, const int* active) {
  constexpr int TILE = 32 * S;
  dim3 grid((N + TILE - 1) / TILE, (M + TILE - 1) / TILE, batch);
  auto a = (const cplx<TA>*)A;
  auto b = (const cplx<TB>*)B;
  auto c = (cplx<TC>*)C;
  if (!ca && !cb) hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TACC, TC, false, false, S>), grid, dim3(256), 0, st, M, N, K, a, lda, sA, b, ldb, sB, c, ldc, sC, alpha, lower, active);
  else if (ca && !cb) hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TACC, TC, true, false, S>), grid, dim3(256), 0, st, M, N, K, a, lda, sA, b, ldb, sB, c, ldc, sC, alpha, lower, active);
  else if (!ca && cb) hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TACC, TC, false, true, S>), grid, dim3(256), 0, st, M, N, K, a, lda, sA, b, ldb, sB, c, ldc, sC, alpha, lower, active);
  else hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TACC, TC, true, true, S>), grid, dim3(256), 0, st, M, N, K, a, lda, sA, b, ldb, sB, c, ldc, sC, alpha, lower, active);
  return hipGetLastError();
}

// 128 x 128 workgroup tiles for the full (not lower-triangle) FP32-accumulated products of the
// bulk bonds (both sides >= 128: more products per LDS slice and per barrier; measured 12%
// faster for the 128 x 256 x 256 recomposition product, no faster for the lower-triangle Gram,
// whose diagonal tiles would then compute a larger upper part), 64 x 64 otherwise.  Every
// output element accumulates its k-slices in the same order for either tile, so the results
// agree bit for bit.
template <typename TA, typename TB, typename TACC, typename TC>
static hipError_t gemm_dispatch(bool ca, bool cb, int M, int N, int K, const void* A, int lda,
                                long long sA, const void* B, int ldb, long long sB, void* C,
                                int ldc, long long sC, const double* alpha, int batch,
                                hipStream_t st, int lower, const int* active) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if constexpr (sizeof(TACC) == 4) {
    if (!lower && M >= 128 && N >= 128)
      return gemm_launch<TA, TB, TACC, TC, 4>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lower, active);
  }
  return gemm_launch<TA, TB, TACC, TC, 2>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lower, active);
}

hipError_t gemm(int prec_in, int prec_out, bool ca, bool cb, int M, int N, int K, const void* A,
                int lda, long long sA, const void* B, int ldb, long long sB, void* C, int ldc,
                long long sC, const double* alpha, int batch, hipStream_t st, bool lower, const int* active) {
  const int lo = lower ? 1 : 0;
  if (prec_in == 0 && prec_out == 0)
    return gemm_dispatch<float, float, float, float>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lo, active);
  if (prec_in == 0 && prec_out == 1)
    return gemm_dispatch<float, float, float, double>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lo, active);
  if (prec_in == 0 && prec_out == 2)   // c64 operands, FP64 accumulation and output
    return gemm_dispatch<float, float, double, double>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lo, active);
  return gemm_dispatch<double, double, double, double>(ca, cb, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, batch, st, lo, active);
}

// ============================================================================ theta
// theta[(a,s),(t,b)] = sum_c C[a][s][c] B[c][t][b]; then per (a,b) the 4 values over (s,t)
// are mixed by the gate G[s't'][st] and written in place of theta (row 2a+s', column
// t' chi_r + b), and the two-site reduced density matrix
//   rho[x][y] = sum_{a,b} thetaG[x][a,b] conj(thetaG[y][a,b]),  x = 2s'+t'
// is accumulated per tile (FP64) into partial[traj][tile][16] c128.
// Tile: 32 values of a (64 rows) x 32 values of b for both t (64 columns), 4 waves of 64.
// Each wave owns 16 values of a x 16 values of b and all four (s,t) blocks, so the gate mix
// and the RDM stay in registers.  Complex products are four real 16x16x4 MFMAs (re*re,
// -im*im, re*im, im*re) per (s,t) block and k-step of 4.
// Lane layout of the 16x16x4 MFMAs: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k; the
// result D[i][j] sits in lane j + 16 (i / 4), register i % 4 for the f32 instruction and in
// lane j + 16 (i % 4), register i / 4 for the f64 one (checked on the device).
template <typename T>
__global__ __launch_bounds__(256) void k_theta(int chi_l, int chi_m, int chi_r, const cplx<T>* __restrict__ Cs,
                                                    const cplx<T>* __restrict__ Bs, long long s_traj,
                                                    cplx<T>* __restrict__ out, long long s_out, Mat4 gate, GateRef gref,
                                                    double* __restrict__ partial, int n_tiles) {
  using M = MfmaAcc<T>;
  using V = typename M::V;
  __shared__ T A_re[GB_K][64 + 4], A_im[GB_K][64 + 4];   // [k][row = 2*(a-a0)+s]
  __shared__ T B_re[GB_K][64 + 4], B_im[GB_K][64 + 4];   // [k][col = t*32 + (b-b0)]
  __shared__ double red[4][32];
  const int traj = blockIdx.z;
  const cplx<T>* Cp = Cs + traj * s_traj;
  const cplx<T>* Bp = Bs + traj * s_traj;
  cplx<T>* O = out + traj * s_out;
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wa = wv >> 1, wb = wv & 1;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ldb = 2 * chi_r;
  V acc_re[4], acc_im[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    acc_re[x] = V{0, 0, 0, 0};
    acc_im[x] = V{0, 0, 0, 0};
  }
  for (int k0 = 0; k0 < chi_m; k0 += GB_K) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = tid + 256 * r;
      int kk = e & 15, row = e >> 4;
      int a = a0 + (row >> 1), s = row & 1, k = k0 + kk;
      cplx<T> v = {0, 0};
      if (a < chi_l && k < chi_m) v = Cp[(long long)(2 * a + s) * chi_m + k];
      A_re[kk][row] = v.re;
      A_im[kk][row] = v.im;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = tid + 256 * r;
      int col = e & 63, kk = e >> 6;
      int t = col >> 5, b = b0 + (col & 31), k = k0 + kk;
      cplx<T> v = {0, 0};
      if (b < chi_r && k < chi_m) v = Bp[(long long)k * ldb + t * chi_r + b];
      B_re[kk][col] = v.re;
      B_im[kk][col] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < GB_K / 4; ++k4) {
      const int kk = 4 * k4 + kq;
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int row = 2 * (16 * wa + r16) + s;
        ar[s] = A_re[kk][row];
        ai[s] = A_im[kk][row];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = 32 * t + 16 * wb + r16;
        br[t] = B_re[kk][col];
        bi[t] = B_im[kk][col];
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int x = 2 * s + t;
          acc_re[x] = M::mac(ar[s], br[t], acc_re[x]);
          acc_re[x] = M::mac(-ai[s], bi[t], acc_re[x]);
          acc_im[x] = M::mac(ar[s], bi[t], acc_im[x]);
          acc_im[x] = M::mac(ai[s], br[t], acc_im[x]);
        }
    }
    __syncthreads();
  }
  // epilogue: lane holds rows a = a0 + 16 wa + row(kq, i), column b = b0 + 16 wb + r16
  double gg[32];
  load_gate(gate, gref, traj, gg);
  double rr[10], ri[10];
#pragma unroll
  for (int x = 0; x < 10; ++x) rr[x] = ri[x] = 0.0;
  const int b = b0 + 16 * wb + r16;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int a = a0 + 16 * wa + M::row(kq, i);
    if (a >= chi_l || b >= chi_r) continue;
    double vr[4], vi[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      double sr = 0, si = 0;
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const double gr = gg[2 * (4 * x + y)], gi = gg[2 * (4 * x + y) + 1];
        const double tr = (double)acc_re[y][i], tim = (double)acc_im[y][i];
        sr += gr * tr - gi * tim;
        si += gr * tim + gi * tr;
      }
      cplx<T> o;
      o.re = (T)sr;
      o.im = (T)si;
      O[(long long)(2 * a + (x >> 1)) * ldb + (x & 1) * chi_r + b] = o;
      vr[x] = (double)o.re;
      vi[x] = (double)o.im;
    }
    rdm_upper_acc(rr, ri, vr, vi);
  }
  rdm_reduce_write(rr, ri, red, partial + ((long long)traj * n_tiles + blockIdx.y * gridDim.x + blockIdx.x) * 32);
}

// Large-tile FP32 variant for the bulk bonds (chi_L, chi_R >= 64): 64 values of a x 64
// values of b per workgroup (128 rows x 128 columns of theta), 2 x 2 waves of 32 x 32 values,
// each wave 2 x 2 MFMA sub-tiles of 16 x 16 for each of the four (s,t) blocks (128
// accumulator registers per lane, within the 256 registers of two waves per SIMD).  The next K block of 16 is loaded into registers while
// the current one is multiplied out of LDS.  The site tensors are stored in LDS as [k][s][a]
// and [k][t][b] with a row pitch of 144 floats, so that the four k-rows a wave reads at once
// fall in different bank halves.  Workgroup ids are remapped so that all tiles of one
// trajectory run on one XCD (the hardware deals consecutive ids round-robin over the 8 XCDs)
// and share the trajectory's site tensors in that XCD's L2.
constexpr int TL_P = 144;

__global__ __launch_bounds__(256, 2) void k_theta_l(int chi_l, int chi_m, int chi_r, const c32* __restrict__ Cs,
                                                 const c32* __restrict__ Bs, long long s_traj, c32* __restrict__ out,
                                                 long long s_out, Mat4 gate, GateRef gref, double* __restrict__ partial, int tiles_a,
                                                 int tiles_b) {
  __shared__ float A_re[16][TL_P], A_im[16][TL_P];   // [k][s*64 + (a - a0)]
  __shared__ float B_re[16][TL_P], B_im[16][TL_P];   // [k][t*64 + (b - b0)]
  __shared__ double red[4][32];
  // XCD-aware numbering: hardware id w runs on XCD w % 8; logical ids of XCD x are the
  // contiguous range starting at x * q + min(x, r) (q = G / 8, r = G % 8)
  const int G = gridDim.x, w = blockIdx.x;
  const int q8 = G >> 3, r8 = G & 7, x8 = w & 7;
  const int L = x8 * q8 + min(x8, r8) + (w >> 3);
  const int nt = tiles_a * tiles_b;
  const int traj = L / nt, tile = L - traj * nt;
  const int ta = tile / tiles_b, tb = tile - ta * tiles_b;
  const c32* Cp = Cs + traj * s_traj;
  const c32* Bp = Bs + traj * s_traj;
  c32* O = out + traj * s_out;
  const int a0 = ta * 64, b0 = tb * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wa = wv >> 1, wb = wv & 1;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ldb = 2 * chi_r;
  v4f acc_re[2][2][4], acc_im[2][2][4];   // [ia][jb][2s+t]
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        acc_re[ia][jb][x] = v4f{0, 0, 0, 0};
        acc_im[ia][jb][x] = v4f{0, 0, 0, 0};
      }
  c32 pa[8], pb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      const int kk = e & 15, row = e >> 4;   // row = 2 (a - a0) + s
      const int a = a0 + (row >> 1), k = k0 + kk;
      pa[r] = (a < chi_l && k < chi_m) ? Cp[(long long)(2 * a + (row & 1)) * chi_m + k] : c32{0, 0};
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      const int col = e & 127, kk = e >> 7;  // col = t * 64 + (b - b0)
      const int b = b0 + (col & 63), k = k0 + kk;
      pb[r] = (b < chi_r && k < chi_m) ? Bp[(long long)k * ldb + (col >> 6) * chi_r + b] : c32{0, 0};
    }
  };
  gload(0);
  for (int k0 = 0; k0 < chi_m; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      const int kk = e & 15, row = e >> 4;
      const int c = (row & 1) * 64 + (row >> 1);
      A_re[kk][c] = pa[r].re;
      A_im[kk][c] = pa[r].im;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      const int col = e & 127, kk = e >> 7;
      B_re[kk][col] = pb[r].re;
      B_im[kk][col] = pb[r].im;
    }
    __syncthreads();
    if (k0 + 16 < chi_m) gload(k0 + 16);
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int kk = 4 * k4 + kq;
      float ar[2][2], ai[2][2], br[2][2], bi[2][2];
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int ca = s2 * 64 + 32 * wa + 16 * i2 + r16;
          ar[i2][s2] = A_re[kk][ca];
          ai[i2][s2] = A_im[kk][ca];
          const int cb = s2 * 64 + 32 * wb + 16 * i2 + r16;
          br[i2][s2] = B_re[kk][cb];
          bi[i2][s2] = B_im[kk][cb];
        }
#pragma unroll
      for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
              const int x = 2 * s2 + t2;
              v4f cr = acc_re[ia][jb][x], ci = acc_im[ia][jb][x];
              cr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ia][s2], br[jb][t2], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[ia][s2], bi[jb][t2], cr, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ia][s2], bi[jb][t2], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[ia][s2], br[jb][t2], ci, 0, 0, 0);
              acc_re[ia][jb][x] = cr;
              acc_im[ia][jb][x] = ci;
            }
    }
    __syncthreads();
  }
  // epilogue: lane holds a = a0 + 32 wa + 16 ia + 4 kq + i, b = b0 + 32 wb + 16 jb + r16
  double gg[32];
  load_gate(gate, gref, traj, gg);
  double rr[10], ri[10];
#pragma unroll
  for (int x = 0; x < 10; ++x) rr[x] = ri[x] = 0.0;
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int b = b0 + 32 * wb + 16 * jb + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = a0 + 32 * wa + 16 * ia + 4 * kq + i;
        if (a >= chi_l || b >= chi_r) continue;
        double vr[4], vi[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          double sr = 0, si = 0;
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const double gr = gg[2 * (4 * x + y)], gi = gg[2 * (4 * x + y) + 1];
            const double tr = (double)acc_re[ia][jb][y][i], tim = (double)acc_im[ia][jb][y][i];
            sr += gr * tr - gi * tim;
            si += gr * tim + gi * tr;
          }
          c32 o;
          o.re = (float)sr;
          o.im = (float)si;
          O[(long long)(2 * a + (x >> 1)) * ldb + (x & 1) * chi_r + b] = o;
          vr[x] = (double)o.re;
          vi[x] = (double)o.im;
        }
        rdm_upper_acc(rr, ri, vr, vi);
      }
    }
  rdm_reduce_write(rr, ri, red, partial + ((long long)traj * nt + tile) * 32);
}

int theta_variant_ok(int prec, int variant, int chi_l, int chi_r) {
  if (variant == 0) return 1;
  if (variant == 1) return prec == 0 && chi_l >= 16 && chi_r >= 16;
  return 0;
}

int theta_default_variant(int prec, int chi_l, int chi_r) { return (prec == 0 && chi_l >= 64 && chi_r >= 64) ? 1 : 0; }

hipError_t theta(int prec, int chi_l, int chi_m, int chi_r, const void* Cs, const void* Bs,
                 long long s_traj, void* out, long long s_out, const Mat4& gate, const GateRef& gref, double* partial,
                 int n_traj, hipStream_t st, int variant) {
  if (variant < 0) variant = theta_default_variant(prec, chi_l, chi_r);
  if (!theta_variant_ok(prec, variant, chi_l, chi_r)) return hipErrorInvalidValue;
  if (variant == 1) {
    const int ta = (chi_l + 63) / 64, tb = (chi_r + 63) / 64;
    const long long blocks = (long long)ta * tb * n_traj;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_theta_l, dim3((unsigned)blocks), dim3(256), 0, st, chi_l, chi_m, chi_r, (const c32*)Cs,
                       (const c32*)Bs, s_traj, (c32*)out, s_out, gate, gref, partial, ta, tb);
    return hipGetLastError();
  }
  dim3 grid((chi_r + 31) / 32, (chi_l + 31) / 32, n_traj);
  int nt = grid.x * grid.y;
  if (prec == 0)
    hipLaunchKernelGGL(k_theta<float>, grid, dim3(256), 0, st, chi_l, chi_m, chi_r, (const c32*)Cs, (const c32*)Bs, s_traj, (c32*)out, s_out, gate, gref, partial, nt);
  else
    hipLaunchKernelGGL(k_theta<double>, grid, dim3(256), 0, st, chi_l, chi_m, chi_r, (const c64d*)Cs, (const c64d*)Bs, s_traj, (c64d*)out, s_out, gate, gref, partial, nt);
  return hipGetLastError();
}

// number of RDM tile partials the theta variant writes per trajectory (never more than for
// 32 x 32 tiles)
int theta_tiles(int variant, int chi_l, int chi_r) {
  if (variant == 1) return ((chi_r + 63) / 64) * ((chi_l + 63) / 64);
  return ((chi_r + 31) / 32) * ((chi_l + 31) / 32);
}

// device layer counter
__global__ void k_set_int(int* p, int v) { *p = v; }
__global__ void k_inc_int(int* p) { *p += 1; }
hipError_t set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}
hipError_t inc_int(int* p, hipStream_t st) {
  hipLaunchKernelGGL(k_inc_int, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

// batched strided block copy (16-byte or 8-byte elements)
template <typename T>
__global__ void k_copy_blocks(cplx<T>* dst, long long s_dst, const cplx<T>* src, long long s_src, long long elems,
                              int n_traj) {
  const long long total = elems * n_traj;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long t = e / elems, i = e - t * elems;
    dst[t * s_dst + i] = src[t * s_src + i];
  }
}

hipError_t copy_blocks_k(int prec, void* dst, long long s_dst, const void* src, long long s_src, long long elems,
                         int n_traj, hipStream_t st) {
  long long total = elems * n_traj;
  int nb = (int)std::min<long long>((total + 255) / 256, 65536);
  if (nb < 1) return hipSuccess;
  if (prec == 0) hipLaunchKernelGGL(k_copy_blocks<float>, dim3(nb), dim3(256), 0, st, (c32*)dst, s_dst, (const c32*)src, s_src, elems, n_traj);
  else hipLaunchKernelGGL(k_copy_blocks<double>, dim3(nb), dim3(256), 0, st, (c64d*)dst, s_dst, (const c64d*)src, s_src, elems, n_traj);
  return hipGetLastError();
}

// ============================================================================ Kraus pair
// X[(a,s),(t,b)] <- sum_{s0,t0} Ks[s][s0] Kt[t][t0] X[(a,s0),(t0,b)] in place, with the
// per-trajectory 2x2 operators ks/kt [traj][2][2] c128 (identity when flagged off).
template <typename T>
__global__ void k_kraus_pair(int chi_l, int chi_r, cplx<T>* X, long long s_traj, const double* __restrict__ kops,
                             int n_traj) {
  long long total = (long long)n_traj * chi_l * chi_r;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    int b = e % chi_r;
    long long r = e / chi_r;
    int a = r % chi_l;
    int traj = r / chi_l;
    const double* k = kops + traj * 16;   // Ks then Kt, each 2x2 c128
    cplx<T>* x = X + traj * s_traj;
    const int ld = 2 * chi_r;
    double vr[2][2], vi[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        cplx<T> v = x[(long long)(2 * a + s) * ld + t * chi_r + b];
        vr[s][t] = v.re;
        vi[s][t] = v.im;
      }
    // apply Kt on t
    double wr[2][2], wi[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        double sr = 0, si = 0;
#pragma unroll
        for (int t0 = 0; t0 < 2; ++t0) {
          double kr = k[8 + 2 * (2 * t + t0)], ki = k[8 + 2 * (2 * t + t0) + 1];
          sr += kr * vr[s][t0] - ki * vi[s][t0];
          si += kr * vi[s][t0] + ki * vr[s][t0];
        }
        wr[s][t] = sr;
        wi[s][t] = si;
      }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        double sr = 0, si = 0;
#pragma unroll
        for (int s0 = 0; s0 < 2; ++s0) {
          double kr = k[2 * (2 * s + s0)], ki = k[2 * (2 * s + s0) + 1];
          sr += kr * wr[s0][t] - ki * wi[s0][t];
          si += kr * wi[s0][t] + ki * wr[s0][t];
        }
        cplx<T> o;
        o.re = (T)sr;
        o.im = (T)si;
        x[(long long)(2 * a + s) * ld + t * chi_r + b] = o;
      }
  }
}

hipError_t kraus_pair(int prec, int chi_l, int chi_r, void* X, long long s_traj, const double* kops,
                      int n_traj, hipStream_t st) {
  long long total = (long long)n_traj * chi_l * chi_r;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  if (prec == 0) hipLaunchKernelGGL(k_kraus_pair<float>, dim3(blocks), dim3(256), 0, st, chi_l, chi_r, (c32*)X, s_traj, kops, n_traj);
  else hipLaunchKernelGGL(k_kraus_pair<double>, dim3(blocks), dim3(256), 0, st, chi_l, chi_r, (c64d*)X, s_traj, kops, n_traj);
  return hipGetLastError();
}

// ============================================================================ scale + cast
// out[i][j] = in[i][j] * col_scale[j]   (conj_t: out[j][i] = conj(in[i][j]) * col_scale[j])
// in: c128 rows x cols (ld_in); out: T (ld_out).  col_scale per trajectory or NULL.
template <typename T>
__global__ void k_scale_cast(int rows, int cols, const c64d* __restrict__ in, int ld_in, long long s_in,
                             const double* __restrict__ col_scale, long long s_scale, bool conj_t,
                             cplx<T>* __restrict__ out, int ld_out, long long s_out, int n_traj) {
  long long total = (long long)n_traj * rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    int j = e % cols;
    long long r = e / cols;
    int i = r % rows;
    int traj = r / rows;
    c64d v = in[traj * s_in + (long long)i * ld_in + j];
    double sc = col_scale ? col_scale[traj * s_scale + j] : 1.0;
    cplx<T> o;
    if (!conj_t) {
      o.re = (T)(v.re * sc);
      o.im = (T)(v.im * sc);
      out[traj * s_out + (long long)i * ld_out + j] = o;
    } else {
      o.re = (T)(v.re * sc);
      o.im = (T)(-v.im * sc);
      out[traj * s_out + (long long)j * ld_out + i] = o;
    }
  }
}

hipError_t scale_cast(int prec, int rows, int cols, const void* in, int ld_in, long long s_in,
                      const double* col_scale, long long s_scale, bool conj_t, void* out, int ld_out,
                      long long s_out, int n_traj, hipStream_t st) {
  long long total = (long long)n_traj * rows * cols;
  if (total <= 0) return hipSuccess;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  if (prec == 0) hipLaunchKernelGGL(k_scale_cast<float>, dim3(blocks), dim3(256), 0, st, rows, cols, (const c64d*)in, ld_in, s_in, col_scale, s_scale, conj_t, (c32*)out, ld_out, s_out, n_traj);
  else hipLaunchKernelGGL(k_scale_cast<double>, dim3(blocks), dim3(256), 0, st, rows, cols, (const c64d*)in, ld_in, s_in, col_scale, s_scale, conj_t, (c64d*)out, ld_out, s_out, n_traj);
  return hipGetLastError();
}

// ============================================================================ fill
template <typename T>
__global__ void k_init_sites(cplx<T>* state, const long long* __restrict__ site_off, const int* __restrict__ site_len,
                             int n_sites, long long s_traj, int n_traj) {
  // zero every site tensor, then A[0][0][0] = 1 (|0> with bond index 0)
  long long per = s_traj;
  long long total = per * n_traj;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    state[e] = cplx<T>{0, 0};
  }
}

template <typename T>
__global__ void k_set_one(cplx<T>* state, const long long* __restrict__ site_off, int n_sites, long long s_traj,
                          int n_traj) {
  int traj = blockIdx.x * blockDim.x + threadIdx.x;
  if (traj >= n_traj) return;
  for (int k = 0; k < n_sites; ++k) state[traj * s_traj + site_off[k]] = cplx<T>{(T)1, (T)0};
}

hipError_t init_state(int prec, void* state, const long long* d_site_off, int n_sites, long long s_traj,
                      int n_traj, hipStream_t st) {
  long long total = s_traj * n_traj;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  if (prec == 0) {
    hipLaunchKernelGGL(k_init_sites<float>, dim3(blocks), dim3(256), 0, st, (c32*)state, d_site_off, nullptr, n_sites, s_traj, n_traj);
    hipLaunchKernelGGL(k_set_one<float>, dim3((n_traj + 255) / 256), dim3(256), 0, st, (c32*)state, d_site_off, n_sites, s_traj, n_traj);
  } else {
    hipLaunchKernelGGL(k_init_sites<double>, dim3(blocks), dim3(256), 0, st, (c64d*)state, d_site_off, nullptr, n_sites, s_traj, n_traj);
    hipLaunchKernelGGL(k_set_one<double>, dim3((n_traj + 255) / 256), dim3(256), 0, st, (c64d*)state, d_site_off, n_sites, s_traj, n_traj);
  }
  return hipGetLastError();
}

}  // namespace mpsb
