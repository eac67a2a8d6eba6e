// Batched FP64 Hermitian eigensolver for the truncation Gram matrices and the centre hops.
//
// For each matrix (one workgroup per matrix and phase):
//   E1  blocked Householder reduction to tridiagonal form, A = Q T Q^dag,
//       Q = H_0 H_1 ... H_{n-3}, H_j = I - 2 u_j u_j^dag, only the lower triangle of A is read
//       or written; the reflector vectors overwrite the strict lower triangle;
//   E2  a diagonal phase similarity makes T real symmetric; the `keep` largest
//       eigenvalues by Sturm-count bisection (one thread per eigenvalue); eigenvectors of
//       the real tridiagonal by inverse iteration with partial-pivoting LU (one thread
//       per eigenvalue); eigenvalues <= zero_tol * lambda_max are dropped (value 0, vector
//       0: such directions carry no weight of the state);
//       clusters of relatively close eigenvalues are reorthogonalised inside the iteration;
//   E2b the kept vectors are orthonormalised in descending eigenvalue order (blocked
//       Gram-Schmidt with reorthogonalisation), which inverse iteration alone does not
//       guarantee for small eigenvalues with tiny absolute gaps;
//   E3  back-transformation evec = Q diag(omega) X with blocked compact-WY reflectors.
// Outputs: eigenvalues (descending), eigenvectors n x keep (row-major, ld keep) c128,
// the trace of the input and the sum of the kept eigenvalues.
#include <float.h>

#include "common.h"
#include "kernels.h"

namespace mpsb {

constexpr int ET = 256;           // threads per workgroup
constexpr int EMAX = 512;         // largest matrix dimension

// Cross-lane moves of doubles on the VALU, without the LDS crossbar: DPP within rows of 16
// lanes (quad_perm 0xB1 = lane ^ 1, 0x4E = lane ^ 2, row_half_mirror 0x141 = 7 - lane within
// 8, row_ror:8 0x128 = lane ^ 8) and the CDNA4 permlane swaps across rows.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// lanes 32..63 of a trade places with lanes 0..31 of b (permlane32_swap)
__device__ inline void swap_halves(double& a, double& b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// the odd 16-lane rows of a trade places with the even rows of b (permlane16_swap)
__device__ inline void swap_rows(double& a, double& b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// sum over the sub-groups of 8 lanes (lane & ~7), in every lane
__device__ inline double oct_sum(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  return x + dpp_f64<0x141>(x);
}

// sum over the 64 lanes, in every lane
__device__ inline double wave_sum(double x) {
  double y = x;
  swap_halves(x, y);
  x += y;
  y = x;
  swap_rows(x, y);
  x += y;
  x += dpp_f64<0x128>(x);
  return oct_sum(x);
}

template <int NT = ET>
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// q += V_r conj(W_c) + W_r conj(V_c), one complex element of a rank-2 update (fixed fma order)
__device__ inline void rank2_acc(c64d& q, c64d vr, c64d wr, c64d vc, c64d wc) {
  q.re = fma(vr.re, wc.re, q.re);
  q.re = fma(vr.im, wc.im, q.re);
  q.im = fma(vr.im, wc.re, q.im);
  q.im = fma(-vr.re, wc.im, q.im);
  q.re = fma(wr.re, vc.re, q.re);
  q.re = fma(wr.im, vc.im, q.re);
  q.im = fma(wr.im, vc.re, q.im);
  q.im = fma(-wr.re, vc.im, q.im);
}

// ---------------------------------------------------------------------------- E1
// Blocked Householder tridiagonalisation reading and writing only the lower triangle.
// Panels of NB columns are reduced with the trailing matrix kept in the deferred form
// A - 2 (V W^dag + W V^dag); each column needs one pass over the lower triangle of the
// trailing matrix (the matrix-vector product), and the panel's rank-2NB update is applied
// once at the end of the panel, in the same pass as the next panel's first matrix-vector
// product (so a panel of NB columns reads the trailing triangle NB times and writes it
// once).  The panel vectors live in LDS (column-major by vector, so
// that lanes read consecutive rows).  u_j is kept in column j below the diagonal.
// One workgroup per matrix runs a chain of dependent steps per column, so the time per
// matrix is set by latency rather than by HBM bandwidth: the row sums of the matrix-vector
// product are reduced on the VALU (permlane swaps and DPP, no LDS round trips), column slots
// past the trailing triangle are skipped, and WPE > 1 trades registers per wave for more
// waves per SIMD (two 512-thread workgroups per CU for n <= 256).  The n <= 128 instance
// keeps the update as a pass of its own (FUSE = false): the fused pass's registers would cost
// it a third workgroup per CU (measured 8% slower).
template <int NMAX, int NB, int RB, int NT, int WPE = 1, bool FUSE = true>
__global__ __launch_bounds__(NT, WPE) void k_tridiag(int n, c64d* __restrict__ Ag, long long sA, double* __restrict__ ws,
                                                long long sW, const int* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  static_assert(RB == 2 || RB == 4, "row blocks of 2 or 4 rows");
  __shared__ c64d Vt[NB][NMAX], Wt[NB][NMAX];
  __shared__ c64d su[NMAX], sp[NMAX];
  // column parts of the waves: waves NPART.. add theirs into part[wv - NPART] in a second step
  constexpr int NPART = NT / 64 > 4 ? 4 : NT / 64;
  __shared__ c64d part[NPART][NMAX];
  __shared__ c64d cdot[2 * NB];
  __shared__ double red[NT / 64];
  c64d* A = Ag + blockIdx.x * sA;
  double* W = ws + blockIdx.x * sW;
  double* d = W;                          // [n]
  c64d* ec = (c64d*)(W + n);              // [n]   subdiagonal T[j+1][j]
  double* tr = W + 3 * n;                 // [1]   trace
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int SLOTS = NMAX / 64;

  double t = 0;
  for (int i = tid; i < n; i += NT) t += A[(long long)i * n + i].re;
  t = block_sum<NT>(t, red);
  if (tid == 0) tr[0] = t;

  // The matrix-vector product below acts on column j, with m = n - j - 1 rows under the
  // diagonal; u at the lane's columns is held in registers across a pass when there are at
  // most 4 slots, read from LDS otherwise (register budget of the n <= 512 instance).
  int j = 0, m = 0;
  constexpr bool UK_REG = SLOTS <= 4 && NT <= 256;
  c64d colacc[SLOTS], ukv[UK_REG ? SLOTS : 1];
  auto start_product = [&]() {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int kk = lane + 64 * s;
      colacc[s] = c64d{0, 0};
      if constexpr (UK_REG) ukv[s] = su[kk < m ? kk : 0];
    }
  };
  // Row blocks of RB rows, NT / 64 * RB apart for a wave.  Slots past a block's last row
  // hold no element of the lower triangle and are skipped (wave-uniform), so the work
  // follows the triangle rather than NMAX.
  auto load_block = [&](c64d (&buf)[RB][SLOTS], int ib) {
    const int ns = (min(ib + RB, m) - 1) / 64 + 1;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int i = ib + rr;
      const c64d* row = A + (long long)(j + 1 + i) * n + (j + 1);
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int kk = lane + 64 * s;
        buf[rr][s] = (s < ns && i < m && kk <= i) ? row[kk] : c64d{0, 0};
      }
    }
  };
  // p = (lower-stored Hermitian A22) u on a block of rows: row parts by the wave (the RB rows'
  // sums into sp), column parts accumulated in registers (lane owns columns lane + 64 s).
  // One element a = A[i][kk] (kk = lane + 64 s, zero outside the triangle):
  auto mul_elem = [&](const c64d a, const c64d ui, int i, int s, double& pr, double& pim) {
    const int kk = lane + 64 * s;
    c64d uk;
    if constexpr (UK_REG) uk = ukv[s];
    else uk = su[kk < m ? kk : 0];
    pr = fma(a.re, uk.re, pr);
    pr = fma(-a.im, uk.im, pr);
    pim = fma(a.re, uk.im, pim);
    pim = fma(a.im, uk.re, pim);
    // strictly lower elements also act on row kk through A[kk][i] = conj(A[i][kk])
    const double cr = kk < i ? a.re : 0.0, ci = kk < i ? a.im : 0.0;
    colacc[s].re = fma(cr, ui.re, colacc[s].re);
    colacc[s].re = fma(ci, ui.im, colacc[s].re);
    colacc[s].im = fma(cr, ui.im, colacc[s].im);
    colacc[s].im = fma(-ci, ui.re, colacc[s].im);
  };
  // the row sums rs (re and im of each row of the block) over the wave, into sp: a
  // reduce-scatter butterfly over the 2 RB sums, each exchange halving the values a lane
  // carries (lanes 32..63, then odd rows, then lanes 8..15 of a row take the upper half), so
  // lane group g = lane / (32 / RB) ends with the full sum of value g
  auto store_rows = [&](double (&rs)[2 * RB], int ib) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      swap_halves(rs[q], rs[q + RB]);
      rs[q] += rs[q + RB];
    }
#pragma unroll
    for (int q = 0; q < RB / 2; ++q) {
      swap_rows(rs[q], rs[q + RB / 2]);
      rs[q] += rs[q + RB / 2];
    }
    if constexpr (RB == 4) {
      const bool up = (lane & 8) != 0;
      const double send = up ? rs[0] : rs[1];
      rs[0] = (up ? rs[1] : rs[0]) + dpp_f64<0x128>(send);
    } else {
      rs[0] += dpp_f64<0x128>(rs[0]);
    }
    rs[0] = oct_sum(rs[0]);
    if ((lane & (32 / RB - 1)) == 0) {
      const int g = lane / (32 / RB);
      if (ib + (g >> 1) < m) ((double*)&sp[ib + (g >> 1)])[g & 1] = rs[0];
    }
  };
  auto mul_block = [&](const c64d (&buf)[RB][SLOTS], int ib) {
    const int ns = (min(ib + RB, m) - 1) / 64 + 1;
    double rs[2 * RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int i = ib + rr;
      const c64d ui = i < m ? su[i] : c64d{0, 0};
      double pr = 0, pim = 0;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s)
        if (s < ns) mul_elem(buf[rr][s], ui, i, s, pr, pim);
      rs[2 * rr] = pr;
      rs[2 * rr + 1] = pim;
    }
    store_rows(rs, ib);
  };
  // the column parts of the waves into part[]: waves NPART.. add theirs in a second step
  auto store_parts = [&]() {
    if (wv < NPART) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int kk = lane + 64 * s;
        if (kk < m) part[wv][kk] = colacc[s];
      }
    }
  };
  // Householder reflector of column j from its corrected part below the diagonal in su:
  // u = (x + alpha e^{i arg x0} e_1) / |..| into su and column j of A, the subdiagonal
  // element of T into ec[j]
  auto reflect = [&]() {
    double s2 = 0;
    for (int i = tid; i < m; i += NT) s2 += norm2(su[i]);
    s2 = block_sum<NT>(s2, red);
    const double alpha = sqrt(s2);
    const c64d x0 = su[0];
    const double ax0 = sqrt(norm2(x0));
    const bool skip = !(alpha > 1e-300);
    const c64d ph = ax0 > 0 ? c64d{x0.re / ax0, x0.im / ax0} : c64d{1.0, 0.0};
    const double vn = skip ? 1.0 : sqrt(2.0 * alpha * (alpha + ax0));
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      c64d xi = su[i];
      if (i == 0) xi = xi + alpha * ph;
      c64d u = skip ? c64d{0, 0} : c64d{xi.re / vn, xi.im / vn};
      su[i] = u;
      A[(long long)(j + 1 + i) * n + j] = u;
    }
    if (tid == 0) ec[j] = skip ? x0 : c64d{-ph.re * alpha, -ph.im * alpha};
  };
  // w_k = p - (u^dag p) u with p = A22 u - 2 (V (W^dag u) + W (V^dag u)) over the panel's k
  // earlier vectors (cdot holds their dot products with u), after the parts are stored
  auto finish = [&](int k) {
    if constexpr (NT / 64 > NPART) {
      static_assert(NT / 64 <= 2 * NPART, "at most two waves per part row");
      if (wv >= NPART) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int kk = lane + 64 * s;
          if (kk < m) part[wv - NPART][kk] = part[wv - NPART][kk] + colacc[s];
        }
      }
      __syncthreads();
    }
    for (int i = tid; i < m; i += NT) {
      c64d p = sp[i];
#pragma unroll
      for (int w = 0; w < NPART; ++w) p = p + part[w][i];
      const int r = j + 1 + i;
      for (int kk = 0; kk < k; ++kk) {
        c64d corr = Vt[kk][r] * cdot[2 * kk + 1] + Wt[kk][r] * cdot[2 * kk];
        p = p - 2.0 * corr;
      }
      sp[i] = p;
    }
    __syncthreads();
    double kq = 0;
    for (int i = tid; i < m; i += NT) kq += su[i].re * sp[i].re + su[i].im * sp[i].im;
    kq = block_sum<NT>(kq, red);
    for (int r = tid; r <= j; r += NT) Wt[k][r] = c64d{0, 0};
    for (int i = tid; i < m; i += NT) Wt[k][j + 1 + i] = sp[i] - kq * su[i];
    __syncthreads();
  };

  // first: the panel's column 0 was already reduced by the previous panel's fused pass
  bool first_done = false;
  for (int j0 = 0; j0 + 2 < n; j0 += NB) {
    const int jb = min(NB, n - 2 - j0);
    for (int k = first_done ? 1 : 0; k < jb; ++k) {
      j = j0 + k;
      m = n - j - 1;
      // corrected column j (rows j..n-1) -> su (rows j+1..) and the diagonal
      for (int r = j + tid; r < n; r += NT) {
        c64d a = A[(long long)r * n + j];
        for (int kk = 0; kk < k; ++kk) {
          c64d corr = Vt[kk][r] * conj(Wt[kk][j]) + Wt[kk][r] * conj(Vt[kk][j]);
          a = a - 2.0 * corr;
        }
        if (r == j) d[j] = a.re;
        else su[r - j - 1] = a;
      }
      __syncthreads();
      reflect();
      for (int r = tid; r <= j; r += NT) Vt[k][r] = c64d{0, 0};
      __syncthreads();
      for (int i = tid; i < m; i += NT) Vt[k][j + 1 + i] = su[i];
      start_product();
      for (int i0 = wv * RB; i0 < m; i0 += (NT / 64) * RB) {
        c64d av[RB][SLOTS];
        load_block(av, i0);
        mul_block(av, i0);
      }
      store_parts();
      // dot products of the panel vectors with u (rows j+1..n-1)
      for (int dd = wv; dd < 2 * k; dd += NT / 64) {
        const int kk = dd >> 1;
        const bool isw = dd & 1;
        double cr = 0, ci = 0;
        for (int i = lane; i < m; i += 64) {
          c64d v = isw ? Wt[kk][j + 1 + i] : Vt[kk][j + 1 + i];
          c64d u = su[i];
          cr += v.re * u.re + v.im * u.im;
          ci += v.re * u.im - v.im * u.re;
        }
        cr = wave_sum(cr);
        ci = wave_sum(ci);
        if (lane == 0) cdot[dd] = c64d{cr, ci};   // even: V^dag u, odd: W^dag u
      }
      __syncthreads();
      finish(k);
    }
    // trailing update of the lower triangle, rows/cols >= t0:
    // A[r][c] -= 2 sum_k (V[r][k] conj(W[c][k]) + W[r][k] conj(V[c][k]))
    const int t0 = j0 + jb;
    if (FUSE && t0 + 2 < n) {
      // The next panel's first column is reduced here, fused with this update: column t0 of
      // the updated matrix first (with the update's own arithmetic), its reflector, then one
      // pass over the rows and columns past t0 that applies the update and accumulates the
      // reflector's matrix-vector product from the updated values in registers.  This saves
      // one read of the trailing triangle per panel; the results equal those of a separate
      // update followed by the product, bit for bit.
      j = t0;
      m = n - t0 - 1;
      for (int r = t0 + tid; r < n; r += NT) {
        c64d acc{0, 0};
        for (int kk = 0; kk < jb; ++kk) rank2_acc(acc, Vt[kk][r], Wt[kk][r], Vt[kk][t0], Wt[kk][t0]);
        const c64d xo = A[(long long)r * n + t0];
        const c64d a{fma(-2.0, acc.re, xo.re), fma(-2.0, acc.im, xo.im)};
        if (r == t0) d[t0] = a.re;
        else su[r - t0 - 1] = a;
      }
      __syncthreads();
      reflect();
      __syncthreads();
      start_product();
      for (int i0 = wv * RB; i0 < m; i0 += (NT / 64) * RB) {
        const int ns = (min(i0 + RB, m) - 1) / 64 + 1;
        double rs[2 * RB];
        c64d ui[RB];
        int rw[RB];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
          const int i = i0 + rr;
          ui[rr] = i < m ? su[i] : c64d{0, 0};
          rw[rr] = min(t0 + 1 + i, n - 1);
          rs[2 * rr] = 0;
          rs[2 * rr + 1] = 0;
        }
        // slot by slot: the update of the RB rows' elements in this slot, then their
        // contributions to the product (row sums and column parts in the same order as a
        // separate product over the stored values)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          if (s < ns) {
            const int kk = lane + 64 * s;
            const int c = min(t0 + 1 + kk, n - 1);
            c64d acc[RB];
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) acc[rr] = c64d{0, 0};
            for (int q = 0; q < jb; ++q) {
              const c64d vc = Vt[q][c], wc = Wt[q][c];
#pragma unroll
              for (int rr = 0; rr < RB; ++rr) rank2_acc(acc[rr], Vt[q][rw[rr]], Wt[q][rw[rr]], vc, wc);
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
              const int i = i0 + rr;
              c64d a{0, 0};
              if (i < m && kk <= i) {
                c64d* x = A + (long long)(t0 + 1 + i) * n + (t0 + 1 + kk);
                const c64d xo = *x;
                a = c64d{fma(-2.0, acc[rr].re, xo.re), fma(-2.0, acc[rr].im, xo.im)};
                *x = a;
              }
              mul_elem(a, ui[rr], i, s, rs[2 * rr], rs[2 * rr + 1]);
            }
          }
        }
        store_rows(rs, i0);
      }
      store_parts();
      __syncthreads();
      // the finished panel's vectors are no longer read: slot 0 takes the new reflector
      for (int r = tid; r <= t0; r += NT) Vt[0][r] = c64d{0, 0};
      for (int i = tid; i < m; i += NT) Vt[0][t0 + 1 + i] = su[i];
      finish(0);
      first_done = true;
      continue;
    }
    first_done = false;
    // the separate update (the last panel's, or every panel's without FUSE): rows/cols >= t0,
    // RB rows per wave and SLOTS columns per lane register-blocked
    // rows per wave in the trailing update: RB, except for the small instance under a tight
    // register budget, where one row per wave leaves room to load ahead (measured faster)
    constexpr int RBT = (WPE > 1 && NMAX <= 128) ? 1 : RB;
    for (int r0 = t0 + wv * RBT; r0 < n; r0 += (NT / 64) * RBT) {
      const int ns = (min(r0 + RBT, n) - 1 - t0) / 64 + 1;   // slots with columns <= last row
      // the current values are loaded first, so that their latency overlaps the accumulation,
      // where the registers allow it (full budget, or one row per wave); otherwise the other
      // waves on the SIMD cover it
      constexpr bool PRELOAD = WPE == 1 || RBT == 1;
      c64d x[PRELOAD ? RBT : 1][SLOTS], acc[RBT][SLOTS];
#pragma unroll
      for (int rr = 0; rr < RBT; ++rr) {
        const int r = r0 + rr;
        const c64d* row = A + (long long)r * n;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int c = t0 + lane + 64 * s;
          if constexpr (PRELOAD) x[rr][s] = (s < ns && r < n && c <= r) ? row[c] : c64d{0, 0};
          acc[rr][s] = c64d{0, 0};
        }
      }
      for (int kk = 0; kk < jb; ++kk) {
        c64d vr[RBT], wr[RBT];
#pragma unroll
        for (int rr = 0; rr < RBT; ++rr) {
          const int r = min(r0 + rr, n - 1);
          vr[rr] = Vt[kk][r];
          wr[rr] = Wt[kk][r];
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          if (s < ns) {
            const int c = min(t0 + lane + 64 * s, n - 1);
            const c64d vc = Vt[kk][c], wc = Wt[kk][c];
#pragma unroll
            for (int rr = 0; rr < RBT; ++rr) rank2_acc(acc[rr][s], vr[rr], wr[rr], vc, wc);
          }
        }
      }
#pragma unroll
      for (int rr = 0; rr < RBT; ++rr) {
        const int r = r0 + rr;
        if (r >= n) continue;
        c64d* row = A + (long long)r * n;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int c = t0 + lane + 64 * s;
          if (s < ns && c <= r) {
            const c64d xo = PRELOAD ? x[PRELOAD ? rr : 0][s] : row[c];
            row[c] = c64d{fma(-2.0, acc[rr][s].re, xo.re), fma(-2.0, acc[rr][s].im, xo.im)};
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(long long)(n - 2) * n + (n - 2)].re;
      d[n - 1] = A[(long long)(n - 1) * n + (n - 1)].re;
      ec[n - 2] = A[(long long)(n - 1) * n + (n - 2)];
    } else {
      d[0] = A[0].re;
    }
  }
}

// ---------------------------------------------------------------------------- E2
// Sturm counts: numbers of eigenvalues of the real symmetric tridiagonal (d, e) below x1 and
// below x2, from the pivots of the LDL^T factorisations of T - x (two independent chains
// interleaved).  1/q is the hardware reciprocal refined by one Newton step (relative error
// below 2^-50, a perturbation of e^2 of that order); pivots below pivmin are replaced by
// -pivmin.
__device__ inline double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ inline void sturm_count2(int n, const double* d, const double* e2, double x1, double x2, double pivmin,
                                    int& c1, int& c2) {
  int n1 = 0, n2 = 0;
  double q1 = d[0] - x1, q2 = d[0] - x2;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  if (fabs(q2) < pivmin) q2 = -pivmin;
  n1 += q1 < 0;
  n2 += q2 < 0;
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
    q1 = fma(-ei, recip(q1), di - x1);
    q2 = fma(-ei, recip(q2), di - x2);
    if (fabs(q1) < pivmin) q1 = -pivmin;
    if (fabs(q2) < pivmin) q2 = -pivmin;
    n1 += q1 < 0;
    n2 += q2 < 0;
  }
  c1 = n1;
  c2 = n2;
}

__device__ inline uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(ET) void k_tri_eig(int n, int keep, double zero_tol, double* __restrict__ ws, long long sW,
                                                double* __restrict__ evals, long long sE, double* __restrict__ kept_sum,
                                                const int* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  __shared__ double sd[EMAX], se[EMAX], se2[EMAX];
  __shared__ c64d sph[EMAX];   // phases of the subdiagonal
  __shared__ double red[ET / 64];
  __shared__ double s_bounds[3];
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
    const c64d e = (i + 1 < n) ? ec[i] : c64d{0.0, 0.0};
    double a = (i + 1 < n) ? sqrt(norm2(e)) : 0.0;
    se[i] = a;
    se2[i] = a * a;
    sph[i] = a > 0 ? c64d{e.re / a, e.im / a} : c64d{1.0, 0.0};
  }
  __syncthreads();
  if (tid == 0) {
    c64d w = {1.0, 0.0};
    om[0] = w;
#pragma unroll 8
    for (int i = 0; i + 1 < n; ++i) {
      if (se[i] > 0) w = w * sph[i];
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
    double dmax = 0;
    for (int i = 0; i < n; ++i) dmax = fmax(dmax, sd[i]);
    s_bounds[2] = dmax;   // lambda_max >= the largest diagonal entry
  }
  __syncthreads();
  const double glo = s_bounds[0], ghi = s_bounds[1];
  // an eigenvalue whose bracket lies below zero_tol * (lower bound of lambda_max) is dropped
  // whatever its exact value, so its bisection stops there
  const double cut_lb = zero_tol * s_bounds[2];
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  double emax2 = 0;
  for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, se2[i]);
  const double pivmin = DBL_MIN * fmax(1.0, emax2);

  // ---- shared multisection: the counts below 2 ET points (the Gershgorin ends and a
  // geometric grid between the zero-weight cut and the upper end, where the kept eigenvalues
  // of a Gram matrix lie), one Sturm pass with two points per thread; every eigenvalue then
  // starts its trisection from the tightest bracket of the grid
  __shared__ double gx[2 * ET];
  __shared__ int gc[2 * ET];
  {
    constexpr int NPT = 2 * ET;
    const double top = ghi, bot = fmax(cut_lb, top * 1e-300);
    const double lr = (top > bot && bot > 0) ? log(top / bot) : 0.0;
    double x[2];
    for (int h = 0; h < 2; ++h) {
      const int p = 2 * tid + h;
      if (p == 0) x[h] = glo;
      else if (p == NPT - 1 || !(lr > 0)) x[h] = ghi;
      else x[h] = fmin(ghi, fmax(glo, bot * exp(lr * (double)(p - 1) / (double)(NPT - 2))));
    }
    int c0, c1;
    sturm_count2(n, sd, se2, x[0], x[1], pivmin, c0, c1);
    gx[2 * tid] = x[0];
    gx[2 * tid + 1] = x[1];
    gc[2 * tid] = c0;
    gc[2 * tid + 1] = c1;
  }
  __syncthreads();

  // ---- bisection for the keep largest eigenvalues
  for (int k = tid; k < keep; k += ET) {
    const int idx = n - 1 - k;   // ascending index
    // trisection: count(lo) <= idx < count(hi) is kept; start from the grid points (ascending,
    // counts nondecreasing) that bracket idx most tightly
    double lo = glo, hi = ghi;
    for (int p = 0; p < 2 * ET; ++p) {
      if (gc[p] <= idx) lo = fmax(lo, gx[p]);
      else hi = fmin(hi, gx[p]);
    }
    for (int it = 0; it < 140; ++it) {
      const double w = hi - lo;
      const double m1 = lo + w * (1.0 / 3.0), m2 = lo + w * (2.0 / 3.0);
      if (w <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin || m1 <= lo || m2 >= hi || m2 <= m1 ||
          hi <= cut_lb)
        break;
      int c1, c2;
      sturm_count2(n, sd, se2, m1, m2, pivmin, c1, c2);
      if (c1 > idx) hi = m1;
      else if (c2 > idx) { lo = m1; hi = m2; }
      else lo = m2;
    }
    ev[k] = 0.5 * (lo + hi);
  }
  __syncthreads();
  const double lmax = ev[0];
  const double cut = fmax(zero_tol * fmax(lmax, 0.0), 1e-300);

  // ---- clusters of relatively close kept eigenvalues (gap < 1e-3 of the eigenvalue):
  // their vectors are computed by one thread, each orthogonalised against the previous
  // members of its cluster after every solve.  Other eigenvalues are isolated relative to
  // their size, so inverse iteration alone yields vectors accurate to eps * lambda_max / gap.
  __shared__ short cl_end[EMAX];
  if (tid == 0) {
    int k = 0;
    while (k < keep) {
      int e = k + 1;
      while (e < keep && ev[e - 1] > cut && ev[e] > cut && (ev[e - 1] - ev[e]) < 1e-3 * ev[e - 1]) ++e;
      for (int q = k; q < e; ++q) cl_end[q] = (short)(q == k ? e : -1);
      k = e;
    }
  }
  __syncthreads();
  for (int k0 = tid; k0 < keep; k0 += ET) {
    const int kend = cl_end[k0];
    if (kend < 0) continue;
    for (int k = k0; k < kend; ++k) {
      const double lam = ev[k];
      if (!(lam > cut)) {
        for (int i = 0; i < n; ++i) X[(long long)i * keep + k] = 0.0;
        continue;
      }
      // perturbed shift so that the factorisation is never exactly singular
      const double sig = lam + 4.0 * DBL_EPSILON * tnorm * (1.0 + 0.37 * (k & 7));
      const double tiny = DBL_EPSILON * tnorm + 1e-300;
      double cd = sd[0] - sig, cs = (n > 1) ? se[0] : 0.0;
      for (int i = 0; i + 1 < n; ++i) {
        const double sub = se[i], nd = sd[i + 1] - sig, ns = (i + 2 < n) ? se[i + 1] : 0.0;
        const int o = i * keep + k;   // < 2^17
        if (fabs(cd) >= fabs(sub)) {
          double l = (cd != 0.0) ? sub / cd : 0.0;
          U0[o] = 1.0 / ((cd != 0.0) ? cd : tiny);
          U1[o] = cs;
          U2[o] = 0.0;
          L[o] = l;
          PV[o] = 0.0;
          cd = nd - l * cs;
          cs = ns;
        } else {
          double l = cd / sub;
          U0[o] = 1.0 / sub;
          U1[o] = nd;
          U2[o] = ns;
          L[o] = l;
          PV[o] = 1.0;
          cd = cs - l * nd;
          cs = -l * ns;
        }
      }
      U0[(long long)(n - 1) * keep + k] = 1.0 / ((cd != 0.0) ? cd : tiny);
      // two solves: the first from a pseudo-random right-hand side generated on the fly, the
      // second from the first's result scaled by 1 / max|y| while it is read; the 2-norm of the
      // last solve is accumulated as it is written.  U0 holds the reciprocal pivots, and the
      // factors are loaded CH steps at a time, so that the dependent chain of a solve waits
      // for memory once per chunk rather than once per step.
      constexpr int CH = 4;
      double sc = 1.0, nn2 = 0.0;
      for (int itr = 0; itr < 2; ++itr) {
        if (itr > 0) {
          double xcur = X[k] * sc;
          for (int ib = 0; ib + 1 < n; ib += CH) {
            double xa[CH], pa[CH], la[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
              const int i = ib + q;
              if (i + 1 < n) {
                const int o = i * keep + k;   // < 2^17
                xa[q] = X[o + keep];
                pa[q] = PV[o];
                la[q] = L[o];
              }
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
              const int i = ib + q;
              if (i + 1 < n) {
                double xi = xcur, xn = xa[q] * sc;
                if (pa[q] != 0.0) { double tmp = xi; xi = xn; xn = tmp; }
                xn -= la[q] * xi;
                X[i * keep + k] = xi;
                xcur = xn;
              }
            }
          }
          X[(long long)(n - 1) * keep + k] = xcur;
        }
        double y1 = 0.0, y2 = 0.0, mx = 0.0;
        nn2 = 0.0;
        for (int ib = n - 1; ib >= 0; ib -= CH) {
          double xa[CH], u0[CH], u1[CH], u2[CH];
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int i = ib - q;
            if (i >= 0) {
              const int o = i * keep + k;   // < 2^17
              xa[q] = itr == 0 ? 0.5 + (hash32((uint32_t)(i * 7919 + k * 104729 + 17)) >> 8) * (1.0 / 16777216.0) : X[o];
              u0[q] = U0[o];
              u1[q] = U1[o];
              u2[q] = U2[o];
            }
          }
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int i = ib - q;
            if (i >= 0) {
              double v = xa[q];
              if (i + 1 < n) v -= u1[q] * y1;
              if (i + 2 < n) v -= u2[q] * y2;
              const double y = v * u0[q];
              X[i * keep + k] = y;
              y2 = y1;
              y1 = y;
              mx = fmax(mx, fabs(y));
              nn2 += y * y;
            }
          }
        }
        sc = (mx > 0) ? 1.0 / mx : 1.0;
        // orthogonalise against the previous (finished, unit) members of the cluster
        for (int p = k0; p < k; ++p) {
          double dot = 0;
          for (int i = 0; i < n; ++i) dot += X[(long long)i * keep + p] * X[(long long)i * keep + k];
          for (int i = 0; i < n; ++i) X[(long long)i * keep + k] -= dot * X[(long long)i * keep + p];
        }
        if (itr == 0) continue;   // the unit 2-norm is only needed for the final vector
        if (k > k0) {   // the orthogonalisation changed the vector
          nn2 = 0;
          for (int r = 0; r < n; ++r) {
            const double y = X[(long long)r * keep + k];
            nn2 += y * y;
          }
        }
        const double inv = nn2 > 0 ? 1.0 / sqrt(nn2) : 0.0;
        for (int i = 0; i < n; ++i) X[(long long)i * keep + k] *= inv;
      }
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

// ---------------------------------------------------------------------------- E2b
// Orthonormalisation of the tridiagonal eigenvectors in descending eigenvalue order.
// Inverse iteration gives vector k an error of about eps lambda_max / |lambda_k - lambda_j|
// along eigenvector j, so the vectors of small eigenvalues whose absolute gaps are tiny
// (although their relative gaps are not) come out far from orthogonal; a truncation with
// such vectors no longer projects the state.  Every kept vector is therefore projected out
// of all vectors before it (the Q factor of the QR factorisation of the vectors in
// descending order): blocks of 16 columns are projected against the finished columns in
// chunks of 16 (block modified Gram-Schmidt, two passes; the chunk products W = X_c^T B and
// B -= X_c W run on FP64 16x16x4 MFMAs, the first split over the four waves by rows and
// summed in LDS, with the next chunk's loads in flight), then orthonormalised inside by
// Cholesky QR, twice (Gram matrix on MFMAs, 16 x 16 Cholesky factor and its inverse on one
// wave in LDS, B <- B R^-1 on MFMAs).  Vectors of well-separated eigenvalues change at rounding
// level.  A column whose relative norm after its projections falls below 1e-4 is projected
// once more (one more round); below 1e-7 (the resolution of a Gram-based factor) it carries
// no reliable direction: it is left out of the factor and refilled with a pseudo-random
// vector orthogonalised the same way in the next round, so that the kept vectors stay a
// complete orthonormal set.  Columns of dropped eigenvalues stay zero.
typedef double v4d_t __attribute__((ext_vector_type(4)));
__device__ inline v4d_t mfma64(double a, double b, v4d_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <int NMAX>
__global__ __launch_bounds__(ET) void k_tri_orth(int n, int keep, double* __restrict__ ws, long long sW,
                                                 const double* __restrict__ evals, long long sE,
                                                 const int* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  constexpr int BW = 16, S = BW + 1;   // row stride of the LDS panels (odd: rows fall in different banks)
  constexpr int PF = NMAX * BW / ET;   // chunk elements loaded ahead per thread
  __shared__ double Bs[NMAX * S];      // the block, [i][j]; rows n .. NP-1 are zero
  __shared__ double Xs[NMAX * S];      // a chunk of finished columns, [i][kk]; rows n .. NP-1 zero
  __shared__ double Wpart[4 * BW * BW];   // the waves' partial products
  __shared__ double Wp[BW * BW];       // projections on the chunk [kk][j], or Gram / Cholesky factor [k][j]
  __shared__ double rho[BW];           // relative norms of the block's columns after their projections
  __shared__ double gdiag[BW];         // diagonal of the block's Gram matrix
  __shared__ int s_nk, s_redo;
  static_assert(ET == 256, "one element of W per thread");
  double* X = ws + blockIdx.x * sW + 6 * (long long)n;
  const double* ev = evals + blockIdx.x * sE;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;   // MFMA operand coordinates of a lane
  if (tid == 0) {
    int nk = 0;
    while (nk < keep && ev[nk] > 0.0) ++nk;
    s_nk = nk;
  }
  __syncthreads();
  const int nk = s_nk;
  const int NP = (n + 15) & ~15;       // rows rounded up to whole 16-row tiles

  // W = (sum over 4-row steps of A^T B) for two row-major NP x 16 panels in LDS, summed over
  // the waves into Wp
  auto panel_product = [&](const double* A, const double* B) {
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int st = wv; st < (NP >> 2); st += 4) {
      const int r = 4 * st + lk;
      acc = mfma64(A[r * S + li], B[r * S + li], acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Wpart[wv * BW * BW + (lk + 4 * q) * BW + li] = acc[q];
    __syncthreads();
    Wp[tid] = (Wpart[tid] + Wpart[BW * BW + tid]) + (Wpart[2 * BW * BW + tid] + Wpart[3 * BW * BW + tid]);
    __syncthreads();
  };

  for (int c0 = 0; c0 < nk; c0 += BW) {
    const int pc = min(BW, nk - c0);
    for (int e = tid; e < NP * BW; e += ET) {
      const int i = e >> 4, j = e & 15;
      Bs[i * S + j] = (i < n && j < pc) ? X[(long long)i * keep + c0 + j] : 0.0;
    }
    for (int round = 0; round < 3; ++round) {
      // two passes over the finished columns, chunk by chunk; chunk t of the sequence is
      // columns 16 (t mod (c0 / 16)) .. + 15, loaded one step ahead into registers
      const int nch = c0 / BW, nseq = 2 * nch;
      double pf[PF];
      auto fetch = [&](int t) {
        const int k0 = (t % nch) * BW;
#pragma unroll
        for (int m = 0; m < PF; ++m) {
          const int e = tid + m * ET, i = e >> 4, kk = e & 15;
          pf[m] = (e < NP * BW && i < n) ? X[(long long)i * keep + k0 + kk] : 0.0;
        }
      };
      if (nseq > 0) fetch(0);
      for (int t = 0; t < nseq; ++t) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PF; ++m) {
          const int e = tid + m * ET;
          if (e < NP * BW) Xs[(e >> 4) * S + (e & 15)] = pf[m];
        }
        __syncthreads();
        if (t + 1 < nseq) fetch(t + 1);
        panel_product(Xs, Bs);   // W[kk][j] = sum_i Xs[i][kk] Bs[i][j]
        // Bs[i][j] -= sum_kk Xs[i][kk] W[kk][j], one 16-row tile per wave at a time
        for (int rt = wv; rt < (NP >> 4); rt += 4) {
          v4d_t c;
#pragma unroll
          for (int q = 0; q < 4; ++q) c[q] = Bs[(16 * rt + lk + 4 * q) * S + li];
#pragma unroll
          for (int st = 0; st < 4; ++st) c = mfma64(-Xs[(16 * rt + li) * S + 4 * st + lk], Wp[(4 * st + lk) * BW + li], c);
#pragma unroll
          for (int q = 0; q < 4; ++q) Bs[(16 * rt + lk + 4 * q) * S + li] = c[q];
        }
      }
      __syncthreads();
      // inside the block: Cholesky QR, twice
      for (int cp = 0; cp < 2; ++cp) {
        panel_product(Bs, Bs);   // Gram matrix G[k][j] in Wp
        if (wv == 0) {
          // G = R^T R on one wave, in place in LDS (upper triangle); pivots below 1e-14 of the
          // column's squared norm leave the column out (R_kk = 1, rest of row k zero)
          if (lane < BW) gdiag[lane] = Wp[lane * BW + lane];
          __builtin_amdgcn_wave_barrier();
          for (int k = 0; k < BW; ++k) {
            const double gkk = Wp[k * BW + k], g0 = gdiag[k];
            const bool ok = k < pc && g0 > 0.0 && gkk > 1e-14 * g0;
            if (cp == 0 && lane == 0) rho[k] = (k < pc && g0 > 0.0) ? sqrt(fmax(gkk, 0.0) / g0) : 1.0;
            const double rkk = ok ? sqrt(gkk) : 1.0;
            __builtin_amdgcn_wave_barrier();
            if (lane < BW) {
              const double v = Wp[k * BW + lane];
              Wp[k * BW + lane] = lane > k ? (ok ? v / rkk : 0.0) : (lane == k ? rkk : 0.0);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int m = 0; m < BW * BW / 64; ++m) {
              const int e = lane + 64 * m, i = e >> 4, j = e & 15;
              if (i > k && j >= i) Wp[e] = fma(-Wp[k * BW + i], Wp[k * BW + j], Wp[e]);
            }
            __builtin_amdgcn_wave_barrier();
          }
          // R^-1 into Wpart, lane j < 16 computing column j by back-substitution
          if (lane < BW) {
            const int j = lane;
            for (int i = 0; i < BW; ++i) Wpart[i * BW + j] = 0.0;
            Wpart[j * BW + j] = 1.0 / Wp[j * BW + j];
            for (int i = j - 1; i >= 0; --i) {
              double acc = 0.0;
              for (int k = i + 1; k <= j; ++k) acc = fma(Wp[i * BW + k], Wpart[k * BW + j], acc);
              Wpart[i * BW + j] = -acc / Wp[i * BW + i];
            }
          }
        }
        __syncthreads();
        // B <- B R^-1 on MFMAs, one 16-row tile per wave at a time (a tile is read before it
        // is overwritten)
        for (int rt = wv; rt < (NP >> 4); rt += 4) {
          double a[4];
#pragma unroll
          for (int st = 0; st < 4; ++st) a[st] = Bs[(16 * rt + li) * S + 4 * st + lk];
          v4d_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int st = 0; st < 4; ++st) c = mfma64(a[st], Wpart[(4 * st + lk) * BW + li], c);
#pragma unroll
          for (int q = 0; q < 4; ++q) Bs[(16 * rt + lk + 4 * q) * S + li] = c[q];
        }
        __syncthreads();
      }
      // a column that cancelled to below 1e-4 of its norm is projected once more (one more
      // round); one below 1e-7 is refilled with a pseudo-random vector first
      if (tid == 0) {
        int redo = 0;
        for (int j = 0; j < pc; ++j) redo |= rho[j] < 1e-4;
        s_redo = redo;
      }
      __syncthreads();
      if (!s_redo || round == 2) break;
      for (int e = tid; e < n * BW; e += ET) {
        const int i = e >> 4, j = e & 15;
        if (j < pc && rho[j] < 1e-7)
          Bs[i * S + j] = (double)(hash32((uint32_t)(i * 7919 + (c0 + j) * 104729 + round * 15485863 + 3)) >> 8) *
                              (1.0 / 16777216.0) - 0.5;
      }
      __syncthreads();
    }
    // the block is finished: write it back
    for (int e = tid; e < n * BW; e += ET) {
      const int i = e >> 4, j = e & 15;
      if (j < pc) X[(long long)i * keep + c0 + j] = Bs[i * S + j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- E3
// evec = Q diag(omega) X, Q = H_0 ... H_{n-3} with u_j in column j below the diagonal;
// reflectors are applied in blocks of NB from the last block to the first as
// (I - V T V^dag), with V staged in LDS.  Thread c owns column c of Z (and, when keep is
// smaller than the workgroup, one of several row slices of it).
template <int NMAX, int NB>
__global__ __launch_bounds__(ET) void k_backtransform(int n, int keep, const c64d* __restrict__ Ag, long long sA,
                                                      double* __restrict__ ws, long long sW,
                                                      c64d* __restrict__ Zg, long long sZ, const int* __restrict__ mask) {
  if (mask && !mask[blockIdx.x]) return;
  __shared__ c64d Vb[NMAX][NB];
  __shared__ c64d Tm[NB][NB];
  __shared__ c64d Sv[NB][NB];
  __shared__ c64d Wred[ET][NB];
  const c64d* A = Ag + blockIdx.x * sA;
  double* W = ws + blockIdx.x * sW;
  const c64d* om = (const c64d*)(W + 4 * n);
  const double* X = W + 6 * n;
  c64d* Z = Zg + blockIdx.x * sZ;
  const int tid = threadIdx.x;
  const int nslice = keep >= ET ? 1 : ET / keep;           // row slices per column
  const int c = tid % keep, slice = tid / keep;
  const bool active = tid < keep * nslice;
  // Z = diag(omega) X
  for (int i = tid; i < n * keep; i += ET) {
    const int r = i / keep;
    const double x = X[i];
    Z[i] = c64d{om[r].re * x, om[r].im * x};
  }
  __syncthreads();
  const int nref = n - 2;
  if (nref <= 0) return;
  const int nblk = (nref + NB - 1) / NB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = blk * NB, nb = min(NB, nref - j0);
    for (int e = tid; e < n * NB; e += ET) {
      const int i = e / NB, a = e % NB;
      const int ja = j0 + a;
      Vb[i][a] = (a < nb && i > ja) ? A[(long long)i * n + ja] : c64d{0, 0};
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += ET) {
      const int a = e / nb, b = e % nb;
      c64d s = {0, 0};
      for (int i = j0 + 1; i < n; ++i) s = s + cmulc(Vb[i][a], Vb[i][b]);
      Sv[a][b] = s;
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += ET) Tm[e / NB][e % NB] = c64d{0, 0};
    __syncthreads();
    for (int jj = 0; jj < nb; ++jj) {
      if (tid < jj) {
        const int a = tid;
        c64d s = {0, 0};
        for (int b = a; b < jj; ++b) s = s + Tm[a][b] * Sv[b][jj];
        Tm[a][jj] = -2.0 * s;
      }
      if (tid == 0) Tm[jj][jj] = c64d{2.0, 0.0};
      __syncthreads();
    }
    // Wt = V^dag Z (column c, partial over this thread's row slice)
    c64d acc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) acc[a] = c64d{0, 0};
    if (active) {
      int i = j0 + 1 + slice;
      for (; i + 3 * nslice < n; i += 4 * nslice) {
        c64d z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = Z[(long long)(i + u * nslice) * keep + c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int a = 0; a < NB; ++a) acc[a] = acc[a] + cmulc(Vb[i + u * nslice][a], z[u]);
      }
      for (; i < n; i += nslice) {
        const c64d z = Z[(long long)i * keep + c];
#pragma unroll
        for (int a = 0; a < NB; ++a) acc[a] = acc[a] + cmulc(Vb[i][a], z);
      }
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) Wred[tid][a] = acc[a];
    __syncthreads();
    c64d wt[NB];
    if (active) {
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        c64d s = {0, 0};
        for (int q = 0; q < nslice; ++q) s = s + Wred[q * keep + c][a];
        wt[a] = s;
      }
      // wt <- T wt
      c64d tw[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        c64d s = {0, 0};
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b >= a && b < nb) s = s + Tm[a][b] * wt[b];
        tw[a] = s;
      }
      // Z -= V tw
      int i = j0 + 1 + slice;
      for (; i + 3 * nslice < n; i += 4 * nslice) {
        c64d z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = Z[(long long)(i + u * nslice) * keep + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c64d s = {0, 0};
#pragma unroll
          for (int a = 0; a < NB; ++a) s = s + Vb[i + u * nslice][a] * tw[a];
          Z[(long long)(i + u * nslice) * keep + c] = z[u] - s;
        }
      }
      for (; i < n; i += nslice) {
        c64d s = {0, 0};
#pragma unroll
        for (int a = 0; a < NB; ++a) s = s + Vb[i][a] * tw[a];
        Z[(long long)i * keep + c] = Z[(long long)i * keep + c] - s;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- E3 (MFMA)
// Panel form of the back-transformation on FP64 16x16x4 MFMAs.  E3a computes, once per
// matrix, the compact-WY factor T of every block of 16 reflectors (I - V T V^dag =
// H_j0 ... H_j0+nb-1) from S = V^dag V into the workspace.  E3b gives each workgroup a panel
// of 16 eigenvector columns: the panel Z = diag(omega) X[:, panel] stays in LDS while the
// blocks are applied from the last to the first (W = V^dag Z, W <- T W, Z -= V W), V read
// from the matrix as MFMA operands (the panels of one matrix share it in L2: workgroups are
// numbered so that they run on one XCD); the panel is written out once.
// MFMA lane layout (f64 16x16x4): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i % 4), register i / 4.
// workspace per matrix: d, e, trace, omega, X and the inverse-iteration arrays (6 n + 6 n keep
// doubles), then the T factors (2 * 16 * 16 doubles per block of 16 reflectors)
__host__ __device__ inline size_t bt_tfac_offset(int n, int keep) { return (size_t)6 * n + (size_t)6 * n * keep + 64; }

__global__ __launch_bounds__(256) void k_bt_tfac(int n, const c64d* __restrict__ Ag, long long sA, double* __restrict__ ws,
                                                 long long sW, int keep, const int* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  __shared__ double Sp[4][2][16][16];
  __shared__ c64d Sv[16][16];
  __shared__ c64d Tm[16][16];
  const c64d* A = Ag + blockIdx.x * sA;
  double* W = ws + blockIdx.x * sW;
  c64d* Tout = (c64d*)(W + bt_tfac_offset(n, keep));
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  const int nref = n - 2;
  const int nblk = nref > 0 ? (nref + 15) / 16 : 0;
  for (int blk = 0; blk < nblk; ++blk) {
    const int j0 = 16 * blk, nb = min(16, nref - j0);
    // S[a][b] = sum_i conj(V[i][a]) V[i][b]; lane r16 + 16 kq holds V[row][r16] for both operands
    v4d_t sr = {0, 0, 0, 0}, si = {0, 0, 0, 0};
    for (int i0 = j0 + 1 + 4 * wv; i0 < n; i0 += 16) {
      const int row = i0 + kq;
      c64d v = {0, 0};
      if (row < n && r16 < nb && row > j0 + r16) v = A[(long long)row * n + j0 + r16];
      sr = mfma64(v.re, v.re, sr);
      sr = mfma64(v.im, v.im, sr);
      si = mfma64(v.re, v.im, si);
      si = mfma64(-v.im, v.re, si);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Sp[wv][0][kq + 4 * r][r16] = sr[r];
      Sp[wv][1][kq + 4 * r][r16] = si[r];
    }
    __syncthreads();
    {
      const int a = tid >> 4, b = tid & 15;
      Sv[a][b] = c64d{Sp[0][0][a][b] + Sp[1][0][a][b] + Sp[2][0][a][b] + Sp[3][0][a][b],
                      Sp[0][1][a][b] + Sp[1][1][a][b] + Sp[2][1][a][b] + Sp[3][1][a][b]};
      Tm[a][b] = c64d{0, 0};
    }
    __syncthreads();
    for (int jj = 0; jj < nb; ++jj) {
      if (tid < jj) {
        const int a = tid;
        c64d s = {0, 0};
        for (int b = a; b < jj; ++b) s = s + Tm[a][b] * Sv[b][jj];
        Tm[a][jj] = -2.0 * s;
      }
      if (tid == 0) Tm[jj][jj] = c64d{2.0, 0.0};
      __syncthreads();
    }
    Tout[(long long)blk * 256 + tid] = Tm[tid >> 4][tid & 15];
    __syncthreads();
  }
}

template <int NMAX, int BNT>
__global__ __launch_bounds__(BNT, BNT / 128) void k_bt_panel(int n, int keep, const c64d* __restrict__ Ag, long long sA,
                                                  const double* __restrict__ ws, long long sW, c64d* __restrict__ Zg,
                                                  long long sZ, int n_panels, const int* __restrict__ active) {
  // 80 KB of LDS so that two panels share a CU: the panel (rows of 16 doubles read 4 rows at
  // a time: conflict-free without padding), three slots of partial W (and, while W is folded,
  // the W arrays as a fourth) and the reduced W
  static_assert(BNT == 256 || BNT == 512, "four or eight waves");
  constexpr int NW = BNT / 64;
  __shared__ double Zr[NMAX][16], Zi[NMAX][16];
  __shared__ __align__(16) double Wp[3][2][16][16];   // partial W sums, then this block's T factor
  __shared__ double Wr[16][16], Wi[16][16];
  // XCD-aware numbering: the panels of a matrix are consecutive logical ids on one XCD
  const int G = gridDim.x, w = blockIdx.x;
  const int q8 = G >> 3, r8 = G & 7, x8 = w & 7;
  const int L = x8 * q8 + min(x8, r8) + (w >> 3);
  const int mat = L / n_panels, panel = L - mat * n_panels;
  if (active && !active[mat]) return;
  const c64d* A = Ag + mat * sA;
  const double* W = ws + mat * sW;
  const c64d* om = (const c64d*)(W + 4 * n);
  const double* X = W + 6 * n;
  const c64d* Tg = (const c64d*)(W + bt_tfac_offset(n, keep));
  c64d* Z = Zg + mat * sZ;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  const int c0 = panel * 16, pc = min(16, keep - c0);
  for (int e = tid; e < n * 16; e += BNT) {
    const int r = e >> 4, c = e & 15;
    const double x = c < pc ? X[(long long)r * keep + c0 + c] : 0.0;
    Zr[r][c] = om[r].re * x;
    Zi[r][c] = om[r].im * x;
  }
  __syncthreads();
  const int nref = n - 2;
  const int nblk = nref > 0 ? (nref + 15) / 16 : 0;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = 16 * blk, nb = min(16, nref - j0);
    // this block's T factor, one element per thread of the first 256: loaded now, so that its
    // latency is hidden behind the W accumulation, and put into LDS once the partial W sums
    // are consumed
    const c64d tfac = tid < 256 ? Tg[(long long)blk * 256 + tid] : c64d{0, 0};
    // W[a][c] = sum_rows conj(V[row][a]) Z[row][c]; groups of four waves take chunks of 16 NCH
    // rows, NCH independent accumulator chains per wave (rows i0, i0 + 16, ...)
    constexpr int NCH = NW == 8 ? 2 : 4;   // accumulator chains per wave (register budget)
    v4d_t wr[NCH], wi[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) wr[h] = wi[h] = v4d_t{0, 0, 0, 0};
    for (int i0 = j0 + 1 + 4 * (wv & 3) + 16 * NCH * (wv >> 2); i0 < n; i0 += 4 * NCH * NW) {
      c64d v[NCH];
      double zr[NCH], zi[NCH];
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        const int row = i0 + 16 * h + kq;
        v[h] = c64d{0, 0};
        zr[h] = zi[h] = 0;
        if (row < n) {
          if (r16 < nb && row > j0 + r16) v[h] = A[(long long)row * n + j0 + r16];
          zr[h] = Zr[row][r16];
          zi[h] = Zi[row][r16];
        }
      }
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        wr[h] = mfma64(v[h].re, zr[h], wr[h]);
        wi[h] = mfma64(v[h].re, zi[h], wi[h]);
      }
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        wr[h] = mfma64(v[h].im, zi[h], wr[h]);
        wi[h] = mfma64(-v[h].im, zr[h], wi[h]);
      }
    }
    v4d_t wr0, wi0;
    if constexpr (NCH == 4) {
      wr0 = (wr[0] + wr[1]) + (wr[2] + wr[3]);
      wi0 = (wi[0] + wi[1]) + (wi[2] + wi[3]);
    } else {
      wr0 = wr[0] + wr[1];
      wi0 = wi[0] + wi[1];
    }
    if constexpr (NW == 8) {
      // first fold: waves 4-7 hand their sums to waves 0-3 (slots Wp[0..2] and the W arrays,
      // which the previous block no longer reads)
      if (wv >= 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = kq + 4 * r;
          if (wv < 7) {
            Wp[wv - 4][0][a][r16] = wr0[r];
            Wp[wv - 4][1][a][r16] = wi0[r];
          } else {
            Wr[a][r16] = wr0[r];
            Wi[a][r16] = wi0[r];
          }
        }
      }
      __syncthreads();
      if (wv < 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = kq + 4 * r;
          if (wv < 3) {
            wr0[r] += Wp[wv][0][a][r16];
            wi0[r] += Wp[wv][1][a][r16];
          } else {
            wr0[r] += Wr[a][r16];
            wi0[r] += Wi[a][r16];
          }
        }
      }
      __syncthreads();
    }
    if (wv > 0 && wv < 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Wp[wv - 1][0][kq + 4 * r][r16] = wr0[r];
        Wp[wv - 1][1][kq + 4 * r][r16] = wi0[r];
      }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = kq + 4 * r;
        Wr[a][r16] = wr0[r] + Wp[0][0][a][r16] + Wp[1][0][a][r16] + Wp[2][0][a][r16];
        Wi[a][r16] = wi0[r] + Wp[0][1][a][r16] + Wp[1][1][a][r16] + Wp[2][1][a][r16];
      }
    }
    __syncthreads();
    // the partial sums have been read: their space holds T for the product below
    c64d* Ts = (c64d*)&Wp[0][0][0][0];
    if (tid < 256) Ts[tid] = tfac;
    __syncthreads();
    {
      // W <- T W (T upper triangular), one (a, c) per thread of the first 256
      const int a = (tid >> 4) & 15, c = tid & 15;
      double tr = 0, ti = 0;
      if (tid < 256) {
        for (int b = a; b < nb; ++b) {
          const c64d t = Ts[a * 16 + b];
          tr += t.re * Wr[b][c] - t.im * Wi[b][c];
          ti += t.re * Wi[b][c] + t.im * Wr[b][c];
        }
      }
      __syncthreads();
      if (tid < 256) {
        Wr[a][c] = tr;
        Wi[a][c] = ti;
      }
    }
    __syncthreads();
    // Z -= V W over 16-row tiles (rows <= j0 get zero from the masked V)
    for (int rt = (j0 + 1) / 16 + wv; 16 * rt < n; rt += NW) {
      const int r0 = 16 * rt;
      v4d_t dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4) {
        const int a = k0 + kq, row = r0 + r16;
        c64d v = {0, 0};
        if (row < n && a < nb && row > j0 + a) v = A[(long long)row * n + j0 + a];
        const double br = Wr[a][r16], bi = Wi[a][r16];
        dr = mfma64(v.re, br, dr);
        di = mfma64(v.re, bi, di);
        dr = mfma64(-v.im, bi, dr);
        di = mfma64(v.im, br, di);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + kq + 4 * r;
        if (row < n) {
          Zr[row][r16] -= dr[r];
          Zi[row][r16] -= di[r];
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * 16; e += BNT) {
    const int r = e >> 4, c = e & 15;
    if (c < pc) Z[(long long)r * keep + c0 + c] = c64d{Zr[r][c], Zi[r][c]};
  }
}

size_t heev_ws_doubles(int n, int keep) { return bt_tfac_offset(n, keep) + (size_t)((n + 15) / 16) * 512; }
size_t heev_gws_doubles(int keep) { return (size_t)keep * keep + 64; }

hipError_t heev_phase(int phase, int n, int keep, double zero_tol, void* A, long long sA, double* ws, long long sW,
                      double* gws, long long sG, double* evals, long long sE, double* kept_sum, void* Z, long long sZ,
                      int batch, hipStream_t st, const int* active) {
  if (n > EMAX || keep > n || keep > EMAX / 2 || keep < 1) return hipErrorInvalidValue;
  (void)gws;
  (void)sG;
  switch (phase) {
    case 0:
      if (n <= 128) hipLaunchKernelGGL((k_tridiag<128, 8, 2, 512, 4, false>), dim3(batch), dim3(512), 0, st, n, (c64d*)A, sA, ws, sW, active);
      else if (n <= 256) hipLaunchKernelGGL((k_tridiag<256, 6, 2, 512, 4>), dim3(batch), dim3(512), 0, st, n, (c64d*)A, sA, ws, sW, active);
      else hipLaunchKernelGGL((k_tridiag<512, 4, 2, 512>), dim3(batch), dim3(512), 0, st, n, (c64d*)A, sA, ws, sW, active);
      break;
    case 1:
      hipLaunchKernelGGL(k_tri_eig, dim3(batch), dim3(ET), 0, st, n, keep, zero_tol, ws, sW, evals, sE, kept_sum, active);
      break;
    case 2:
      if (n <= 128) hipLaunchKernelGGL((k_tri_orth<128>), dim3(batch), dim3(ET), 0, st, n, keep, ws, sW, evals, sE, active);
      else if (n <= 256) hipLaunchKernelGGL((k_tri_orth<256>), dim3(batch), dim3(ET), 0, st, n, keep, ws, sW, evals, sE, active);
      else hipLaunchKernelGGL((k_tri_orth<512>), dim3(batch), dim3(ET), 0, st, n, keep, ws, sW, evals, sE, active);
      break;
    default: {
      if (n <= 128) {   // blocked LDS form
        hipLaunchKernelGGL((k_backtransform<256, 16>), dim3(batch), dim3(ET), 0, st, n, keep, (const c64d*)A, sA, ws, sW, (c64d*)Z, sZ, active);
        break;
      }
      // 128 < n <= 512: MFMA panel form (T factors, then 16-column panels)
      hipLaunchKernelGGL(k_bt_tfac, dim3(batch), dim3(256), 0, st, n, (const c64d*)A, sA, ws, sW, keep, active);
      const int np = (keep + 15) / 16;
      const long long blocks = (long long)np * batch;
      if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
      if (n <= 256)
        hipLaunchKernelGGL((k_bt_panel<256, 512>), dim3((unsigned)blocks), dim3(512), 0, st, n, keep, (const c64d*)A, sA, ws, sW, (c64d*)Z, sZ, np, active);
      else
        hipLaunchKernelGGL((k_bt_panel<512, 512>), dim3((unsigned)blocks), dim3(512), 0, st, n, keep, (const c64d*)A, sA, ws, sW, (c64d*)Z, sZ, np, active);
      break;
    }
  }
  return hipGetLastError();
}

// trace of the input is kept at ws[3n] by E1
}  // namespace mpsb
