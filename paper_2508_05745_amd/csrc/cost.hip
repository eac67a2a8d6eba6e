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

// ------------------------------------------------------------------ internal-bond moments
// For the cost taken across the block's internal bond (a, s) : (t, b), the purity of branch j
// needs the block Gram Gamma[(a,s),(a',s')] = sum_{t,b} theta[a,s,t,b] conj(theta[a',s',t,b])
// (2 chi_l x 2 chi_l, a contraction over 2 chi_r).  Only its 2 x 2 blocks gamma_{aa'} enter,
// through the 4 x 4 Hermitian moment matrix
//   N[(w,x),(y,z)] = sum_{a,a'} gamma_{aa'}[w][x] conj(gamma_{aa'}[y][z]),
// with Tr Gamma_j^2 = sum E_{s1 s2} E_{s3 s4} N[(s2,s3),(s1,s4)], E_j = K'_j^dag K'_j, and
// rho_q = sum_a gamma_{aa}.  One workgroup per state, of one wave (large batches) or four (the
// tile pairs dealt to the waves longest first); a wave takes its 32 x 32 tiles (I <= J) of Gamma
// one at a time, each a complex product on the FP64 MFMA 16x16x4 with operands straight from
// global memory (two complex values per lane per load, the next chunk in flight during the
// current one's products); the tile goes through LDS, each lane folds 4 of its 2 x 2 blocks into
// its moments (tile (J, I) = tile (I, J)^dag is accounted for by symmetry), and the workgroup
// reduces the moments in a fixed order (deterministic).
typedef double v4d_t __attribute__((ext_vector_type(4)));
__device__ inline v4d_t mfma64(double a, double b, v4d_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Raw elements (row, k), (row, k + 1) (K and k even: both in the row), or element (0, 0) when
// outside the block (masked to zero where used).  The load is unconditional so that it can be
// in flight while other products run.
template <typename T>
struct RawPair {
  cplx<T> x, y;
  bool ok;
};
template <typename T>
__device__ inline RawPair<T> load_pair(const cplx<T>* __restrict__ th, int row, int k, int n, int K, long long ld) {
  RawPair<T> r;
  r.ok = row < n && k < K;
  const cplx<T>* q = th + (r.ok ? row * ld + k : 0);
  r.x = q[0];
  r.y = q[1];
  return r;
}
template <typename T>
__device__ inline cd elem(const RawPair<T>& r, int e) {
  const cplx<T> v = e ? r.y : r.x;
  return r.ok ? cd{(double)v.re, (double)v.im} : cd{0, 0};
}

// acc += g g^dag for the 4-vector g (16 doubles: 4 real diagonal entries, then the 6 entries
// (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) as re, im)
__device__ inline void fold(double (&m)[16], const cd (&g)[4]) {
  for (int i = 0; i < 4; ++i) m[i] += norm2(g[i]);
  int o = 4;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      const cd z = g[i] * conj(g[j]);
      m[o] += z.re;
      m[o + 1] += z.im;
      o += 2;
    }
}

constexpr int BT = 32, BS = BT + 1;   // tile edge; LDS row stride (doubles)

// Owner wave of tile pair tp of an nt x nt tile grid among NW waves: the pairs are dealt
// longest first (off-diagonal tiles cost 4 sub-products, diagonal ones 3) to the least loaded
// wave, lowest index on ties -- the same deterministic schedule in every wave.
template <int NW>
__device__ inline int tile_owner(int tp, int nt) {
  static_assert(NW == 1 || NW == 4, "one or four waves");
  if (NW == 1) return 0;
  int l0 = 0, l1 = 0, l2 = 0, l3 = 0;               // loads of the four waves
  for (int pass = 0; pass < 2; ++pass)              // off-diagonal pairs, then diagonal ones
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J) {
        const bool diag = I == J;
        if (diag != (pass == 1)) continue;
        int best = 0, lb = l0;
        if (l1 < lb) { best = 1; lb = l1; }
        if (l2 < lb) { best = 2; lb = l2; }
        if (l3 < lb) { best = 3; lb = l3; }
        const int c = diag ? 3 : 4;
        l0 += best == 0 ? c : 0;
        l1 += best == 1 ? c : 0;
        l2 += best == 2 ? c : 0;
        l3 += best == 3 ? c : 0;
        if (I * nt - I * (I - 1) / 2 + (J - I) == tp) return best;   // row-major index of (I, J)
      }
  return 0;
}

// The moments are kept as two packed sums (4 real diagonal entries, then 6 complex off-diagonal
// ones): blocks whose mirror block (a', a) = gamma^dag is not in a computed tile go to mb, the
// others to ms; the mirrors' share is P conj(mb) P^T (P swapping entries 1 and 2), added once at
// the end.  G3: the complex product with three real products per step (T1 = Xr Yr^T, T2 = Xi Yi^T,
// T3 = (Xr + Xi)(Yr - Yi)^T; re = T1 + T2, im = T3 - T1 + T2) instead of four.
template <typename T, int NW, bool G3>
__global__ __launch_bounds__(64 * NW, 2) void k_bond_moments(int chi_l, int chi_r,
                                                                   const cplx<T>* __restrict__ theta, double* rho,
                                                                   double* nmom) {
  __shared__ double tre[NW][BT * BS], tim[NW][BT * BS];
  const int n = 2 * chi_l, K = 2 * chi_r;
  const int nt = (n + BT - 1) / BT, npairs = nt * (nt + 1) / 2;
  const cplx<T>* th = theta + (long long)blockIdx.x * n * K;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  double ms[16], mb[16], r[4];
  for (int i = 0; i < 16; ++i) ms[i] = mb[i] = 0;
  for (int i = 0; i < 4; ++i) r[i] = 0;
  double* sre = tre[wv];
  double* sim = tim[wv];
  for (int tp = 0; tp < npairs; ++tp) {
    if (tile_owner<NW>(tp, nt) != wv) continue;
    int I = 0, rem = tp;              // tp -> (I, J), I <= J, row-major over the upper triangle
    while (rem >= nt - I) { rem -= nt - I; ++I; }
    const int J = I + rem;
    const bool diag = I == J;         // sub-product (1, 0) of a diagonal tile is (0, 1)^dag: skipped
    v4d_t ar[2][2], ai[2][2], a3[2][2];
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) ar[x][y] = ai[x][y] = a3[x][y] = v4d_t{0, 0, 0, 0};
    const int rI = BT * I + li, rJ = BT * J + li;
    // two register buffers of the operands: chunk c (8 complex columns) is loaded into buffer
    // c % 2 while the products of chunk c - 1 run
    RawPair<T> ra[2][2], rb[2][2];
    auto load = [&](int buf, int k) {
      for (int h = 0; h < 2; ++h) {
        ra[buf][h] = load_pair(th, rI + 16 * h, k + 2 * lq, n, K, K);
        rb[buf][h] = load_pair(th, rJ + 16 * h, k + 2 * lq, n, K, K);
      }
    };
    auto products = [&](int buf) {
      for (int e = 0; e < 2; ++e) {
        cd a[2], b[2];
        for (int h = 0; h < 2; ++h) {
          a[h] = elem(ra[buf][h], e);
          b[h] = elem(rb[buf][h], e);
        }
        if (G3) {
          for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) {
              if (diag && x == 1 && y == 0) continue;
              ar[x][y] = mfma64(a[x].re, b[y].re, ar[x][y]);
              ai[x][y] = mfma64(a[x].im, b[y].im, ai[x][y]);
              a3[x][y] = mfma64(a[x].re + a[x].im, b[y].re - b[y].im, a3[x][y]);
            }
        } else {
          // Gamma_IJ = X_I X_J^dag: re = Xr Xr^T + Xi Xi^T, im = Xi Xr^T - Xr Xi^T
          for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) {
              if (diag && x == 1 && y == 0) continue;
              ar[x][y] = mfma64(a[x].re, b[y].re, ar[x][y]);
              ai[x][y] = mfma64(a[x].im, b[y].re, ai[x][y]);
            }
          for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) {
              if (diag && x == 1 && y == 0) continue;
              ar[x][y] = mfma64(a[x].im, b[y].im, ar[x][y]);
              ai[x][y] = mfma64(-a[x].re, b[y].im, ai[x][y]);
            }
        }
      }
    };
    load(0, 0);
    for (int k0 = 0; k0 < K; k0 += 16) {
      load(1, k0 + 8);
      products(0);
      load(0, k0 + 16);
      products(1);
    }
    // D[i][j] of a 16 x 16 product sits in lane j + 16 (i % 4), register i / 4
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y)
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * x + 4 * v + lq, j = 16 * y + li;
          if (G3) {
            sre[i * BS + j] = ar[x][y][v] + ai[x][y][v];
            sim[i * BS + j] = (a3[x][y][v] - ar[x][y][v]) + ai[x][y][v];
          } else {
            sre[i * BS + j] = ar[x][y][v];
            sim[i * BS + j] = ai[x][y][v];
          }
        }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = 0; q < 4; ++q) {
      const int blk = lane + 64 * q, al = blk >> 4, bl = blk & 15;
      // in a diagonal tile the lower-left quadrant (not computed) is the mirror of the
      // upper-right one
      const bool lower_left = diag && al >= 8 && bl < 8;
      const bool mirrored = !diag || (al < 8 && bl >= 8);
      cd g[4];
      for (int w = 0; w < 2; ++w)
        for (int x = 0; x < 2; ++x) {
          const int o = (2 * al + w) * BS + 2 * bl + x;
          g[2 * w + x] = lower_left ? cd{0, 0} : cd{sre[o], sim[o]};
        }
      if (mirrored) fold(mb, g);
      else fold(ms, g);
      if (diag && al == bl) {
        r[0] += g[0].re;
        r[1] += g[3].re;
        r[2] += g[1].re;
        r[3] += g[1].im;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // fixed-order reduction: within each wave by shuffles, then the waves in order
  __shared__ double red[NW][36];
  for (int x = 0; x < 36; ++x) {
    double s = x < 16 ? ms[x] : (x < 32 ? mb[x - 16] : r[x - 32]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wv][x] = s;
  }
  __syncthreads();
  if (threadIdx.x < 36) {
    const int x = threadIdx.x;
    double s = red[0][x];
    for (int w = 1; w < NW; ++w) s += red[w][x];
    red[0][x] = s;
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    const double* Ms = red[0];
    const double* Mb = red[0] + 16;
    const double* R = red[0] + 32;
    // normalised by ||theta||^2 (rho) and ||theta||^4 (N)
    const double tr = R[0] + R[1];
    const double s1 = 1.0 / tr, s2 = s1 * s1;
    if (threadIdx.x < 8) {
      const double v[8] = {R[0], 0.0, R[2], R[3], R[2], -R[3], R[1], 0.0};
      rho[blockIdx.x * 8 + threadIdx.x] = s1 * v[threadIdx.x];
    }
    // entry (p, q) of a packed Hermitian 4 x 4
    auto entry = [](const double* M, int p, int q) {
      if (p == q) return cd{M[p], 0.0};
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      const int o = 4 + 2 * (lo * (7 - lo) / 2 + (hi - lo - 1));
      return cd{M[o], p < q ? M[o + 1] : -M[o + 1]};
    };
    // N[(p),(q)] with p, q in 0..3 (p = 2 w + x, q = 2 y + z), full Hermitian 4 x 4, c128
    for (int e = threadIdx.x; e < 16; e += 32) {
      const int p = e >> 2, q = e & 3;
      const int pp = p == 1 ? 2 : (p == 2 ? 1 : p), qq = q == 1 ? 2 : (q == 2 ? 1 : q);
      const cd v = entry(Ms, p, q) + entry(Mb, p, q) + conj(entry(Mb, pp, qq));
      nmom[blockIdx.x * 32 + 2 * e] = s2 * v.re;
      nmom[blockIdx.x * 32 + 2 * e + 1] = s2 * v.im;
    }
  }
}

hipError_t bond_moments(int batch, const void* theta, int chi_l, int chi_r, int prec, double* rho, double* nmom,
                        hipStream_t st) {
  // one wave per state once the batch fills the chip (two waves per SIMD), four otherwise; the
  // three-product complex step (measured 5-20% faster than four products)
  if (batch >= 2048) {
    if (prec == 0)
      hipLaunchKernelGGL((k_bond_moments<float, 1, true>), dim3(batch), dim3(64), 0, st, chi_l, chi_r,
                         (const c32*)theta, rho, nmom);
    else
      hipLaunchKernelGGL((k_bond_moments<double, 1, true>), dim3(batch), dim3(64), 0, st, chi_l, chi_r,
                         (const c64d*)theta, rho, nmom);
  } else {
    if (prec == 0)
      hipLaunchKernelGGL((k_bond_moments<float, 4, true>), dim3(batch), dim3(256), 0, st, chi_l, chi_r,
                         (const c32*)theta, rho, nmom);
    else
      hipLaunchKernelGGL((k_bond_moments<double, 4, true>), dim3(batch), dim3(256), 0, st, chi_l, chi_r,
                         (const c64d*)theta, rho, nmom);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ 4 x 4 matrices on 16 lanes
// A state's 4 x 4 complex matrices are spread over a group of 16 lanes: lane g of the group
// holds entry (g >> 2, g & 3).  Products exchange rows and columns by lane shuffles within the
// group (no per-lane 4 x 4 or 8 x 8 arrays, which would not fit in registers).  Every lane of a
// group follows the same control flow (group-uniform loop counts).
__device__ inline cd gsh(cd x, int src) { return cd{__shfl(x.re, src, 16), __shfl(x.im, src, 16)}; }

__device__ inline cd gmm(cd a, cd b, int g) {   // (A B)[i][j]
  const int i = g >> 2, j = g & 3;
  cd s = {0, 0};
  for (int k = 0; k < 4; ++k) cfma(s, gsh(a, 4 * i + k), gsh(b, 4 * k + j));
  return s;
}

// max over the columns of the column sums of v (v >= 0 per entry), in every lane of the group
__device__ inline double gcolmax(double v) {
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 8, 16);
  v = fmax(v, __shfl_xor(v, 1, 16));
  return fmax(v, __shfl_xor(v, 2, 16));
}

// exp(A) by scaling and squaring with a degree-18 Taylor polynomial (||A / 2^s||_1 <= 1/4)
__device__ cd gexpm(cd a, int g) {
  double nrm = gcolmax(sqrt(norm2(a)));
  int s = 0;
  while (nrm > 0.25 && s < 60) { nrm *= 0.5; ++s; }
  const double sc = ldexp(1.0, -s);
  const cd x = sc * a;
  const cd one = (g >> 2) == (g & 3) ? cd{1, 0} : cd{0, 0};
  cd term = one, out = one;
  for (int k = 1; k <= 18; ++k) {
    term = (1.0 / k) * gmm(term, x, g);
    out = out + term;
  }
  for (int r = 0; r < s; ++r) out = gmm(out, out, g);
  return out;
}

// Frechet derivative L(A, E) of the exponential: the upper-right block of
// exp([[A, E], [0, A]]), by the same scaling (the 8 x 8 block's 1-norm) and Taylor degree,
// kept in its 4 x 4 blocks: term_k = [[T_k, F_k], [0, T_k]] with T_k = T_{k-1} A / k,
// F_k = (F_{k-1} A + T_{k-1} E) / k, and a squaring maps [[P, Q], [0, P]] to
// [[P^2, P Q + Q P], [0, P^2]].
__device__ cd gfrechet(cd a, cd e, int g) {
  double nrm = gcolmax(sqrt(norm2(a)) + sqrt(norm2(e)));
  int s = 0;
  while (nrm > 0.25 && s < 60) { nrm *= 0.5; ++s; }
  const double sc = ldexp(1.0, -s);
  const cd x = sc * a, y = sc * e;
  const cd one = (g >> 2) == (g & 3) ? cd{1, 0} : cd{0, 0};
  cd T = one, F = {0, 0}, P = one, Q = {0, 0};
  for (int k = 1; k <= 18; ++k) {
    const double f = 1.0 / k;
    const cd Fn = f * (gmm(F, x, g) + gmm(T, y, g));
    T = f * gmm(T, x, g);
    F = Fn;
    P = P + T;
    Q = Q + F;
  }
  for (int r = 0; r < s; ++r) {
    Q = gmm(P, Q, g) + gmm(Q, P, g);
    P = gmm(P, P, g);
  }
  return Q;
}

// Q(A, B) = sum A[s1][s2] B[s3][s4] N[(s2,s3)][(s1,s4)]: Tr Gamma_j^2 = Q(E_j, E_j), symmetric in
// its two arguments (cyclicity of the trace)
__device__ inline cd bond_q(const cd (&a)[2][2], const cd (&b)[2][2], const cd (&N)[4][4]) {
  cd s = {0, 0};
  for (int s1 = 0; s1 < 2; ++s1)
    for (int s2 = 0; s2 < 2; ++s2)
      for (int s3 = 0; s3 < 2; ++s3)
        for (int s4 = 0; s4 < 2; ++s4) s = s + (a[s1][s2] * b[s3][s4]) * N[2 * s2 + s3][2 * s1 + s4];
  return s;
}

__device__ inline int pair_index(int a, int c) { return a * (7 - a) / 2 + (c - a - 1); }   // a < c

constexpr double P_TINY = 1e-300;
constexpr double LN2 = 0.69314718055994530942;

// Per lane (j, i) = (g >> 2, g & 3) of a state's group: X = iH entry, U_ji, the branch j it
// serves (K'_j, sigma~_j, E_j, p_j, P_j).
struct Branch {
  cd h, U;
  cd Ki[2][2];   // K_i of the lane's column i
  cd Kp[2][2], rho[2][2], sig[2][2], E[2][2], N[4][4];
  double p, P;
};

__device__ __forceinline__ void branch_setup(int g, const double* rho_in, const double* nm, const double* kraus, const double* params,
                             const double* uref, Branch& br) {
  const int a = g >> 2, c = g & 3;
  for (int x = 0; x < 4; ++x) br.rho[x >> 1][x & 1] = cd{rho_in[2 * x], rho_in[2 * x + 1]};
  // normalise rho (the reduction of an unnormalised theta is allowed)
  const double tr = br.rho[0][0].re + br.rho[1][1].re;
  for (int x = 0; x < 4; ++x) br.rho[x >> 1][x & 1] = (1.0 / tr) * br.rho[x >> 1][x & 1];
  auto kraus_at = [&](int i, int x, int y) { return cd{kraus[2 * (4 * i + 2 * x + y)], kraus[2 * (4 * i + 2 * x + y) + 1]}; };
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) br.Ki[x][y] = kraus_at(c, x, y);
  // H = sum_k params_k L_k: E_kk (k < 4), E_pq + E_qp (4 + pair), i (E_qp - E_pq) (10 + pair)
  if (a == c) br.h = cd{params[a], 0.0};
  else {
    const int lo = a < c ? a : c, hi = a < c ? c : a, pi = pair_index(lo, hi);
    br.h = cd{params[4 + pi], a < c ? -params[10 + pi] : params[10 + pi]};
  }
  const cd x = cd{-br.h.im, br.h.re};   // iH
  const cd ex = gexpm(x, g);
  // U = exp(iH) U_ref
  cd u = {0, 0};
  for (int k = 0; k < 4; ++k) cfma(u, gsh(ex, 4 * a + k), cd{uref[2 * (4 * k + c)], uref[2 * (4 * k + c) + 1]});
  br.U = u;
  // branch j = a: K'_j = sum_m U_jm K_m
  cd row[4];
  for (int m = 0; m < 4; ++m) row[m] = gsh(u, 4 * a + m);
  for (int x2 = 0; x2 < 2; ++x2)
    for (int y = 0; y < 2; ++y) {
      cd s = {0, 0};
      for (int m = 0; m < 4; ++m) cfma(s, row[m], kraus_at(m, x2, y));
      br.Kp[x2][y] = s;
    }
  cd t[2][2];
  for (int x2 = 0; x2 < 2; ++x2)
    for (int y = 0; y < 2; ++y) {
      cd s = {0, 0};
      for (int m = 0; m < 2; ++m) cfma(s, br.Kp[x2][m], br.rho[m][y]);
      t[x2][y] = s;
    }
  for (int x2 = 0; x2 < 2; ++x2)
    for (int y = 0; y < 2; ++y) {
      cd s = {0, 0};
      for (int m = 0; m < 2; ++m) cfma_conj(s, t[x2][m], br.Kp[y][m]);
      br.sig[x2][y] = s;
    }
  br.p = br.sig[0][0].re + br.sig[1][1].re;
  if (nm) {
    for (int e = 0; e < 16; ++e) br.N[e >> 2][e & 3] = cd{nm[2 * e], nm[2 * e + 1]};
    for (int x2 = 0; x2 < 2; ++x2)
      for (int y = 0; y < 2; ++y) {
        cd s = {0, 0};
        for (int m = 0; m < 2; ++m) cfma(s, conj(br.Kp[m][x2]), br.Kp[m][y]);
        br.E[x2][y] = s;
      }
    br.P = bond_q(br.E, br.E, br.N).re;
  } else {
    double P = 0;
    for (int x2 = 0; x2 < 2; ++x2)
      for (int y = 0; y < 2; ++y) P += (br.sig[x2][y] * br.sig[y][x2]).re;
    br.P = P;
  }
}

// nm == nullptr: the noisy qubit against the rest of the block (P_j = Tr sigma~_j^2); else the
// block's internal bond, nm the moment matrix N [4][4] c128 per state (P_j = Q(E_j, E_j)).
__global__ __launch_bounds__(256) void k_cost_eval(int batch, const double* rho, const double* nm, const double* kraus,
                                                   const double* params, const double* uref, int kind, double* f) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x, g = threadIdx.x & 15;
  const int b = gid >> 4, bb = b < batch ? b : batch - 1;   // every lane of a group works
  Branch br;
  branch_setup(g, rho + bb * 8, nm ? nm + bb * 32 : nullptr, kraus, params + bb * 16, uref + bb * 32, br);
  double term = 0;
  if (br.p > P_TINY) term = kind == 0 ? br.p - br.P / br.p : -br.p * log(br.P / (br.p * br.p)) / LN2;
  // the 4 lanes of row j hold branch j's term: a quarter from each, summed over the group
  double v = 0.25 * term;
  v += __shfl_xor(v, 1, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 8, 16);
  if (g == 0 && b < batch) f[b] = v;
}

__global__ __launch_bounds__(256) void k_cost_grad(int batch, const double* rho, const double* nm, const double* kraus,
                                                   const double* params, const double* uref, int kind,
                                                   const double* grad_f, double* grad) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x, g = threadIdx.x & 15;
  const int b = gid >> 4, bb = b < batch ? b : batch - 1;
  const int a = g >> 2, c = g & 3;
  Branch br;
  branch_setup(g, rho + bb * 8, nm ? nm + bb * 32 : nullptr, kraus, params + bb * 16, uref + bb * 32, br);
  // G[j][i] = g_p Tr(K_i rho K'_j^dag) + g_P d P_j / d U_ji, lane (j, i) = (a, c)
  const double p = br.p, P = br.P;
  double gp = 0, gP = 0;
  if (p > P_TINY) {
    if (kind == 0) { gp = 1.0 + P / (p * p); gP = -1.0 / p; }
    else { gp = -log(P / (p * p)) / LN2 + 2.0 / LN2; gP = -p / (P * LN2); }
  }
  cd t[2][2], B[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      cd s = {0, 0};
      for (int m = 0; m < 2; ++m) cfma(s, br.Ki[x][m], br.rho[m][y]);
      t[x][y] = s;
    }
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      cd s = {0, 0};
      for (int m = 0; m < 2; ++m) cfma_conj(s, t[x][m], br.Kp[y][m]);
      B[x][y] = s;
    }
  const cd trB = B[0][0] + B[1][1];
  cd trSB = {0, 0};   // d P_j / d U_ji / 2
  if (nm) {
    cd D[2][2];       // K'_j^dag K_i
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) {
        cd e = {0, 0};
        for (int m = 0; m < 2; ++m) cfma(e, conj(br.Kp[m][x]), br.Ki[m][y]);
        D[x][y] = e;
      }
    trSB = bond_q(D, br.E, br.N);
  } else {
    for (int x = 0; x < 2; ++x)
      for (int m = 0; m < 2; ++m) trSB = trSB + br.sig[x][m] * B[m][x];
  }
  const cd G = gp * trB + (2.0 * gP) * trSB;
  // M = U_ref G^T, E = M^dag; L(X^dag, E) with X^dag = (iH)^dag = -iH
  const double* ur = uref + bb * 32;
  cd mt = {0, 0};
  for (int k = 0; k < 4; ++k) cfma(mt, cd{ur[2 * (4 * a + k)], ur[2 * (4 * a + k) + 1]}, gsh(G, 4 * c + k));
  const cd e = conj(gsh(mt, 4 * c + a));
  const cd L = gfrechet(cd{br.h.im, -br.h.re}, e, g);
  // d f / d params_k = 2 Re sum conj(L) (i L_k): i E_kk -> Im L_kk; i (E_pq + E_qp) -> Im L_pq +
  // Im L_qp; i * i (E_qp - E_pq) -> Re L_pq - Re L_qp (p < q)
  const cd Lt = gsh(L, 4 * c + a);
  const double gf = grad_f ? grad_f[bb] : 1.0;
  if (b < batch) {
    if (a == c) grad[b * 16 + a] = gf * 2.0 * L.im;
    else if (a < c) {
      const int pi = pair_index(a, c);
      grad[b * 16 + 4 + pi] = gf * 2.0 * (L.im + Lt.im);
      grad[b * 16 + 10 + pi] = gf * 2.0 * (L.re - Lt.re);
    }
  }
}

hipError_t cost_eval(int batch, const double* rho, const double* nm, const double* kraus, const double* params,
                     const double* u_ref, int kind, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_cost_eval, dim3((batch + 15) / 16), dim3(256), 0, st, batch, rho, nm, kraus, params, u_ref, kind,
                     f);
  return hipGetLastError();
}

hipError_t cost_grad(int batch, const double* rho, const double* nm, const double* kraus, const double* params,
                     const double* u_ref, int kind, const double* grad_f, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_cost_grad, dim3((batch + 15) / 16), dim3(256), 0, st, batch, rho, nm, kraus, params, u_ref, kind,
                     grad_f, grad);
  return hipGetLastError();
}

}  // namespace mpsb
