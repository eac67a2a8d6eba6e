// Host runtime of the mpsb library: the C ABI declared in include/mpsb.h.
//
// A batch holds n_traj trajectories of an n-qubit chain as matrix product states with fixed
// bond capacities cap[k] = min(chi, 2^(k+1), 2^(n-k-1)); site k is a c64 / c128 tensor
// [a][s][b] (a < cap[k-1], b < cap[k]) so that every contraction of the sweep is a plain
// strided batched GEMM.  Trajectories share their shape, so each step of the sweep is one
// batched launch over all trajectories.  Directions of the state that carry no weight (zero
// eigenvalues of a Gram matrix) are represented by zero vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpsb.h"
#include "common.h"
#include "kernels.h"

using namespace mpsb;

static thread_local std::string g_err;
static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(MPSB_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr double ZERO_TOL_FP64 = 1e-26;   // relative drop threshold of Gram eigenvalues
constexpr double ZERO_TOL_FP32 = 1e-13;

struct Layout {
  int n_traj, n, chi, prec;
  size_t esz;                       // bytes per complex element of the state
  std::vector<int> cap;             // [n-1]
  std::vector<long long> off;       // [n] element offsets of the sites inside a trajectory
  long long s_traj;                 // elements per trajectory
  // work buffer (byte offsets)
  size_t o_status, o_siteoff, o_x, o_partial, o_kops, o_gram, o_ews, o_gws, o_evals, o_z, o_kept, o_alpha,
      o_invs, o_sqrt, o_wm, o_rm, o_rho1, o_tmp, o_obs, o_norm, o_pbuf, o_exp;
  long long s_x, s_partial, s_gram, s_ews, s_gws, s_evals, s_z, s_wm, s_tmp;
  int exp_chunk;
  long long s_env;                  // c128 elements per environment slot
  size_t state_bytes, work_bytes;
  int max_tiles;
};

int dl(const Layout& L, int k) { return k == 0 ? 1 : L.cap[k - 1]; }
int dr(const Layout& L, int k) { return k == L.n - 1 ? 1 : L.cap[k]; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int make_layout(int n_traj, int n, int chi, int prec, Layout& L) {
  if (n_traj <= 0 || n_traj > (1 << 30)) return fail(MPSB_EINVAL, "n_traj must be in 1..2^30");
  if (n < 2 || n > MPSB_MAX_QUBITS) return fail(MPSB_EINVAL, "n_qubits must be in 2..MPSB_MAX_QUBITS");
  if (chi < 1 || chi > MPSB_MAX_CHI) return fail(MPSB_EINVAL, "chi must be in 1..MPSB_MAX_CHI");
  if (prec != MPSB_FP32_BULK && prec != MPSB_FP64) return fail(MPSB_EINVAL, "precision must be MPSB_FP32_BULK or MPSB_FP64");
  L.n_traj = n_traj;
  L.n = n;
  L.chi = chi;
  L.prec = prec;
  L.esz = prec == MPSB_FP64 ? 16 : 8;
  L.cap.assign(n - 1, 1);
  for (int k = 0; k < n - 1; ++k) {
    long long a = 1, b = 1;
    for (int i = 0; i <= k && a < chi; ++i) a *= 2;
    for (int i = 0; i < n - k - 1 && b < chi; ++i) b *= 2;
    L.cap[k] = (int)std::min<long long>(chi, std::min(a, b));
  }
  L.off.assign(n, 0);
  long long acc = 0;
  int cmax = 1;
  for (int k = 0; k < n; ++k) {
    L.off[k] = acc;
    acc += 2LL * dl(L, k) * dr(L, k);
    acc = (acc + 31) / 32 * 32;
  }
  for (int k = 0; k < n - 1; ++k) cmax = std::max(cmax, L.cap[k]);
  L.s_traj = acc;
  L.state_bytes = (size_t)acc * L.esz * n_traj;
  const long long c = cmax;
  const long long T = n_traj;
  L.max_tiles = ((int)(c + 31) / 32) * ((int)(c + 31) / 32);
  L.s_x = 4 * c * c;                                  // elements (prec)
  L.s_partial = (long long)L.max_tiles * 32;          // doubles
  L.s_gram = 4 * c * c;                               // c128 elements
  L.s_ews = (long long)heev_ws_doubles(2 * (int)c, (int)c);
  L.s_gws = (long long)heev_gws_doubles((int)c);
  L.s_evals = 2 * c;
  L.s_z = 2 * c * c;                                  // c128
  L.s_wm = c * c;                                     // prec elements
  L.s_tmp = 4 * c * c;                                // prec elements (hop results)
  // expect chunk: (n + 1) environments + 8 scratch matrices of 2c^2 c128 per trajectory
  L.s_env = 2 * c * c;
  long long per_exp = (long long)(n + 1 + 8) * L.s_env * 16;
  long long budget = 1LL << 31;
  L.exp_chunk = (int)std::max<long long>(1, std::min<long long>(T, budget / std::max<long long>(per_exp, 1)));
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.o_status = take(256);
  L.o_siteoff = take(sizeof(long long) * n);
  L.o_kops = take(sizeof(double) * 16 * T);
  L.o_kept = take(sizeof(double) * T);
  L.o_alpha = take(sizeof(double) * T);
  L.o_rho1 = take(sizeof(double) * 8 * T);
  L.o_norm = take(sizeof(double) * T);
  L.o_pbuf = take(sizeof(double) * 4 * T);
  L.o_obs = take(sizeof(double) * (2 * n - 1) * T);
  // gate-step region and expect region overlap
  size_t base = o;
  L.o_x = take(L.esz * L.s_x * T);
  L.o_partial = take(sizeof(double) * L.s_partial * T);
  L.o_gram = take(16 * L.s_gram * T);
  L.o_ews = take(sizeof(double) * L.s_ews * T);
  L.o_gws = take(sizeof(double) * L.s_gws * T);
  L.o_evals = take(sizeof(double) * L.s_evals * T);
  L.o_z = take(16 * L.s_z * T);
  L.o_invs = take(sizeof(double) * c * T);
  L.o_sqrt = take(sizeof(double) * c * T);
  L.o_wm = take(L.esz * L.s_wm * T);
  L.o_rm = take(L.esz * L.s_wm * T);
  L.o_tmp = take(L.esz * L.s_tmp * T);
  size_t gate_end = o;
  o = base;
  L.o_exp = take((size_t)per_exp * L.exp_chunk);
  L.work_bytes = std::max(gate_end, o);
  return MPSB_OK;
}

}  // namespace

// kernel classes timed by the optional profiler
enum ProfClass {
  PC_THETA = 0, PC_EVENTS, PC_KRAUS, PC_GRAM, PC_TRIDIAG, PC_TRIEIG, PC_HOPEIG, PC_BACK, PC_RECOMPOSE, PC_HOPGEMM,
  PC_SMALL, PC_EXPECT, PC_TRIDIAG_S, PC_TRIDIAG_L, PC_BACK_L, PC_COUNT
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> cls;                 // class of each recorded pair
  double ms[PC_COUNT] = {0};
  long long count[PC_COUNT] = {0};
};

struct mpsb_batch {
  Prof prof;
  Layout L;
  uint64_t seed;
  char* state;
  char* work;
  hipStream_t st;
  int centre;
  int next_layer;
  bool has_circuit;
  // circuit (host copy)
  int depth;
  std::vector<double> gates;
  int n_channels;
  std::vector<double> kraus;
  std::vector<int> n_kraus;
  std::vector<int> events;
  int mode;
  std::vector<double> fixed_u;
};

namespace {

template <typename T> T* W(mpsb_batch* h, size_t off) { return (T*)(h->work + off); }

void prof_collect(mpsb_batch* h);

// RAII section: records a start / end event pair on the batch stream when profiling.
struct ProfSec {
  mpsb_batch* h;
  bool active;
  ProfSec(mpsb_batch* h_, int c) : h(h_), active(h_->prof.on) {
    if (!active) return;
    Prof& P = h->prof;
    if (P.used >= 16384) prof_collect(h);
    if (P.used + 2 > P.pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { active = false; return; }
        P.pool.push_back(e);
      }
    }
    P.cls.push_back(c);
    (void)hipEventRecord(P.pool[P.used], h->st);
    P.used++;
  }
  ~ProfSec() {
    if (!active) return;
    Prof& P = h->prof;
    (void)hipEventRecord(P.pool[P.used], h->st);
    P.used++;
  }
};

void prof_collect(mpsb_batch* h) {
  Prof& P = h->prof;
  if (P.used == 0) return;
  (void)hipStreamSynchronize(h->st);
  for (size_t i = 0; i + 1 < P.used; i += 2) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, P.pool[i], P.pool[i + 1]) == hipSuccess) {
      P.ms[P.cls[i / 2]] += ms;
      P.count[P.cls[i / 2]] += 1;
    }
  }
  P.used = 0;
  P.cls.clear();
}

hipError_t heev_all(mpsb_batch* h, int n, int keep, double zt, void* A, long long sA, double* ws, long long sW,
                    double* gws, long long sG, double* ev, long long sE, double* kept, void* Z, long long sZ, int batch,
                    bool hop = false) {
  // one class per kernel instance: the tridiagonalisation has instances for n <= 128,
  // n <= 256 and n <= 512, the back-transformation for n <= 256 and n <= 512
  const int tri = n <= 128 ? PC_TRIDIAG_S : n <= 256 ? PC_TRIDIAG : PC_TRIDIAG_L;
  const int cls[4] = {tri, PC_TRIEIG, PC_HOPEIG, n <= 256 ? PC_BACK : PC_BACK_L};
  for (int ph = 0; ph < 4; ++ph) {
    if (ph == 2) continue;
    ProfSec s(h, hop ? PC_HOPEIG : cls[ph]);
    hipError_t e = heev_phase(ph, n, keep, zt, A, sA, ws, sW, gws, sG, ev, sE, kept, Z, sZ, batch, h->st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
char* site_ptr(mpsb_batch* h, int k) { return h->state + (size_t)h->L.off[k] * h->L.esz; }
int* status_ptr(mpsb_batch* h) { return W<int>(h, h->L.o_status); }

int check_status(mpsb_batch* h) {
  int s = 0;
  HIPCHK(hipMemcpyAsync(&s, status_ptr(h), sizeof(int), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (s != 0) {
    int z = 0;
    HIPCHK(hipMemcpyAsync(status_ptr(h), &z, sizeof(int), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (s & 2) return fail(MPSB_ENUM, "a forced branch had zero probability");
    return fail(MPSB_ENUM, "non-finite or zero norm encountered in a trajectory");
  }
  return MPSB_OK;
}

// batched strided copy of a (rows x row_bytes) block from the temp buffer into a site
hipError_t copy_blocks(void* dst, size_t dpitch, const void* src, size_t spitch, size_t bytes, int n_traj, hipStream_t st) {
  return hipMemcpy2DAsync(dst, dpitch, src, spitch, bytes, n_traj, hipMemcpyDeviceToDevice, st);
}

double zero_tol(const Layout& L) { return L.prec == MPSB_FP64 ? ZERO_TOL_FP64 : ZERO_TOL_FP32; }

// Move the orthogonality centre from site j to j+1: C_j = Q R via the Gram matrix C^dag C.
int hop_right(mpsb_batch* h, int j) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  const int cl = dl(L, j), cr = dr(L, j), cr2 = dr(L, j + 1);
  char* Cj = site_ptr(h, j);
  char* Bn = site_ptr(h, j + 1);
  double* gram = W<double>(h, L.o_gram);
  {
    ProfSec s(h, PC_HOPGEMM);
    HIPCHK(gemm(p, 1, true, false, cr, cr, 2 * cl, Cj, cr, L.s_traj, Cj, cr, L.s_traj, gram, cr, L.s_gram, nullptr, T, h->st));
  }
  if (cr <= 128) {
    ProfSec sh(h, PC_HOPEIG);
    HIPCHK(hop_chol(p, cr, 1, 2 * cl, gram, L.s_gram, Cj, L.s_traj, W<char>(h, L.o_rm), L.s_wm, zero_tol(L), T, h->st));
  } else {
  HIPCHK(heev_all(h, cr, cr, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
              W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), W<double>(h, L.o_z), L.s_z, T, true));
  ProfSec shop(h, PC_HOPGEMM);
  double* invs = W<double>(h, L.o_invs);
  double* sq = W<double>(h, L.o_sqrt);
  HIPCHK(hop_scales(W<double>(h, L.o_evals), L.s_evals, cr, invs, sq, T, h->st));
  // Wm = W Lambda^{-1/2}, Rm = Lambda^{1/2} W^dag
  HIPCHK(scale_cast(p, cr, cr, W<double>(h, L.o_z), cr, L.s_z, invs, cr, false, W<char>(h, L.o_wm), cr, L.s_wm, T, h->st));
  HIPCHK(scale_cast(p, cr, cr, W<double>(h, L.o_z), cr, L.s_z, sq, cr, true, W<char>(h, L.o_rm), cr, L.s_wm, T, h->st));
  }
  char* tmp = W<char>(h, L.o_tmp);
  if (cr > 128) {
    // A_j = C Wm  -> tmp -> site j
    HIPCHK(gemm(p, p, false, false, 2 * cl, cr, cr, Cj, cr, L.s_traj, W<char>(h, L.o_wm), cr, L.s_wm, tmp, cr, L.s_tmp, nullptr, T, h->st));
    HIPCHK(copy_blocks(Cj, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)2 * cl * cr * L.esz, T, h->st));
  }
  // C_{j+1} = Rm B_{j+1}
  HIPCHK(gemm(p, p, false, false, cr, 2 * cr2, cr, W<char>(h, L.o_rm), cr, L.s_wm, Bn, 2 * cr2, L.s_traj, tmp, 2 * cr2, L.s_tmp, nullptr, T, h->st));
  HIPCHK(copy_blocks(Bn, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)cr * 2 * cr2 * L.esz, T, h->st));
  h->centre = j + 1;
  return MPSB_OK;
}

// Move the centre from site j to j-1: C_j = L Q via the Gram matrix C C^dag.
int hop_left(mpsb_batch* h, int j) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  const int cl = dl(L, j), cr = dr(L, j), cl2 = dl(L, j - 1);
  char* Cj = site_ptr(h, j);
  char* Ap = site_ptr(h, j - 1);
  double* gram = W<double>(h, L.o_gram);
  {
    ProfSec s(h, PC_HOPGEMM);
    HIPCHK(gemm(p, 1, false, true, cl, cl, 2 * cr, Cj, 2 * cr, L.s_traj, Cj, 2 * cr, L.s_traj, gram, cl, L.s_gram, nullptr, T, h->st));
  }
  char* tmp = W<char>(h, L.o_tmp);
  if (cl <= 128) {
    ProfSec sh(h, PC_HOPEIG);
    HIPCHK(hop_chol(p, cl, 0, 2 * cr, gram, L.s_gram, Cj, L.s_traj, W<char>(h, L.o_rm), L.s_wm, zero_tol(L), T, h->st));
    ProfSec shg(h, PC_HOPGEMM);
    // C_{j-1} = A_{j-1} R^dag
    HIPCHK(gemm(p, p, false, true, 2 * cl2, cl, cl, Ap, cl, L.s_traj, W<char>(h, L.o_rm), cl, L.s_wm, tmp, cl, L.s_tmp, nullptr, T, h->st));
    HIPCHK(copy_blocks(Ap, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)2 * cl2 * cl * L.esz, T, h->st));
    h->centre = j - 1;
    return MPSB_OK;
  }
  HIPCHK(heev_all(h, cl, cl, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
              W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), W<double>(h, L.o_z), L.s_z, T, true));
  ProfSec shop(h, PC_HOPGEMM);
  double* invs = W<double>(h, L.o_invs);
  double* sq = W<double>(h, L.o_sqrt);
  HIPCHK(hop_scales(W<double>(h, L.o_evals), L.s_evals, cl, invs, sq, T, h->st));
  // Wm = Lambda^{-1/2} W^dag, Rm = W Lambda^{1/2}
  HIPCHK(scale_cast(p, cl, cl, W<double>(h, L.o_z), cl, L.s_z, invs, cl, true, W<char>(h, L.o_wm), cl, L.s_wm, T, h->st));
  HIPCHK(scale_cast(p, cl, cl, W<double>(h, L.o_z), cl, L.s_z, sq, cl, false, W<char>(h, L.o_rm), cl, L.s_wm, T, h->st));
  // B_j = Wm C
  HIPCHK(gemm(p, p, false, false, cl, 2 * cr, cl, W<char>(h, L.o_wm), cl, L.s_wm, Cj, 2 * cr, L.s_traj, tmp, 2 * cr, L.s_tmp, nullptr, T, h->st));
  HIPCHK(copy_blocks(Cj, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)cl * 2 * cr * L.esz, T, h->st));
  // C_{j-1} = A_{j-1} Rm
  HIPCHK(gemm(p, p, false, false, 2 * cl2, cl, cl, Ap, cl, L.s_traj, W<char>(h, L.o_rm), cl, L.s_wm, tmp, cl, L.s_tmp, nullptr, T, h->st));
  HIPCHK(copy_blocks(Ap, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)2 * cl2 * cl * L.esz, T, h->st));
  h->centre = j - 1;
  return MPSB_OK;
}

int move_centre(mpsb_batch* h, int lo, int hi) {
  // bring the centre into [lo, hi]
  while (h->centre < lo) {
    int r = hop_right(h, h->centre);
    if (r) return r;
  }
  while (h->centre > hi) {
    int r = hop_left(h, h->centre);
    if (r) return r;
  }
  return MPSB_OK;
}

void fill_channel_slot(mpsb_batch* h, EventArgs& ea, int slot, int ch) {
  ea.n_kraus[slot] = h->n_kraus[ch];
  for (int x = 0; x < 32; ++x) {
    ea.kraus[slot][x] = h->kraus[(size_t)ch * 32 + x];
    ea.fixed_u[slot][x] = h->fixed_u.empty() ? 0.0 : h->fixed_u[(size_t)ch * 32 + x];
  }
}

EventArgs base_event_args(mpsb_batch* h, int layer, int32_t* branch, double* w_record, int mode) {
  EventArgs ea;
  memset(&ea, 0, sizeof(ea));
  ea.n_traj = h->L.n_traj;
  ea.n_qubits = h->L.n;
  ea.layer = layer;
  ea.mode = mode;
  ea.seed = h->seed;
  ea.branch_out = branch;
  ea.w_out = w_record;
  ea.rec_stride = h->L.n;
  ea.rec_qbase = 0;
  return ea;
}

// Two-site step on (q, q+1): gate, noise events, truncation to keep columns, split.
// left_to_right: the new centre goes to q+1 (A_q left-orthonormal), else to q.
int two_site_step(mpsb_batch* h, int layer, int q, const Mat4& gate, int ch_s, int ch_t, bool left_to_right, int keep,
                  double* discarded, int disc_stride, int accumulate, int32_t* branch, double* w_record) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  int r = move_centre(h, q, q + 1);
  if (r) return r;
  const int cl = dl(L, q), cm = dr(L, q), cr = dr(L, q + 1);
  const int D = cm;
  char* Sq = site_ptr(h, q);
  char* Sn = site_ptr(h, q + 1);
  char* X = W<char>(h, L.o_x);
  double* partial = W<double>(h, L.o_partial);
  double* kops = W<double>(h, L.o_kops);
  {
    ProfSec s(h, PC_THETA);
    HIPCHK(theta(p, cl, cm, cr, Sq, Sn, L.s_traj, X, L.s_x, gate, partial, T, h->st));
  }
  const int nt = theta_tiles(p, cl, cr);
  if (ch_s >= 0 || ch_t >= 0) {
    EventArgs ea = base_event_args(h, layer, branch, w_record, h->mode);
    if (ch_s >= 0) fill_channel_slot(h, ea, 0, ch_s);
    if (ch_t >= 0) fill_channel_slot(h, ea, 1, ch_t);
    {
      ProfSec s(h, PC_EVENTS);
      HIPCHK(launch_gate_events(ea, partial, nt, q, ch_s >= 0, ch_t >= 0, kops, status_ptr(h), h->st));
    }
    ProfSec s(h, PC_KRAUS);
    HIPCHK(kraus_pair(p, cl, cr, X, L.s_x, kops, T, h->st));
  }
  double* gram = W<double>(h, L.o_gram);
  double* Z = W<double>(h, L.o_z);
  double* alpha = W<double>(h, L.o_alpha);
  const int n = left_to_right ? 2 * cl : 2 * cr;
  {
    ProfSec s(h, PC_GRAM);
    if (left_to_right)
      HIPCHK(gemm(p, 1, false, true, 2 * cl, 2 * cl, 2 * cr, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cl, L.s_gram, nullptr, T, h->st));
    else
      HIPCHK(gemm(p, 1, true, false, 2 * cr, 2 * cr, 2 * cl, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cr, L.s_gram, nullptr, T, h->st));
  }
  const int kk = std::min(keep, D);
  HIPCHK(heev_all(h, n, kk, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
              W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), Z, L.s_z, T));
  HIPCHK(trunc_factors(W<double>(h, L.o_kept), W<double>(h, L.o_ews), L.s_ews, n, alpha, discarded, disc_stride, accumulate, T, h->st));
  ProfSec srec(h, PC_RECOMPOSE);
  if (left_to_right) {
    // A_q = U (2cl x D), columns >= kk zero; C_{q+1} = alpha A_q^dag X
    HIPCHK(scale_cast(p, 2 * cl, kk, Z, kk, L.s_z, nullptr, 0, false, Sq, D, L.s_traj, T, h->st));
    if (kk < D) HIPCHK(zero_cols(p, Sq, L.s_traj, 2 * cl, D, kk, D - kk, T, h->st));
    HIPCHK(gemm(p, p, true, false, D, 2 * cr, 2 * cl, Sq, D, L.s_traj, X, 2 * cr, L.s_x, Sn, 2 * cr, L.s_traj, alpha, T, h->st));
    h->centre = q + 1;
  } else {
    // B_{q+1} = V^dag (D x 2cr), rows >= kk zero; C_q = alpha X V
    if (kk < D) HIPCHK(zero_cols(p, Sn, L.s_traj, D, 2 * cr, 0, 2 * cr, T, h->st));
    HIPCHK(scale_cast(p, 2 * cr, kk, Z, kk, L.s_z, nullptr, 0, true, Sn, 2 * cr, L.s_traj, T, h->st));
    HIPCHK(gemm(p, p, false, true, 2 * cl, D, 2 * cr, X, 2 * cr, L.s_x, Sn, 2 * cr, L.s_traj, Sq, D, L.s_traj, alpha, T, h->st));
    h->centre = q;
  }
  return MPSB_OK;
}

int idle_step(mpsb_batch* h, int layer, int q, int ch, int mode, const int* d_forced, int32_t* branch,
              double* w_record, double* p_out, bool per_call_record = false) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  int r = move_centre(h, q, q);
  if (r) return r;
  char* S = site_ptr(h, q);
  double* rho1 = W<double>(h, L.o_rho1);
  double* kops = W<double>(h, L.o_kops);
  ProfSec sidle(h, PC_SMALL);
  HIPCHK(site_rdm(p, dl(L, q), dr(L, q), S, L.s_traj, rho1, T, h->st));
  EventArgs ea = base_event_args(h, layer, branch, w_record, mode);
  if (per_call_record) {
    ea.rec_stride = 1;
    ea.rec_qbase = q;
  }
  fill_channel_slot(h, ea, 0, ch);
  HIPCHK(launch_site_event(ea, rho1, q, 0, d_forced, kops, p_out, status_ptr(h), h->st));
  HIPCHK(site_apply(p, dl(L, q), dr(L, q), S, L.s_traj, kops, T, h->st));
  return MPSB_OK;
}

bool unitary_ok(const double* m, int nrow, int ncol, double tol) {
  // columns orthonormal: sum_r conj(m[r][i]) m[r][j] = delta_ij
  for (int i = 0; i < ncol; ++i)
    for (int j = 0; j < ncol; ++j) {
      double re = 0, im = 0;
      for (int r = 0; r < nrow; ++r) {
        double ar = m[2 * (r * ncol + i)], ai = m[2 * (r * ncol + i) + 1];
        double br = m[2 * (r * ncol + j)], bi = m[2 * (r * ncol + j) + 1];
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
      }
      if (std::fabs(re - (i == j ? 1.0 : 0.0)) > tol || std::fabs(im) > tol) return false;
    }
  return true;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char* mps_last_error(void) { return g_err.c_str(); }

int mps_batch_plan(int n_traj, int n_qubits, int chi, int precision, size_t* state_bytes, size_t* work_bytes) {
  if (!state_bytes || !work_bytes) return fail(MPSB_EINVAL, "null output pointer");
  Layout L;
  int r = make_layout(n_traj, n_qubits, chi, precision, L);
  if (r) return r;
  *state_bytes = L.state_bytes;
  *work_bytes = L.work_bytes;
  return MPSB_OK;
}

int mps_batch_create(int n_traj, int n_qubits, int chi, int precision, uint64_t seed, void* state_buf,
                     size_t state_bytes, void* work_buf, size_t work_bytes, void* stream, mpsb_handle* out) {
  if (!out) return fail(MPSB_EINVAL, "null handle pointer");
  Layout L;
  int r = make_layout(n_traj, n_qubits, chi, precision, L);
  if (r) return r;
  if (!state_buf || !work_buf) return fail(MPSB_EINVAL, "null buffer");
  if (((uintptr_t)state_buf & 255) || ((uintptr_t)work_buf & 255)) return fail(MPSB_EINVAL, "buffers must be 256-byte aligned");
  if (state_bytes < L.state_bytes || work_bytes < L.work_bytes) return fail(MPSB_ENOMEM, "buffer smaller than planned");
  mpsb_batch* h = new mpsb_batch();
  h->L = L;
  h->seed = seed;
  h->state = (char*)state_buf;
  h->work = (char*)work_buf;
  h->st = (hipStream_t)stream;
  h->centre = 0;
  h->next_layer = 0;
  h->has_circuit = false;
  h->depth = 0;
  h->n_channels = 0;
  h->mode = MPSB_OPTIMAL;
  std::vector<long long> off(L.off.begin(), L.off.end());
  hipError_t e = hipMemcpyAsync(W<long long>(h, L.o_siteoff), off.data(), sizeof(long long) * L.n, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemsetAsync(status_ptr(h), 0, 256, h->st);
  if (e == hipSuccess) e = init_state(L.prec == MPSB_FP64 ? 1 : 0, h->state, W<long long>(h, L.o_siteoff), L.n, L.s_traj, L.n_traj, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) {
    delete h;
    return fail(MPSB_EHIP, std::string("initialising the state: ") + hipGetErrorString(e));
  }
  *out = h;
  return MPSB_OK;
}

int mps_circuit_validate(int n, const mpsb_circuit* c) {
  if (!c) return fail(MPSB_EINVAL, "null argument");
  if (n < 2 || n > MPSB_MAX_QUBITS) return fail(MPSB_EINVAL, "n_qubits out of range");
  if (c->depth < 0 || c->depth > 65535) return fail(MPSB_EINVAL, "depth must be in 0..65535");
  if (c->n_channels < 0 || c->n_channels > MPSB_MAX_CHANNELS) return fail(MPSB_EINVAL, "n_channels out of range");
  if (c->unravel_mode != MPSB_ORTHOGONAL && c->unravel_mode != MPSB_FIXED && c->unravel_mode != MPSB_OPTIMAL)
    return fail(MPSB_EINVAL, "unknown unravel mode");
  if (c->depth > 0 && (!c->gates || !c->events)) return fail(MPSB_EINVAL, "null gates / events");
  if (c->n_channels > 0 && (!c->kraus || !c->n_kraus)) return fail(MPSB_EINVAL, "null kraus table");
  if (c->unravel_mode == MPSB_FIXED && c->n_channels > 0 && !c->fixed_u) return fail(MPSB_EINVAL, "FIXED mode needs fixed_u");
  const int mp = n / 2;
  // gates
  for (int l = 0; l < c->depth; ++l) {
    int par = l % 2;
    for (int i = 0; par + 2 * i + 1 < n; ++i) {
      const double* g = c->gates + ((size_t)l * mp + i) * 32;
      for (int x = 0; x < 32; ++x)
        if (!std::isfinite(g[x])) return fail(MPSB_ENUM, "non-finite gate entry");
      if (!unitary_ok(g, 4, 4, 1e-12)) return fail(MPSB_EINVAL, "gate " + std::to_string(l) + "/" + std::to_string(i) + " is not unitary");
    }
  }
  // channels
  for (int ch = 0; ch < c->n_channels; ++ch) {
    int r = c->n_kraus[ch];
    if (r < 1 || r > 4) return fail(MPSB_EINVAL, "n_kraus must be in 1..4");
    const double* k = c->kraus + (size_t)ch * 32;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < r; ++i)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int m = 0; m < 2; ++m) {
            // (K^dag K)[a][b] += conj(K[m][a]) K[m][b]
            double xr = k[2 * (4 * i + 2 * m + a)], xi = k[2 * (4 * i + 2 * m + a) + 1];
            double yr = k[2 * (4 * i + 2 * m + b)], yi = k[2 * (4 * i + 2 * m + b) + 1];
            s[2 * (2 * a + b)] += xr * yr + xi * yi;
            s[2 * (2 * a + b) + 1] += xr * yi - xi * yr;
          }
    for (int x = 0; x < 32; ++x)
      if (!std::isfinite(k[x])) return fail(MPSB_ENUM, "non-finite Kraus entry");
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        if (std::fabs(s[2 * (2 * a + b)] - (a == b ? 1.0 : 0.0)) > 1e-12 || std::fabs(s[2 * (2 * a + b) + 1]) > 1e-12)
          return fail(MPSB_EKRAUS, "channel " + std::to_string(ch) + " is not trace preserving");
    if (c->unravel_mode == MPSB_FIXED) {
      // the used columns of U must be orthonormal
      std::vector<double> sub(4 * r * 2);
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < r; ++i)
          for (int z = 0; z < 2; ++z) sub[2 * (j * r + i) + z] = c->fixed_u[(size_t)ch * 32 + 2 * (4 * j + i) + z];
      if (!unitary_ok(sub.data(), 4, r, 1e-12)) return fail(MPSB_EINVAL, "fixed mixing is not an isometry on the used columns");
    }
  }
  for (int l = 0; l < c->depth; ++l)
    for (int q = 0; q < n; ++q) {
      int e = c->events[(size_t)l * n + q];
      if (e < -1 || e >= c->n_channels) return fail(MPSB_EINVAL, "event channel id out of range");
    }
  return MPSB_OK;
}

int mps_batch_set_circuit(mpsb_handle h, const mpsb_circuit* c) {
  if (!h || !c) return fail(MPSB_EINVAL, "null argument");
  const int n = h->L.n;
  const int mp = n / 2;
  int rv = mps_circuit_validate(n, c);
  if (rv) return rv;
  h->depth = c->depth;
  h->gates.assign(c->gates, c->gates + (size_t)c->depth * mp * 32);
  h->n_channels = c->n_channels;
  h->kraus.assign(c->kraus, c->kraus + (size_t)c->n_channels * 32);
  h->n_kraus.assign(c->n_kraus, c->n_kraus + c->n_channels);
  h->events.assign(c->events, c->events + (size_t)c->depth * n);
  h->mode = c->unravel_mode;
  if (c->fixed_u) h->fixed_u.assign(c->fixed_u, c->fixed_u + (size_t)c->n_channels * 32);
  else h->fixed_u.clear();
  h->has_circuit = true;
  return MPSB_OK;
}

int apply_layer(mpsb_handle h, int layer, double* discarded, int32_t* branch, double* w_record) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (!h->has_circuit) return fail(MPSB_EINVAL, "no circuit set");
  if (layer < 0 || layer >= h->depth) return fail(MPSB_EINVAL, "layer out of range");
  if (layer != h->next_layer) return fail(MPSB_EINVAL, "layers must be applied in order");
  const Layout& L = h->L;
  const int n = L.n, mp = n / 2, par = layer % 2;
  // ops in sweep order
  struct Op { int q; bool gate; };
  std::vector<Op> ops;
  std::vector<char> covered(n, 0);
  for (int q = par; q + 1 < n; q += 2) { covered[q] = covered[q + 1] = 1; }
  for (int q = 0; q < n; ++q) {
    if (q >= par && (q - par) % 2 == 0 && q + 1 < n) ops.push_back({q, true});
    else if (!covered[q] && h->events[(size_t)layer * n + q] >= 0) ops.push_back({q, false});
  }
  const bool l2r = (par == 0);
  if (!l2r) std::reverse(ops.begin(), ops.end());
  if (branch) HIPCHK(hipMemsetAsync(branch, 0xFF, sizeof(int32_t) * (size_t)L.n_traj * n, h->st));
  if (w_record) HIPCHK(hipMemsetAsync(w_record, 0, sizeof(double) * 32 * (size_t)L.n_traj * n, h->st));
  if (discarded) HIPCHK(hipMemsetAsync(discarded, 0, sizeof(double) * (size_t)L.n_traj * mp, h->st));
  for (const Op& op : ops) {
    int r;
    if (op.gate) {
      Mat4 g;
      const double* gp = h->gates.data() + ((size_t)layer * mp + (op.q - par) / 2) * 32;
      for (int x = 0; x < 32; ++x) g.v[x] = gp[x];
      int ch_s = h->events[(size_t)layer * n + op.q], ch_t = h->events[(size_t)layer * n + op.q + 1];
      double* disc = discarded ? discarded + (op.q - par) / 2 : nullptr;
      r = two_site_step(h, layer, op.q, g, ch_s, ch_t, l2r, L.cap[op.q], disc, mp, 0, branch, w_record);
    } else {
      r = idle_step(h, layer, op.q, h->events[(size_t)layer * n + op.q], h->mode, nullptr, branch, w_record, nullptr);
    }
    if (r) return r;
  }
  h->next_layer = layer + 1;
  return MPSB_OK;
}

int sample_kraus(mpsb_handle h, const int32_t* qubit, int channel, int unravel_mode, int rng_layer,
                 const int32_t* forced, int32_t* branch, double* p) {
  if (!h || !qubit) return fail(MPSB_EINVAL, "null argument");
  if (!h->has_circuit) return fail(MPSB_EINVAL, "no circuit set");
  if (channel < 0 || channel >= h->n_channels) return fail(MPSB_EINVAL, "channel out of range");
  if (unravel_mode != MPSB_ORTHOGONAL && unravel_mode != MPSB_FIXED && unravel_mode != MPSB_OPTIMAL)
    return fail(MPSB_EINVAL, "unknown unravel mode");
  if (unravel_mode == MPSB_FIXED && h->fixed_u.empty()) return fail(MPSB_EINVAL, "FIXED mode needs the circuit's fixed_u");
  if (rng_layer < 0 || rng_layer > 65535) return fail(MPSB_EINVAL, "rng_layer out of range");
  const int T = h->L.n_traj;
  const int q = qubit[0];
  for (int t = 0; t < T; ++t)
    if (qubit[t] != q) return fail(MPSB_ENOTSUP, "all trajectories must use the same qubit");
  if (q < 0 || q >= h->L.n) return fail(MPSB_EINVAL, "qubit out of range");
  if (forced)
    for (int t = 0; t < T; ++t)
      if (forced[t] < -1 || forced[t] > 3) return fail(MPSB_EINVAL, "forced branch must be -1..3");
  int r = move_centre(h, q, q);
  if (r) return r;
  int* d_forced = nullptr;
  if (forced) {
    d_forced = W<int>(h, h->L.o_pbuf);   // 4*T doubles of room
    HIPCHK(hipMemcpyAsync(d_forced, forced, sizeof(int) * T, hipMemcpyHostToDevice, h->st));
    // feasibility first: no state change on a zero-probability forced branch
    const int p_ = h->L.prec == MPSB_FP64 ? 1 : 0;
    HIPCHK(site_rdm(p_, dl(h->L, q), dr(h->L, q), site_ptr(h, q), h->L.s_traj, W<double>(h, h->L.o_rho1), T, h->st));
    EventArgs ea = base_event_args(h, rng_layer, nullptr, nullptr, unravel_mode);
    fill_channel_slot(h, ea, 0, channel);
    HIPCHK(launch_site_event_check(ea, W<double>(h, h->L.o_rho1), 0, d_forced, status_ptr(h), h->st));
    r = check_status(h);
    if (r) return r;
  }
  return idle_step(h, rng_layer, q, channel, unravel_mode, d_forced, branch, nullptr, p, true);
}

int mps_truncate(mpsb_handle h, int chi, double* discarded) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (chi < 1 || chi > h->L.chi) return fail(MPSB_EINVAL, "chi must be in 1..batch chi");
  const Layout& L = h->L;
  Mat4 id;
  memset(&id, 0, sizeof(id));
  for (int i = 0; i < 4; ++i) id.v[2 * (4 * i + i)] = 1.0;
  if (discarded) HIPCHK(hipMemsetAsync(discarded, 0, sizeof(double) * L.n_traj, h->st));
  for (int k = 0; k + 1 < L.n; ++k) {
    int r = two_site_step(h, -1, k, id, -1, -1, true, std::min(chi, L.cap[k]), discarded, 1, 1, nullptr, nullptr);
    if (r) return r;
  }
  int r = move_centre(h, 0, 0);
  if (r) return r;
  return MPSB_OK;
}

int expect(mpsb_handle h, double* mean, double* m2, double* per_traj) {
  if (!h || !mean || !m2) return fail(MPSB_EINVAL, "null argument");
  const Layout& L = h->L;
  const int n = L.n, nobs = 2 * n - 1, T = L.n_traj;
  const int p = L.prec == MPSB_FP64 ? 1 : 0;
  double* obs = per_traj ? per_traj : W<double>(h, L.o_obs);
  double* norms = W<double>(h, L.o_norm);
  const long long se = L.s_env;   // c128 elements per slot
  char* ex = W<char>(h, L.o_exp);
  const int chunk = L.exp_chunk;
  ProfSec sexp(h, PC_EXPECT);
  for (int t0 = 0; t0 < T; t0 += chunk) {
    const int ct = std::min(chunk, T - t0);
    // per trajectory of the chunk: [R_0 .. R_n][L][Lz][Lzp][Y][Tm][site]
    const long long per = (long long)(n + 1 + 8) * se;   // c128 elements
    auto slot = [&](int s) { return (double*)(ex + (size_t)s * se * 16); };
    double* Rs = slot(0);
    double* Lc = slot(n + 1);
    double* Lz = slot(n + 2);
    double* Lzp = slot(n + 3);
    double* Y = slot(n + 4);
    double* Tm = slot(n + 5);
    double* Sw = slot(n + 6);   // 2 slots
    const long long sp = per;   // trajectory stride (c128 elements)
    auto site_c128 = [&](int k) -> const void* {
      const char* s = site_ptr(h, k) + (size_t)t0 * L.s_traj * L.esz;
      if (p == 1) return s;
      return s;  // widened below
    };
    (void)site_c128;
    auto get_site = [&](int k, long long& stride) -> const void* {
      const char* s = site_ptr(h, k) + (size_t)t0 * L.s_traj * L.esz;
      if (p == 1) { stride = L.s_traj; return s; }
      long long len = 2LL * dl(L, k) * dr(L, k);
      (void)widen(s, L.s_traj, Sw, sp, len, ct, h->st);
      stride = sp;
      return Sw;
    };
    // R_n = 1
    HIPCHK(env_init(Rs + (size_t)n * se * 2, sp, ct, h->st));
    for (int k = n - 1; k >= 0; --k) {
      long long ss;
      const void* A = get_site(k, ss);
      const int cl = dl(L, k), cr = dr(L, k);
      double* Rin = Rs + (size_t)(k + 1) * se * 2;
      double* Rout = Rs + (size_t)k * se * 2;
      // Tm = A2 Rin  (A2: (2cl) x cr)
      HIPCHK(gemm(1, 1, false, false, 2 * cl, cr, cr, A, cr, ss, Rin, cr, sp, Tm, cr, sp, nullptr, ct, h->st));
      // Rout = Tm' A'^dag  (Tm', A' : cl x 2cr)
      HIPCHK(gemm(1, 1, false, true, cl, cl, 2 * cr, Tm, 2 * cr, sp, A, 2 * cr, ss, Rout, cl, sp, nullptr, ct, h->st));
    }
    HIPCHK(env_init(Lc, sp, ct, h->st));
    double* ob = obs + (size_t)t0 * nobs;
    for (int k = 0; k < n; ++k) {
      long long ss;
      const void* A = get_site(k, ss);
      const int cl = dl(L, k), cr = dr(L, k);
      double* Rn = Rs + (size_t)(k + 1) * se * 2;
      // Tm = Lc A' (cl x 2cr)
      HIPCHK(gemm(1, 1, false, false, cl, 2 * cr, cl, Lc, cl, sp, A, 2 * cr, ss, Tm, 2 * cr, sp, nullptr, ct, h->st));
      // Lz = A2^dag Tm2 with the s=1 half negated; Lc' = A2^dag Tm2
      double* Lnew = Y;   // temporarily
      HIPCHK(gemm(1, 1, true, false, cr, cr, 2 * cl, A, cr, ss, Tm, cr, sp, Lnew, cr, sp, nullptr, ct, h->st));
      HIPCHK(neg_cols(Tm, sp, cl, 2 * cr, cr, cr, ct, h->st));
      HIPCHK(gemm(1, 1, true, false, cr, cr, 2 * cl, A, cr, ss, Tm, cr, sp, Lz, cr, sp, nullptr, ct, h->st));
      HIPCHK(obs_trace(cr, Lz, sp, Rn, sp, ob + k, nobs, ct, h->st));
      if (k >= 1) {
        const int clp = cl;
        // Y = Z-weighted transfer of Lzp through site k
        HIPCHK(gemm(1, 1, false, false, clp, 2 * cr, clp, Lzp, clp, sp, A, 2 * cr, ss, Tm, 2 * cr, sp, nullptr, ct, h->st));
        HIPCHK(neg_cols(Tm, sp, clp, 2 * cr, cr, cr, ct, h->st));
        HIPCHK(gemm(1, 1, true, false, cr, cr, 2 * clp, A, cr, ss, Tm, cr, sp, Lzp, cr, sp, nullptr, ct, h->st));
        HIPCHK(obs_trace(cr, Lzp, sp, Rn, sp, ob + n + k - 1, nobs, ct, h->st));
      }
      // rotate: Lc <- Lnew, Lzp <- Lz
      HIPCHK(hipMemcpy2DAsync(Lc, sp * 16, Lnew, sp * 16, (size_t)cr * cr * 16, ct, hipMemcpyDeviceToDevice, h->st));
      HIPCHK(hipMemcpy2DAsync(Lzp, sp * 16, Lz, sp * 16, (size_t)cr * cr * 16, ct, hipMemcpyDeviceToDevice, h->st));
    }
    // norm = L_n (1x1)
    HIPCHK(hipMemcpy2DAsync(norms + t0, sizeof(double), Lc, sp * 16, sizeof(double), ct, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(obs_normalise(ob, nobs, norms + t0, ct, h->st));
    (void)Rs;
  }
  HIPCHK(obs_reduce(obs, nobs, T, mean, m2, h->st));
  return MPSB_OK;
}

int mps_profile(mpsb_handle h, int enable) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  prof_collect(h);
  for (int c = 0; c < PC_COUNT; ++c) { h->prof.ms[c] = 0; h->prof.count[c] = 0; }
  h->prof.on = enable != 0;
  return MPSB_OK;
}

int mps_profile_read(mpsb_handle h, double* ms, long long* count, int n) {
  if (!h || !ms || !count) return fail(MPSB_EINVAL, "null argument");
  prof_collect(h);
  for (int c = 0; c < n && c < PC_COUNT; ++c) { ms[c] = h->prof.ms[c]; count[c] = h->prof.count[c]; }
  return PC_COUNT;
}

int mps_batch_sync(mpsb_handle h) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->st));
  return check_status(h);
}

int mps_batch_destroy(mpsb_handle h) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  (void)hipStreamSynchronize(h->st);
  for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
  delete h;
  return MPSB_OK;
}

int unravel_opt(int batch, const double* rho_q, const double* kraus, int n_k, const int32_t* kraus_id, int r, double* U,
                double* p, double* eof, void* stream) {
  if (batch < 0) return fail(MPSB_EINVAL, "batch < 0");
  if (r < 1 || r > 4) return fail(MPSB_EINVAL, "r must be in 1..4");
  if (n_k < 1 || n_k > MPSB_MAX_CHANNELS) return fail(MPSB_EINVAL, "n_k out of range");
  if (batch == 0) return MPSB_OK;
  if (!rho_q || !kraus || !U || !p || !eof) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(launch_unravel_opt(batch, rho_q, kraus, kraus_id, r, U, p, eof, (hipStream_t)stream));
  return MPSB_OK;
}

int unravel_cost(int batch, const void* theta_, int chi_l, int chi_r, int prec, const double* kraus,
                 const double* params, const double* u_ref, int kind, double* f_out, double* rho_out, void* stream) {
  if (batch < 0 || chi_l < 1 || chi_r < 1) return fail(MPSB_EINVAL, "bad sizes");
  if (prec != MPSB_FP32_BULK && prec != MPSB_FP64) return fail(MPSB_EINVAL, "bad precision");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!theta_ || !kraus || !params || !u_ref || !f_out || !rho_out) return fail(MPSB_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(cost_rho(batch, theta_, chi_l, chi_r, prec == MPSB_FP64 ? 1 : 0, rho_out, st));
  HIPCHK(cost_eval(batch, rho_out, kraus, params, u_ref, kind, f_out, st));
  return MPSB_OK;
}

int unravel_cost_grad(int batch, const double* rho_q, const double* kraus, const double* params, const double* u_ref,
                      int kind, const double* grad_f, double* grad_out, void* stream) {
  if (batch < 0) return fail(MPSB_EINVAL, "bad sizes");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!rho_q || !kraus || !params || !u_ref || !grad_out) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(cost_grad(batch, rho_q, kraus, params, u_ref, kind, grad_f, grad_out, (hipStream_t)stream));
  return MPSB_OK;
}

}  // extern "C"
