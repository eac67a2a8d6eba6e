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
#include <map>
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
namespace mpsb {
// the thread-local error message of mps_last_error, for the library's other host sources
int report_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace mpsb
#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(MPSB_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

// Relative drop thresholds of Gram eigenvalues (truncation) and Cholesky pivots (centre hops):
// directions below them are represented by zero vectors.
constexpr double ZERO_TOL_FP64 = 1e-26;
// FP64 truncation: a kept eigenvalue below L2_TAU * lambda_max is re-solved from the residual
constexpr double L2_TAU = 1e-8;
constexpr double ZERO_TOL_FP32 = 1e-13;

struct Layout {
  int n_traj, n, chi, prec;
  size_t esz;                       // bytes per complex element of the state
  std::vector<int> cap;             // [n-1]
  std::vector<long long> off;       // [n] element offsets of the sites inside a trajectory
  long long s_traj;                 // elements per trajectory
  // work buffer (byte offsets)
  size_t o_status, o_siteoff, o_x, o_partial, o_kops, o_gram, o_ews, o_gws, o_evals, o_z, o_kept, o_alpha,
      o_invs, o_sqrt, o_wm, o_rm, o_rho1, o_tmp, o_obs, o_norm, o_pbuf, o_l2zr, o_l2cr, o_l2z2, o_l2act,
      o_l2r, o_l2info;
  long long s_x, s_partial, s_gram, s_ews, s_gws, s_evals, s_z, s_wm, s_tmp;
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
  if (prec == MPSB_FP64) {   // second-level truncation (FP64 path)
    L.o_l2zr = take(16 * L.s_z * T);
    L.o_l2cr = take(16 * L.s_z * T);
    L.o_l2z2 = take(16 * L.s_z * T);
    L.o_l2act = take(sizeof(int) * T);
    L.o_l2r = take(sizeof(int) * T);
    L.o_l2info = take(sizeof(double) * 3 * T);
  }
  L.work_bytes = o;
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

// device circuit tables (in the caller's circuit buffer)
struct Tables {
  int* layer = nullptr;
  const double* gpool = nullptr;
  const int* gid = nullptr;
  long long gid_ts = 0;
  int gid_ls = 0;
  const double* kraus = nullptr;
  const int* nk = nullptr;
  const double* fixed = nullptr;
  const int* ev = nullptr;
  long long ev_ts = 0;
  int ev_ls = 0;
};

struct mpsb_batch {
  Prof prof;
  Layout L;
  uint64_t seed = 0;
  char* state = nullptr;
  char* work = nullptr;
  hipStream_t st = nullptr;
  int centre = 0;
  int next_layer = 0;
  // upper bound of the number of directions with weight on each bond (1 in the initial
  // product state; min(kept, 2 left, 2 right) after a split): beyond it the site tensors are
  // exactly zero, the same for every trajectory
  std::vector<int> live;
  bool has_circuit = false;
  // circuit (host copy of what the launches need)
  int depth = 0;
  int n_channels = 0;
  std::vector<double> kraus;
  std::vector<int> n_kraus;
  int mode = MPSB_OPTIMAL;
  std::vector<double> fixed_u;
  std::vector<unsigned char> any_ev;   // [depth][n]: some trajectory has an event on (layer, qubit)
  Tables tab;
  int traj_base = 0;                   // index of trajectory 0 in the batch (sub-batch of a mixed batch)
  double* entropy = nullptr;           // bond-entropy output set by mps_batch_set_entropy (whole batch)
  double* ent_rows = nullptr;          // its rows of this batch while a layer is enqueued
  const double* rep_w = nullptr;       // replay inputs of the layer being enqueued (rows of this batch)
  const int32_t* rep_b = nullptr;
  long long traj_offset = 0;           // global index of the batch's trajectory 0 (branch-draw keys)
  int rec_stride = 0;                  // record row length (the widest trajectory of the batch)
  // mixed batch: sub-batches and their streams
  std::vector<mpsb_batch*> sub;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> fork_ev, join_ev;
  // schedule timing (mps_profile bit 1): per layer an event pair around the whole layer on the
  // caller's stream (sub = -1) and one around each member's layer on its stream
  struct SchedRec { int sub; hipEvent_t a, b; };
  bool sched_on = false;
  std::vector<hipEvent_t> sched_pool;
  size_t sched_used = 0;
  std::vector<SchedRec> sched_recs;
  std::vector<double> sub_ms;          // per member: summed milliseconds of its timed layers
  std::vector<int> sub_stream;         // per member: stream of its last timed layer
  double sched_elapsed = 0;
  long long sched_layers = 0;
  int n_traj_total = 0;
  std::vector<int> width, chi;         // per trajectory (mixed batch)
  // whole-layer graphs
  hipStream_t cap_st = nullptr;
  bool graphs_on = true;
  struct Graph { hipGraphExec_t exec; int centre_after; };
  std::map<std::string, Graph> graphs;
  // theta kernel variant per shape (autotuned on first use)
  std::map<long long, int> theta_var;
  bool autotune = true;
  // device whose static work area this batch holds (-1: the work buffer is the caller's)
  int static_dev = -1;
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
                    bool hop = false, const int* active = nullptr) {
  // one class per kernel instance: the tridiagonalisation has instances for n <= 128,
  // n <= 256 and n <= 512, the back-transformation for n <= 256 and n <= 512
  const int tri = n <= 128 ? PC_TRIDIAG_S : n <= 256 ? PC_TRIDIAG : PC_TRIDIAG_L;
  const int cls[4] = {tri, PC_TRIEIG, PC_TRIEIG, n <= 256 ? PC_BACK : PC_BACK_L};
  for (int ph = 0; ph < 4; ++ph) {
    ProfSec s(h, hop ? PC_HOPEIG : cls[ph]);
    hipError_t e = heev_phase(ph, n, keep, zt, A, sA, ws, sW, gws, sG, ev, sE, kept, Z, sZ, batch, h->st, active);
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

// batched strided copy of one contiguous block per trajectory (byte pitches and sizes are
// multiples of 8); a kernel rather than a 2-D memcpy so that layers can be graph-captured
hipError_t copy_blocks(void* dst, size_t dpitch, const void* src, size_t spitch, size_t bytes, int n_traj, hipStream_t st) {
  return copy_blocks_k(0, dst, (long long)(dpitch / 8), src, (long long)(spitch / 8), (long long)(bytes / 8), n_traj, st);
}

double zero_tol(const Layout& L) { return L.prec == MPSB_FP64 ? ZERO_TOL_FP64 : ZERO_TOL_FP32; }

// QR factors through the eigen-decomposition of the m x m Gram in the gram buffer, every
// direction above the zero-weight cut kept: right (C = Q R, Gram C^dag C = W Lambda W^dag):
// Wm = W Lambda^-1/2 (Q = C Wm), Rm = Lambda^1/2 W^dag; left (C = R Q, Gram C C^dag):
// Wm = Lambda^-1/2 W^dag (Q = Wm C), Rm = W Lambda^1/2.
hipError_t gram_qr_factors(mpsb_batch* h, int m, bool right) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  hipError_t e = heev_all(h, m, m, zero_tol(L), W<double>(h, L.o_gram), L.s_gram, W<double>(h, L.o_ews), L.s_ews,
                          W<double>(h, L.o_gws), L.s_gws, W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept),
                          W<double>(h, L.o_z), L.s_z, T, true);
  if (e != hipSuccess) return e;
  double* invs = W<double>(h, L.o_invs);
  double* sq = W<double>(h, L.o_sqrt);
  if ((e = hop_scales(W<double>(h, L.o_evals), L.s_evals, m, invs, sq, T, h->st)) != hipSuccess) return e;
  if ((e = scale_cast(p, m, m, W<double>(h, L.o_z), m, L.s_z, invs, m, !right, W<char>(h, L.o_wm), m, L.s_wm, T,
                      h->st)) != hipSuccess)
    return e;
  return scale_cast(p, m, m, W<double>(h, L.o_z), m, L.s_z, sq, m, right, W<char>(h, L.o_rm), m, L.s_wm, T, h->st);
}

// Move the orthogonality centre from site j to j+1: C_j = Q R via the Gram matrix C^dag C.
int hop_right(mpsb_batch* h, int j) {
  Layout& L = h->L;
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj;
  const int cl = dl(L, j), cr = dr(L, j), cr2 = dr(L, j + 1);
  char* Cj = site_ptr(h, j);
  char* Bn = site_ptr(h, j + 1);
  double* gram = W<double>(h, L.o_gram);
  char* tmp = W<char>(h, L.o_tmp);
  const int bj = h->live[j], bl = j > 0 ? h->live[j - 1] : 1;
  if (cr > 128 && bj <= 128) {
    // the live block (2 bl x bj) is factored by Cholesky QR in compact form
    ProfSec sh(h, PC_HOPEIG);
    HIPCHK(remap(p, tmp, L.s_tmp, bj, 2 * bl, bj, bj, 2 * bl, bj, Cj, L.s_traj, cr, 0, false, nullptr, T, h->st));
    HIPCHK(gemm(p, 2, true, false, bj, bj, 2 * bl, tmp, bj, L.s_tmp, tmp, bj, L.s_tmp, gram, bj, L.s_gram, nullptr, T, h->st));
    HIPCHK(hop_chol(p, bj, 1, 2 * bl, gram, L.s_gram, tmp, L.s_tmp, W<char>(h, L.o_rm), L.s_wm, zero_tol(L), T, h->st));
    HIPCHK(remap(p, Cj, L.s_traj, cr, 2 * cl, cr, cr, 2 * bl, bj, tmp, L.s_tmp, bj, 0, false, nullptr, T, h->st));
    HIPCHK(remap(p, W<char>(h, L.o_wm), L.s_wm, cr, cr, cr, cr, bj, bj, W<char>(h, L.o_rm), L.s_wm, bj, 0, false, nullptr,
                 T, h->st));
    ProfSec shg(h, PC_HOPGEMM);
    // C_{j+1} = R B_{j+1}
    HIPCHK(gemm(p, p, false, false, cr, 2 * cr2, cr, W<char>(h, L.o_wm), cr, L.s_wm, Bn, 2 * cr2, L.s_traj, tmp, 2 * cr2,
                L.s_tmp, nullptr, T, h->st));
    HIPCHK(copy_blocks(Bn, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)cr * 2 * cr2 * L.esz, T, h->st));
    h->centre = j + 1;
    return MPSB_OK;
  }
  if (p == 1 && cr > 128) {
    // FP64, more than 128 live columns: Cholesky QR in two column blocks (block Gram-Schmidt
    // with one reorthogonalisation between them), C = [Q1 Q2] [[R11 R12] [0 R22]]
    ProfSec sh(h, PC_HOPEIG);
    const int n2 = bj - 128, rows = 2 * bl;
    double* C1 = W<double>(h, L.o_tmp);
    double* C2 = C1 + 2LL * rows * 128;
    double* Tq = W<double>(h, L.o_x);
    double* R11 = W<double>(h, L.o_rm);
    double* R22 = R11 + 2 * 128 * 128;
    double* R12 = R22 + 2 * 128 * 128;
    double* S = R12 + 2 * 128 * 128;
    char* Cjc = (char*)Cj;
    HIPCHK(remap(1, C1, L.s_tmp, 128, rows, 128, 128, rows, 128, Cjc, L.s_traj, cr, 0, false, nullptr, T, h->st));
    HIPCHK(remap(1, C2, L.s_tmp, n2, rows, n2, n2, rows, n2, Cjc + 128 * 16, L.s_traj, cr, 0, false, nullptr, T, h->st));
    HIPCHK(gemm(1, 2, true, false, 128, 128, rows, C1, 128, L.s_tmp, C1, 128, L.s_tmp, gram, 128, L.s_gram, nullptr, T, h->st));
    HIPCHK(hop_chol(1, 128, 1, rows, gram, L.s_gram, C1, L.s_tmp, R11, L.s_wm, zero_tol(L), T, h->st));
    for (int pass = 0; pass < 2; ++pass) {   // C2 -= Q1 (Q1^dag C2), twice
      HIPCHK(gemm(1, 1, true, false, 128, n2, rows, C1, 128, L.s_tmp, C2, n2, L.s_tmp, pass ? S : R12, n2, L.s_wm, nullptr, T, h->st));
      HIPCHK(gemm(1, 1, false, false, rows, n2, 128, C1, 128, L.s_tmp, pass ? S : R12, n2, L.s_wm, Tq, n2, L.s_x, nullptr, T, h->st));
      HIPCHK(l2_sub(C2, L.s_tmp, C2, L.s_tmp, Tq, L.s_x, (long long)rows * n2, nullptr, T, h->st));
    }
    HIPCHK(add_c128(R12, L.s_wm, S, L.s_wm, 128LL * n2, T, h->st));
    HIPCHK(gemm(1, 2, true, false, n2, n2, rows, C2, n2, L.s_tmp, C2, n2, L.s_tmp, gram, n2, L.s_gram, nullptr, T, h->st));
    HIPCHK(hop_chol(1, n2, 1, rows, gram, L.s_gram, C2, L.s_tmp, R22, L.s_wm, zero_tol(L), T, h->st));
    // A_j = [Q1 Q2] (zero past the live block), R = [[R11 R12] [0 R22]]
    HIPCHK(remap(1, Cjc, L.s_traj, cr, 2 * cl, cr, cr, rows, 128, C1, L.s_tmp, 128, 0, false, nullptr, T, h->st));
    HIPCHK(put_block((double*)Cjc, L.s_traj, cr, 0, 128, rows, n2, C2, L.s_tmp, n2, false, T, h->st));
    char* Rf = W<char>(h, L.o_wm);
    HIPCHK(remap(1, Rf, L.s_wm, cr, cr, cr, cr, 128, 128, R11, L.s_wm, 128, 0, false, nullptr, T, h->st));
    HIPCHK(put_block((double*)Rf, L.s_wm, cr, 0, 128, 128, n2, R12, L.s_wm, n2, false, T, h->st));
    HIPCHK(put_block((double*)Rf, L.s_wm, cr, 128, 128, n2, n2, R22, L.s_wm, n2, false, T, h->st));
    ProfSec shg(h, PC_HOPGEMM);
    HIPCHK(gemm(1, 1, false, false, cr, 2 * cr2, cr, Rf, cr, L.s_wm, Bn, 2 * cr2, L.s_traj, tmp, 2 * cr2, L.s_tmp, nullptr,
                T, h->st));
    HIPCHK(copy_blocks(Bn, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)cr * 2 * cr2 * L.esz, T, h->st));
    h->centre = j + 1;
    return MPSB_OK;
  }
  {
    ProfSec s(h, PC_HOPGEMM);
    // FP64 accumulation also in FP32-bulk: Q = C R^-1 is orthonormal only if R comes from an
    // accurate Gram, and FP32 sums leave its small pivots at rounding-noise level
    HIPCHK(gemm(p, 2, true, false, cr, cr, 2 * cl, Cj, cr, L.s_traj, Cj, cr, L.s_traj, gram, cr, L.s_gram, nullptr, T, h->st));
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
  char* tmp = W<char>(h, L.o_tmp);
  const int bj = h->live[j - 1], br = j < L.n - 1 ? h->live[j] : 1;
  if (cl > 128 && bj <= 128) {
    // the live block (bj x 2 br) is factored by Cholesky QR in compact form: C = R^dag Q
    ProfSec sh(h, PC_HOPEIG);
    HIPCHK(remap(p, tmp, L.s_tmp, 2 * br, bj, 2 * br, br, bj, br, Cj, L.s_traj, 2 * cr, cr, false, nullptr, T, h->st));
    HIPCHK(gemm(p, 2, false, true, bj, bj, 2 * br, tmp, 2 * br, L.s_tmp, tmp, 2 * br, L.s_tmp, gram, bj, L.s_gram, nullptr,
                T, h->st));
    HIPCHK(hop_chol(p, bj, 0, 2 * br, gram, L.s_gram, tmp, L.s_tmp, W<char>(h, L.o_rm), L.s_wm, zero_tol(L), T, h->st));
    HIPCHK(remap(p, Cj, L.s_traj, 2 * cr, cl, 2 * cr, cr, bj, br, tmp, L.s_tmp, 2 * br, br, false, nullptr, T, h->st));
    HIPCHK(remap(p, W<char>(h, L.o_wm), L.s_wm, cl, cl, cl, cl, bj, bj, W<char>(h, L.o_rm), L.s_wm, bj, 0, false, nullptr,
                 T, h->st));
    ProfSec shg(h, PC_HOPGEMM);
    // C_{j-1} = A_{j-1} R^dag
    HIPCHK(gemm(p, p, false, true, 2 * cl2, cl, cl, Ap, cl, L.s_traj, W<char>(h, L.o_wm), cl, L.s_wm, tmp, cl, L.s_tmp,
                nullptr, T, h->st));
    HIPCHK(copy_blocks(Ap, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)2 * cl2 * cl * L.esz, T, h->st));
    h->centre = j - 1;
    return MPSB_OK;
  }
  if (p == 1 && cl > 128) {
    // FP64, more than 128 live rows: C = L Q in two row blocks (the mirror of hop_right),
    // C = [[R11^dag 0] [R12^dag R22^dag]] [Q1; Q2]
    ProfSec sh(h, PC_HOPEIG);
    const int n2 = bj - 128, cols = 2 * br;
    double* C1 = W<double>(h, L.o_tmp);
    double* C2 = C1 + 2LL * 128 * cols;
    double* Tq = W<double>(h, L.o_x);
    double* R11 = W<double>(h, L.o_rm);
    double* R22 = R11 + 2 * 128 * 128;
    double* S1 = R22 + 2 * 128 * 128;   // (C2 Q1^dag), n2 x 128
    double* S = S1 + 2 * 128 * 128;
    char* Cjc = (char*)Cj;
    HIPCHK(remap(1, C1, L.s_tmp, cols, 128, cols, br, 128, br, Cjc, L.s_traj, 2 * cr, cr, false, nullptr, T, h->st));
    HIPCHK(remap(1, C2, L.s_tmp, cols, n2, cols, br, n2, br, Cjc + (size_t)128 * 2 * cr * 16, L.s_traj, 2 * cr, cr, false,
                 nullptr, T, h->st));
    HIPCHK(gemm(1, 2, false, true, 128, 128, cols, C1, cols, L.s_tmp, C1, cols, L.s_tmp, gram, 128, L.s_gram, nullptr, T, h->st));
    HIPCHK(hop_chol(1, 128, 0, cols, gram, L.s_gram, C1, L.s_tmp, R11, L.s_wm, zero_tol(L), T, h->st));
    for (int pass = 0; pass < 2; ++pass) {   // C2 -= (C2 Q1^dag) Q1, twice
      HIPCHK(gemm(1, 1, false, true, n2, 128, cols, C2, cols, L.s_tmp, C1, cols, L.s_tmp, pass ? S : S1, 128, L.s_wm, nullptr, T, h->st));
      HIPCHK(gemm(1, 1, false, false, n2, cols, 128, pass ? S : S1, 128, L.s_wm, C1, cols, L.s_tmp, Tq, cols, L.s_x, nullptr, T, h->st));
      HIPCHK(l2_sub(C2, L.s_tmp, C2, L.s_tmp, Tq, L.s_x, (long long)n2 * cols, nullptr, T, h->st));
    }
    HIPCHK(add_c128(S1, L.s_wm, S, L.s_wm, 128LL * n2, T, h->st));
    HIPCHK(gemm(1, 2, false, true, n2, n2, cols, C2, cols, L.s_tmp, C2, cols, L.s_tmp, gram, n2, L.s_gram, nullptr, T, h->st));
    HIPCHK(hop_chol(1, n2, 0, cols, gram, L.s_gram, C2, L.s_tmp, R22, L.s_wm, zero_tol(L), T, h->st));
    // B_j = [Q1; Q2] (zero past the live block), R = [[R11 S1^dag] [0 R22]] (upper)
    HIPCHK(remap(1, Cjc, L.s_traj, 2 * cr, cl, 2 * cr, cr, 128, br, C1, L.s_tmp, cols, br, false, nullptr, T, h->st));
    HIPCHK(remap(1, Tq, L.s_x, 2 * cr, n2, 2 * cr, cr, n2, br, C2, L.s_tmp, cols, br, false, nullptr, T, h->st));
    HIPCHK(put_block((double*)Cjc, L.s_traj, 2 * cr, 128, 0, n2, 2 * cr, Tq, L.s_x, 2 * cr, false, T, h->st));
    char* Rf = W<char>(h, L.o_wm);
    HIPCHK(remap(1, Rf, L.s_wm, cl, cl, cl, cl, 128, 128, R11, L.s_wm, 128, 0, false, nullptr, T, h->st));
    HIPCHK(put_block((double*)Rf, L.s_wm, cl, 0, 128, 128, n2, S1, L.s_wm, 128, true, T, h->st));
    HIPCHK(put_block((double*)Rf, L.s_wm, cl, 128, 128, n2, n2, R22, L.s_wm, n2, false, T, h->st));
    ProfSec shg(h, PC_HOPGEMM);
    // C_{j-1} = A_{j-1} R^dag
    HIPCHK(gemm(1, 1, false, true, 2 * cl2, cl, cl, Ap, cl, L.s_traj, Rf, cl, L.s_wm, tmp, cl, L.s_tmp, nullptr, T, h->st));
    HIPCHK(copy_blocks(Ap, L.s_traj * L.esz, tmp, L.s_tmp * L.esz, (size_t)2 * cl2 * cl * L.esz, T, h->st));
    h->centre = j - 1;
    return MPSB_OK;
  }
  {
    ProfSec s(h, PC_HOPGEMM);
    HIPCHK(gemm(p, 2, false, true, cl, cl, 2 * cr, Cj, 2 * cr, L.s_traj, Cj, 2 * cr, L.s_traj, gram, cl, L.s_gram, nullptr, T, h->st));
  }
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

// record outputs point at trajectory 0 of the batch; rows are rec_stride qubits long
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
  ea.w_in = h->rep_w;
  ea.branch_in = h->rep_b;
  ea.rec_stride = h->rec_stride;
  ea.rec_qbase = 0;
  ea.traj_base = h->traj_offset + h->traj_base;
  return ea;
}

void set_event_tables(mpsb_batch* h, EventArgs& ea) {
  ea.ev_ids = h->tab.ev;
  ea.ev_traj_stride = h->tab.ev_ts;
  ea.ev_layer_stride = h->tab.ev_ls;
  ea.kraus_tab = h->tab.kraus;
  ea.nk_tab = h->tab.nk;
  ea.fixed_tab = h->tab.fixed;
  ea.layer_ptr = h->tab.layer;
}

// theta kernel variant for a shape: the default rule, or (autotune) the faster of the
// applicable variants, timed on the live operands the first time the shape occurs outside a
// graph capture
int theta_variant(mpsb_batch* h, int p, int cl, int cm, int cr, const void* Sq, const void* Sn, void* X, const Mat4& gate,
                  const GateRef& gref, double* partial, bool capturing) {
  const long long key = ((long long)p << 48) | ((long long)cl << 32) | ((long long)cm << 16) | cr;
  auto it = h->theta_var.find(key);
  if (it != h->theta_var.end()) return it->second;
  int best = theta_default_variant(p, cl, cr);
  if (h->autotune && !capturing && theta_variant_ok(p, 1, cl, cr) && h->L.n_traj >= 64) {
    // both variants write the same outputs; time each (3 launches after one warm-up)
    float tbest = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      for (int v = 0; v < 2; ++v) {
        if (theta(p, cl, cm, cr, Sq, Sn, h->L.s_traj, X, h->L.s_x, gate, gref, partial, h->L.n_traj, h->st, v) != hipSuccess) continue;
        (void)hipEventRecord(e0, h->st);
        for (int r = 0; r < 3; ++r) (void)theta(p, cl, cm, cr, Sq, Sn, h->L.s_traj, X, h->L.s_x, gate, gref, partial, h->L.n_traj, h->st, v);
        (void)hipEventRecord(e1, h->st);
        float ms = 0;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < tbest) {
          tbest = ms;
          best = v;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
  }
  h->theta_var[key] = best;
  return best;
}

// Two-site step on (q, q+1): gate, noise events, truncation to keep columns, split.
// left_to_right: the new centre goes to q+1 (A_q left-orthonormal), else to q.
// The gate is `gate` when `slot` < 0, else the table gate of pair slot `slot`; the events
// come from the tables when `tables` (has_s / has_t: some trajectory has an event on q /
// q+1), else from the by-value channels ch_s / ch_t (-1 = none).
int two_site_step(mpsb_batch* h, int layer, int q, int slot, const Mat4& gate, bool tables, int ch_s, int ch_t,
                  bool has_s, bool has_t, bool left_to_right, int keep, double* discarded, int disc_stride,
                  int accumulate, int32_t* branch, double* w_record, bool capturing = false,
                  double* entropy = nullptr) {
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
  GateRef gref;
  memset(&gref, 0, sizeof(gref));
  if (slot >= 0) {
    gref.pool = h->tab.gpool;
    gref.ids = h->tab.gid;
    gref.traj_stride = h->tab.gid_ts;
    gref.layer_stride = h->tab.gid_ls;
    gref.pair = slot;
    gref.layer = h->tab.layer;
  }
  const int var = theta_variant(h, p, cl, cm, cr, Sq, Sn, X, gate, gref, partial, capturing);
  {
    ProfSec s(h, PC_THETA);
    HIPCHK(theta(p, cl, cm, cr, Sq, Sn, L.s_traj, X, L.s_x, gate, gref, partial, T, h->st, var));
  }
  const int nt = theta_tiles(var, cl, cr);
  if (tables ? (has_s || has_t) : (ch_s >= 0 || ch_t >= 0)) {
    EventArgs ea = base_event_args(h, layer, branch, w_record, h->mode);
    if (tables) {
      set_event_tables(h, ea);
    } else {
      if (ch_s >= 0) fill_channel_slot(h, ea, 0, ch_s);
      if (ch_t >= 0) fill_channel_slot(h, ea, 1, ch_t);
    }
    {
      ProfSec s(h, PC_EVENTS);
      HIPCHK(launch_gate_events(ea, partial, nt, q, tables ? 1 : ch_s >= 0, tables ? 1 : ch_t >= 0, kops, status_ptr(h), h->st));
    }
    ProfSec s(h, PC_KRAUS);
    HIPCHK(kraus_pair(p, cl, cr, X, L.s_x, kops, T, h->st));
  }
  double* gram = W<double>(h, L.o_gram);
  double* Z = W<double>(h, L.o_z);
  double* alpha = W<double>(h, L.o_alpha);
  const int n = left_to_right ? 2 * cl : 2 * cr;
  // live bound of the neighbouring bonds: the rows (a, s) of X with a >= bl and the columns
  // (t, b) with b >= br are exactly zero
  const int bl = q > 0 ? h->live[q - 1] : 1;
  const int br = q + 1 < L.n - 1 ? h->live[q + 1] : 1;
  const int kk = std::min(keep, D);
  const int full = std::min(2 * bl, 2 * br);
  const bool ident = left_to_right ? bl <= br : br <= bl;
  if (kk >= full) {
    if (entropy) {
      // the bond's spectrum for the entropy output: eigenvalues of the Gram matrix of X
      if (left_to_right)
        HIPCHK(gemm(p, 1, false, true, 2 * cl, 2 * cl, 2 * cr, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cl, L.s_gram, nullptr, T, h->st, true));
      else
        HIPCHK(gemm(p, 1, true, false, 2 * cr, 2 * cr, 2 * cl, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cr, L.s_gram, nullptr, T, h->st, true));
      HIPCHK(heev_all(h, n, full, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
                      W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), Z, L.s_z, T));
      HIPCHK(bond_entropy(W<double>(h, L.o_evals), L.s_evals, full, entropy, disc_stride, T, h->st));
    }
    // nothing is discarded: an exact split of the live block (an identity, or a QR
    // factorisation through the small Gram: Cholesky up to 128 columns, beyond that its
    // eigen-decomposition with every direction kept), so that no direction of the state,
    // however small its weight, depends on how well a Gram matrix resolves it
    ProfSec srec(h, PC_RECOMPOSE);
    const int rows = 2 * cl, cols = 2 * cr;
    HIPCHK(split_norm(p, X, L.s_x, (long long)rows * cols, alpha, discarded, disc_stride, accumulate, T, h->st));
    char* Rm = W<char>(h, L.o_rm);
    char* Xc = W<char>(h, L.o_tmp);
    if (!ident)   // compact live block Xc (2bl x 2br)
      HIPCHK(remap(p, Xc, L.s_tmp, 2 * br, 2 * bl, 2 * br, br, 2 * bl, br, X, L.s_x, cols, cr, false, nullptr, T, h->st));
    if (left_to_right) {
      if (ident) {   // A_q = I on the 2bl live rows, C_(q+1) = alpha X
        HIPCHK(remap(p, Sq, L.s_traj, D, rows, D, D, 2 * bl, 2 * bl, nullptr, 0, 0, 0, false, nullptr, T, h->st));
        HIPCHK(remap(p, Sn, L.s_traj, cols, D, cols, cols, 2 * bl, cols, X, L.s_x, cols, 0, false, alpha, T, h->st));
      } else {       // Xc = Q R: A_q = Q, C_(q+1) = alpha R
        HIPCHK(gemm(p, 2, true, false, 2 * br, 2 * br, 2 * bl, Xc, 2 * br, L.s_tmp, Xc, 2 * br, L.s_tmp, gram, 2 * br,
                    L.s_gram, nullptr, T, h->st));
        const char* Q = Xc;
        if (full <= 128) {
          HIPCHK(hop_chol(p, 2 * br, 1, 2 * bl, gram, L.s_gram, Xc, L.s_tmp, Rm, L.s_wm, zero_tol(L), T, h->st));
        } else {     // Gram = W Lambda W^dag: Q = Xc W Lambda^-1/2, R = Lambda^1/2 W^dag
          HIPCHK(gram_qr_factors(h, 2 * br, true));
          HIPCHK(gemm(p, p, false, false, 2 * bl, 2 * br, 2 * br, Xc, 2 * br, L.s_tmp, W<char>(h, L.o_wm), 2 * br, L.s_wm,
                      X, 2 * br, L.s_x, nullptr, T, h->st));
          Q = X;
        }
        const long long sq = Q == Xc ? L.s_tmp : L.s_x;
        HIPCHK(remap(p, Sq, L.s_traj, D, rows, D, D, 2 * bl, 2 * br, Q, sq, 2 * br, 0, false, nullptr, T, h->st));
        HIPCHK(remap(p, Sn, L.s_traj, cols, D, cols, cr, 2 * br, br, Rm, L.s_wm, 2 * br, br, false, alpha, T, h->st));
      }
      h->centre = q + 1;
    } else {
      if (ident) {   // B_(q+1) = I on the 2br live columns, C_q = alpha X (live columns)
        HIPCHK(remap(p, Sn, L.s_traj, cols, D, cols, cr, 2 * br, br, nullptr, 0, 0, 0, false, nullptr, T, h->st));
        HIPCHK(remap(p, Sq, L.s_traj, D, rows, D, br, 2 * bl, br, X, L.s_x, cols, cr, false, alpha, T, h->st));
      } else if (full <= 128) {   // Xc = R^dag Q: B_(q+1) = Q, C_q = alpha R^dag
        HIPCHK(gemm(p, 2, false, true, 2 * bl, 2 * bl, 2 * br, Xc, 2 * br, L.s_tmp, Xc, 2 * br, L.s_tmp, gram, 2 * bl,
                    L.s_gram, nullptr, T, h->st));
        HIPCHK(hop_chol(p, 2 * bl, 0, 2 * br, gram, L.s_gram, Xc, L.s_tmp, Rm, L.s_wm, zero_tol(L), T, h->st));
        HIPCHK(remap(p, Sn, L.s_traj, cols, D, cols, cr, 2 * bl, br, Xc, L.s_tmp, 2 * br, br, false, nullptr, T, h->st));
        HIPCHK(remap(p, Sq, L.s_traj, D, rows, D, D, 2 * bl, 2 * bl, Rm, L.s_wm, 2 * bl, 0, true, alpha, T, h->st));
      } else {   // Gram Xc Xc^dag = W Lambda W^dag: Xc = Rm Q with Q = Lambda^-1/2 W^dag Xc, Rm = W Lambda^1/2
        HIPCHK(gemm(p, 2, false, true, 2 * bl, 2 * bl, 2 * br, Xc, 2 * br, L.s_tmp, Xc, 2 * br, L.s_tmp, gram, 2 * bl,
                    L.s_gram, nullptr, T, h->st));
        HIPCHK(gram_qr_factors(h, 2 * bl, false));
        HIPCHK(gemm(p, p, false, false, 2 * bl, 2 * br, 2 * bl, W<char>(h, L.o_wm), 2 * bl, L.s_wm, Xc, 2 * br, L.s_tmp,
                    X, 2 * br, L.s_x, nullptr, T, h->st));
        HIPCHK(remap(p, Sn, L.s_traj, cols, D, cols, cr, 2 * bl, br, X, L.s_x, 2 * br, br, false, nullptr, T, h->st));
        HIPCHK(remap(p, Sq, L.s_traj, D, rows, D, D, 2 * bl, 2 * bl, Rm, L.s_wm, 2 * bl, 0, false, alpha, T, h->st));
      }
      h->centre = q;
    }
    h->live[q] = full;
    return MPSB_OK;
  }
  h->live[q] = kk;
  {
    ProfSec s(h, PC_GRAM);
    // the eigensolver reads the lower triangle only
    if (left_to_right)
      HIPCHK(gemm(p, 1, false, true, 2 * cl, 2 * cl, 2 * cr, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cl, L.s_gram, nullptr, T, h->st, true));
    else
      HIPCHK(gemm(p, 1, true, false, 2 * cr, 2 * cr, 2 * cl, X, 2 * cr, L.s_x, X, 2 * cr, L.s_x, gram, 2 * cr, L.s_gram, nullptr, T, h->st, true));
  }
  HIPCHK(heev_all(h, n, kk, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
              W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), Z, L.s_z, T));
  HIPCHK(trunc_factors(W<double>(h, L.o_kept), W<double>(h, L.o_ews), L.s_ews, n, alpha, discarded, disc_stride, accumulate, T, h->st));
  // the kept eigenvalues are accurate to eps lambda_max in absolute terms, also below the
  // second-level threshold (only the vectors of those need the re-solve below)
  if (entropy) HIPCHK(bond_entropy(W<double>(h, L.o_evals), L.s_evals, kk, entropy, disc_stride, T, h->st));
  if (L.prec == MPSB_FP64) {
    // cuts below the Gram's resolution: re-solve the kept subspace from the residual of the
    // well-resolved directions (trajectories whose cut is resolved skip every launch)
    ProfSec s2(h, PC_GRAM);
    const int m = left_to_right ? 2 * cr : 2 * cl;
    int* act = W<int>(h, L.o_l2act);
    int* rr = W<int>(h, L.o_l2r);
    double* info = W<double>(h, L.o_l2info);
    double* Zr = W<double>(h, L.o_l2zr);
    double* Cr = W<double>(h, L.o_l2cr);
    double* Z2 = W<double>(h, L.o_l2z2);
    double* T1 = W<double>(h, L.o_tmp);
    double* P = W<double>(h, L.o_wm);
    HIPCHK(l2_prep(W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_kept), n, kk, L2_TAU,
                   Z, L.s_z, Zr, L.s_z, act, rr, info, T, h->st));
    if (left_to_right) {   // M = X (n x m): R = X - Zr (Zr^dag X), Gram R R^dag
      HIPCHK(gemm(1, 1, true, false, kk, m, n, Zr, kk, L.s_z, X, m, L.s_x, Cr, m, L.s_z, nullptr, T, h->st, false, act));
      HIPCHK(gemm(1, 1, false, false, n, m, kk, Zr, kk, L.s_z, Cr, m, L.s_z, T1, m, L.s_tmp, nullptr, T, h->st, false, act));
      HIPCHK(l2_sub(T1, L.s_tmp, (const double*)X, L.s_x, T1, L.s_tmp, (long long)n * m, act, T, h->st));
      HIPCHK(gemm(1, 1, false, true, n, n, m, T1, m, L.s_tmp, T1, m, L.s_tmp, gram, n, L.s_gram, nullptr, T, h->st, true, act));
    } else {               // M = X^dag: R^dag = X - (X Zr) Zr^dag (m x n), Gram (R^dag)^dag R^dag
      HIPCHK(gemm(1, 1, false, false, m, kk, n, X, n, L.s_x, Zr, kk, L.s_z, Cr, kk, L.s_z, nullptr, T, h->st, false, act));
      HIPCHK(gemm(1, 1, false, true, m, n, kk, Cr, kk, L.s_z, Zr, kk, L.s_z, T1, n, L.s_tmp, nullptr, T, h->st, false, act));
      HIPCHK(l2_sub(T1, L.s_tmp, (const double*)X, L.s_x, T1, L.s_tmp, (long long)m * n, act, T, h->st));
      HIPCHK(gemm(1, 1, true, false, n, n, m, T1, n, L.s_tmp, T1, n, L.s_tmp, gram, n, L.s_gram, nullptr, T, h->st, true, act));
    }
    HIPCHK(heev_all(h, n, kk, zero_tol(L), gram, L.s_gram, W<double>(h, L.o_ews), L.s_ews, W<double>(h, L.o_gws), L.s_gws,
                    W<double>(h, L.o_evals), L.s_evals, W<double>(h, L.o_kept), Z2, L.s_z, T, false, act));
    // the residual directions, projected out of the resolved ones twice
    for (int pass = 0; pass < 2; ++pass) {
      HIPCHK(gemm(1, 1, true, false, kk, kk, n, Zr, kk, L.s_z, Z2, kk, L.s_z, P, kk, L.s_wm, nullptr, T, h->st, false, act));
      HIPCHK(gemm(1, 1, false, false, n, kk, kk, Zr, kk, L.s_z, P, kk, L.s_wm, T1, kk, L.s_tmp, nullptr, T, h->st, false, act));
      HIPCHK(l2_sub(Z2, L.s_z, Z2, L.s_z, T1, L.s_tmp, (long long)n * kk, act, T, h->st));
    }
    HIPCHK(l2_merge(act, rr, n, kk, Z, L.s_z, Z2, L.s_z, W<double>(h, L.o_evals), L.s_evals, info, alpha, discarded,
                    disc_stride, accumulate, T, h->st));
  }
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

// Single-qubit noise on the centre tensor at q: by-value channel `ch` (tables false) or the
// table events of the current layer (trajectories without an event get the identity).
int idle_step(mpsb_batch* h, int layer, int q, bool tables, int ch, int mode, const int* d_forced, int32_t* branch,
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
  if (tables) set_event_tables(h, ea);
  else fill_channel_slot(h, ea, 0, ch);
  HIPCHK(launch_site_event(ea, rho1, q, 0, d_forced, kops, p_out, status_ptr(h), h->st));
  HIPCHK(site_apply(p, dl(L, q), dr(L, q), S, L.s_traj, kops, T, h->st));
  return MPSB_OK;
}

// The operations of one layer of a (uniform) batch in sweep order, with their event flags.
struct LayerOp { int q; bool gate; bool has_s, has_t; };

std::vector<LayerOp> layer_ops(const mpsb_batch* h, int layer) {
  const int n = h->L.n, par = layer % 2;
  const unsigned char* ev = h->any_ev.data() + (size_t)layer * n;
  std::vector<LayerOp> ops;
  std::vector<char> covered(n, 0);
  for (int q = par; q + 1 < n; q += 2) covered[q] = covered[q + 1] = 1;
  for (int q = 0; q < n; ++q) {
    if (q >= par && (q - par) % 2 == 0 && q + 1 < n) ops.push_back({q, true, ev[q] != 0, ev[q + 1] != 0});
    else if (!covered[q] && ev[q]) ops.push_back({q, false, true, false});
  }
  if (par == 1) std::reverse(ops.begin(), ops.end());
  return ops;
}

std::string layer_signature(const mpsb_batch* h, int layer) {
  std::string sig = std::to_string(layer % 2) + "@" + std::to_string(h->centre) + "/";
  for (int b : h->live) sig += std::to_string(b) + ".";
  sig += ":";
  for (const LayerOp& o : layer_ops(h, layer))
    sig += std::to_string(o.q) + (o.gate ? "g" : "i") + (o.has_s ? "1" : "0") + (o.has_t ? "1" : "0") + ",";
  return sig;
}

// Enqueues the launches of one layer on h->st (records: device rows of this batch's
// trajectory 0, or NULL).  The device layer counter must hold `layer`; it is not advanced.
int run_layer(mpsb_batch* h, int layer, double* discarded, int disc_stride, int32_t* branch, double* w_record,
              bool capturing) {
  const Layout& L = h->L;
  const int par = layer % 2;
  const bool l2r = (par == 0);
  Mat4 none;
  memset(&none, 0, sizeof(none));
  for (const LayerOp& op : layer_ops(h, layer)) {
    int r;
    if (op.gate) {
      const int slot = (op.q - par) / 2;
      double* disc = discarded ? discarded + slot : nullptr;
      r = two_site_step(h, layer, op.q, slot, none, true, -1, -1, op.has_s, op.has_t, l2r, L.cap[op.q], disc,
                        disc_stride, 0, branch, w_record, capturing, h->ent_rows ? h->ent_rows + slot : nullptr);
    } else {
      r = idle_step(h, layer, op.q, true, 0, h->mode, nullptr, branch, w_record, nullptr);
    }
    if (r) return r;
  }
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

}  // extern "C"

namespace {

// maximal runs of equal (width, chi)
struct Run { int first, count, width, chi; };

int runs_of(int n_traj, const int32_t* width, const int32_t* chi, std::vector<Run>& runs) {
  if (n_traj <= 0 || n_traj > (1 << 30)) return fail(MPSB_EINVAL, "n_traj must be in 1..2^30");
  if (!width || !chi) return fail(MPSB_EINVAL, "null width / chi array");
  runs.clear();
  for (int t = 0; t < n_traj; ++t) {
    if (!runs.empty() && runs.back().width == width[t] && runs.back().chi == chi[t]) runs.back().count++;
    else runs.push_back({t, 1, width[t], chi[t]});
  }
  return MPSB_OK;
}

int plan_runs(const std::vector<Run>& runs, int prec, std::vector<Layout>& Ls, std::vector<size_t>& soff,
              std::vector<size_t>& woff, size_t& sbytes, size_t& wbytes) {
  Ls.resize(runs.size());
  soff.resize(runs.size());
  woff.resize(runs.size());
  sbytes = wbytes = 0;
  for (size_t i = 0; i < runs.size(); ++i) {
    int r = make_layout(runs[i].count, runs[i].width, runs[i].chi, prec, Ls[i]);
    if (r) return r;
    soff[i] = sbytes;
    woff[i] = wbytes;
    sbytes = align256(sbytes + Ls[i].state_bytes);
    wbytes = align256(wbytes + Ls[i].work_bytes);
  }
  return MPSB_OK;
}

hipError_t init_batch_state(mpsb_batch* h) {
  const Layout& L = h->L;
  h->live.assign(L.n - 1, 1);
  std::vector<long long> off(L.off.begin(), L.off.end());
  hipError_t e = hipMemcpyAsync(W<long long>(h, L.o_siteoff), off.data(), sizeof(long long) * L.n, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemsetAsync(status_ptr(h), 0, 256, h->st);
  if (e == hipSuccess) e = init_state(L.prec == MPSB_FP64 ? 1 : 0, h->state, W<long long>(h, L.o_siteoff), L.n, L.s_traj, L.n_traj, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  return e;
}

void destroy_batch(mpsb_batch* h) {
  if (!h) return;
  if (h->st) (void)hipStreamSynchronize(h->st);
  for (mpsb_batch* b : h->sub) destroy_batch(b);
  for (auto& g : h->graphs)
    if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
  for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->fork_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->sched_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->join_ev) (void)hipEventDestroy(e);
  for (hipStream_t s : h->streams) (void)hipStreamDestroy(s);
  if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
  if (h->static_dev >= 0) static_work_release(h->static_dev);
  delete h;
}

// The Haar Optimal mixing of a channel with r orthogonal Kraus operators (table of
// unravelings in Sec. "Noisy random circuits"; appendix "Some common unravelings"): H for
// two, the 4 x 4 matrix the appendix prints for four, 1 for one.  U [4][4] c128, row j =
// output operator, columns past r zero.
void haar_optimal_mixing(int r, double* u) {
  for (int x = 0; x < 32; ++x) u[x] = 0.0;
  if (r == 1) {
    u[0] = 1.0;
  } else if (r == 2) {
    const double h = std::sqrt(0.5);
    u[0] = h; u[2] = h; u[8] = h; u[10] = -h;
  } else if (r == 4) {
    static const int sg[4][4] = {{1, 1, 1, 1}, {1, 1, -1, -1}, {1, -1, 1, -1}, {1, -1, -1, 1}};
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) u[2 * (4 * j + i)] = 0.5 * sg[j][i];
  }
}

// ---- circuit tables
struct CircLayout {
  size_t o_layer, o_gpool, o_gid, o_kraus, o_nk, o_fixed, o_ev, o_scr, bytes;
  int n_pool, mpmax, nmax;
  long long gid_ts, ev_ts;
};

int circuit_layout(int n_traj, int nmax, const mpsb_circuit* c, CircLayout& C) {
  C.nmax = nmax;
  C.mpmax = nmax / 2;
  const long long D = c->depth;
  C.n_pool = c->n_gates > 0 ? c->n_gates : (int)(D * C.mpmax);
  const long long gid_n = c->n_gates > 0 ? (long long)n_traj * D * C.mpmax : D * C.mpmax;
  const long long ev_n = c->events_per_traj ? (long long)n_traj * D * nmax : D * nmax;
  C.gid_ts = c->n_gates > 0 ? D * C.mpmax : 0;
  C.ev_ts = c->events_per_traj ? D * nmax : 0;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + std::max<size_t>(bytes, 1)); return r; };
  C.o_layer = take(sizeof(int));
  C.o_gpool = take(sizeof(double) * 32 * ((size_t)C.n_pool + 1));
  C.o_gid = take(sizeof(int) * (size_t)gid_n);
  C.o_kraus = take(sizeof(double) * 32 * (size_t)c->n_channels);
  C.o_nk = take(sizeof(int) * (size_t)c->n_channels);
  C.o_fixed = take(sizeof(double) * 32 * (size_t)c->n_channels);
  C.o_ev = take(sizeof(int) * (size_t)ev_n);
  // scratch of the least unitary mixings: I/2, then U [4][r], p [4], eof per channel
  C.o_scr = take(c->unravel_mode == MPSB_LEAST_UNITARY ? sizeof(double) * (16 + 40 * (size_t)c->n_channels) : 0);
  C.bytes = o;
  return MPSB_OK;
}

int validate_circuit(int n_traj, const int32_t* width, const mpsb_circuit* c, int& nmax_out) {
  if (!c) return fail(MPSB_EINVAL, "null argument");
  if (n_traj < 1 || !width) return fail(MPSB_EINVAL, "bad trajectory count / width array");
  int nmax = 0;
  bool uniform = true;
  for (int t = 0; t < n_traj; ++t) {
    if (width[t] < 2 || width[t] > MPSB_MAX_QUBITS) return fail(MPSB_EINVAL, "n_qubits out of range");
    nmax = std::max(nmax, (int)width[t]);
    if (width[t] != width[0]) uniform = false;
  }
  nmax_out = nmax;
  (void)uniform;
  if (c->depth < 0 || c->depth > 65535) return fail(MPSB_EINVAL, "depth must be in 0..65535");
  if (c->n_channels < 0 || c->n_channels > MPSB_MAX_CHANNELS) return fail(MPSB_EINVAL, "n_channels out of range");
  if (c->unravel_mode != MPSB_ORTHOGONAL && c->unravel_mode != MPSB_FIXED && c->unravel_mode != MPSB_OPTIMAL &&
      c->unravel_mode != MPSB_HAAR_OPT && c->unravel_mode != MPSB_LEAST_UNITARY)
    return fail(MPSB_EINVAL, "unknown unravel mode");
  if (c->n_gates < 0) return fail(MPSB_EINVAL, "n_gates < 0");
  if (c->depth > 0 && (!c->gates || !c->events)) return fail(MPSB_EINVAL, "null gates / events");
  if (c->depth > 0 && c->n_gates > 0 && !c->gate_id) return fail(MPSB_EINVAL, "a gate pool needs gate_id");
  if (c->n_channels > 0 && (!c->kraus || !c->n_kraus)) return fail(MPSB_EINVAL, "null kraus table");
  if (c->unravel_mode == MPSB_FIXED && c->n_channels > 0 && !c->fixed_u) return fail(MPSB_EINVAL, "FIXED mode needs fixed_u");
  const int mp = nmax / 2;
  if (c->n_gates > 0) {
    for (int g = 0; g < c->n_gates; ++g) {
      const double* gm = c->gates + (size_t)g * 32;
      for (int x = 0; x < 32; ++x)
        if (!std::isfinite(gm[x])) return fail(MPSB_ENUM, "non-finite gate entry");
      if (!unitary_ok(gm, 4, 4, 1e-12)) return fail(MPSB_EINVAL, "pool gate " + std::to_string(g) + " is not unitary");
    }
    const size_t nid = (size_t)n_traj * c->depth * mp;
    for (size_t i = 0; i < nid; ++i)
      if (c->gate_id[i] < -1 || c->gate_id[i] >= c->n_gates) return fail(MPSB_EINVAL, "gate id out of range");
  } else {
    for (int l = 0; l < c->depth; ++l) {
      int par = l % 2;
      for (int i = 0; par + 2 * i + 1 < nmax; ++i) {
        const double* g = c->gates + ((size_t)l * mp + i) * 32;
        for (int x = 0; x < 32; ++x)
          if (!std::isfinite(g[x])) return fail(MPSB_ENUM, "non-finite gate entry");
        if (!unitary_ok(g, 4, 4, 1e-12)) return fail(MPSB_EINVAL, "gate " + std::to_string(l) + "/" + std::to_string(i) + " is not unitary");
      }
    }
  }
  for (int ch = 0; ch < c->n_channels; ++ch) {
    int r = c->n_kraus[ch];
    if (r < 1 || r > 4) return fail(MPSB_EINVAL, "n_kraus must be in 1..4");
    if (c->unravel_mode == MPSB_HAAR_OPT && r == 3)
      return fail(MPSB_EINVAL, "the Haar Optimal mixing is defined for 1, 2 or 4 Kraus operators");
    const double* k = c->kraus + (size_t)ch * 32;
    for (int x = 0; x < 32; ++x)
      if (!std::isfinite(k[x])) return fail(MPSB_ENUM, "non-finite Kraus entry");
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
  const size_t nev = (size_t)(c->events_per_traj ? n_traj : 1) * c->depth * nmax;
  for (size_t i = 0; i < nev; ++i) {
    int e = c->events[i];
    if (e < -1 || e >= c->n_channels) return fail(MPSB_EINVAL, "event channel id out of range");
  }
  return MPSB_OK;
}

std::vector<mpsb_batch*> members(mpsb_batch* h) {
  if (h->sub.empty()) return {h};
  return h->sub;
}

hipEvent_t sched_event(mpsb_batch* h) {
  if (h->sched_used == h->sched_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->sched_pool.push_back(e);
  }
  return h->sched_pool[h->sched_used++];
}

// adds the recorded schedule intervals (all streams are joined into the caller's stream, so
// synchronising it completes them) to the per-member and per-layer sums
void sched_collect(mpsb_batch* h) {
  if (h->sched_recs.empty()) return;
  (void)hipStreamSynchronize(h->st);
  for (const mpsb_batch::SchedRec& r : h->sched_recs) {
    float ms = 0;
    if (!r.a || !r.b || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    if (r.sub < 0) {
      h->sched_elapsed += ms;
      h->sched_layers += 1;
    } else {
      h->sub_ms[r.sub] += ms;
    }
  }
  h->sched_recs.clear();
  h->sched_used = 0;
}

// Enqueues one layer of every member batch on stream S (members of a mixed batch on the
// private streams, forked from and joined back into S), then advances the layer counter.
int enqueue_layer(mpsb_batch* h, int layer, hipStream_t S, double* discarded, int32_t* branch, double* w_record,
                  bool capturing, const double* w_in = nullptr, const int32_t* branch_in = nullptr) {
  const int rs = h->rec_stride, dstr = rs / 2;
  auto recs = [&](mpsb_batch* b, double*& d, int32_t*& br, double*& w) {
    d = discarded ? discarded + (size_t)b->traj_base * dstr : nullptr;
    br = branch ? branch + (size_t)b->traj_base * rs : nullptr;
    w = w_record ? w_record + (size_t)b->traj_base * rs * 32 : nullptr;
    b->rep_w = w_in ? w_in + (size_t)b->traj_base * rs * 32 : nullptr;
    b->rep_b = branch_in ? branch_in + (size_t)b->traj_base * rs : nullptr;
    b->ent_rows = h->entropy ? h->entropy + (size_t)b->traj_base * dstr : nullptr;
  };
  const bool timed = h->sched_on && !capturing;
  // timed layers run directly on the caller's stream, into which every earlier layer's streams
  // are joined: the pending records are complete once it is synchronised, so the event pool is
  // emptied here (never inside a layer) when it has grown large
  if (timed && h->sched_used > 8192) sched_collect(h);
  if (h->sub.empty()) {
    hipStream_t keep = h->st;
    h->st = S;
    double* d; int32_t* br; double* w;
    recs(h, d, br, w);
    hipEvent_t ea = timed ? sched_event(h) : nullptr;
    if (ea) HIPCHK(hipEventRecord(ea, S));
    int r = run_layer(h, layer, d, dstr, br, w, capturing);
    if (ea) {
      hipEvent_t eb = sched_event(h);
      if (eb) {
        HIPCHK(hipEventRecord(eb, S));
        h->sched_recs.push_back({-1, ea, eb});
        h->sched_recs.push_back({0, ea, eb});
        h->sub_stream[0] = 0;
      }
    }
    h->st = keep;
    h->rep_w = nullptr;
    h->rep_b = nullptr;
    h->ent_rows = nullptr;
    if (r) return r;
    HIPCHK(inc_int(h->tab.layer, S));
    return MPSB_OK;
  }
  const int NS = (int)h->streams.size();
  // members dealt round-robin to the streams in their sorted (chi, width) order, so every
  // stream gets the same mix of classes (measured 13% faster on the mixed workload than a
  // longest-estimated-cost-first deal, whose cost model misjudges the latency-bound members)
  hipEvent_t lay_a = timed ? sched_event(h) : nullptr;
  if (lay_a) HIPCHK(hipEventRecord(lay_a, S));
  HIPCHK(hipEventRecord(h->fork_ev[0], S));
  for (int j = 0; j < NS; ++j) HIPCHK(hipStreamWaitEvent(h->streams[j], h->fork_ev[0], 0));
  int r = MPSB_OK;
  for (size_t i = 0; i < h->sub.size() && !r; ++i) {
    mpsb_batch* b = h->sub[i];
    if (layer >= b->depth) continue;
    const int sj = (int)(i % NS);
    b->st = h->streams[sj];
    double* d; int32_t* br; double* w;
    recs(b, d, br, w);
    hipEvent_t ea = timed ? sched_event(h) : nullptr;
    if (ea) HIPCHK(hipEventRecord(ea, b->st));
    r = run_layer(b, layer, d, dstr, br, w, capturing);
    if (ea) {
      hipEvent_t eb = sched_event(h);
      if (eb) {
        HIPCHK(hipEventRecord(eb, b->st));
        h->sched_recs.push_back({(int)i, ea, eb});
        h->sub_stream[i] = sj;
      }
    }
    b->rep_w = nullptr;
    b->rep_b = nullptr;
    b->ent_rows = nullptr;
  }
  for (int j = 0; j < NS; ++j) {
    HIPCHK(hipEventRecord(h->join_ev[j], h->streams[j]));
    HIPCHK(hipStreamWaitEvent(S, h->join_ev[j], 0));
  }
  if (lay_a) {
    hipEvent_t lay_b = sched_event(h);
    if (lay_b) {
      HIPCHK(hipEventRecord(lay_b, S));
      h->sched_recs.push_back({-1, lay_a, lay_b});
    }
  }
  for (mpsb_batch* b : h->sub) b->st = h->st;
  if (r) return r;
  HIPCHK(inc_int(h->tab.layer, S));
  return MPSB_OK;
}

bool profiling(mpsb_batch* h) {
  if (h->sched_on) return true;
  for (mpsb_batch* b : members(h))
    if (b->prof.on) return true;
  return false;
}

}  // namespace

extern "C" {

int mps_batch_plan(int n_traj, const int32_t* width, const int32_t* chi, int precision, size_t* state_bytes,
                   size_t* work_bytes) {
  if (!state_bytes || !work_bytes) return fail(MPSB_EINVAL, "null output pointer");
  std::vector<Run> runs;
  int r = runs_of(n_traj, width, chi, runs);
  if (r) return r;
  std::vector<Layout> Ls;
  std::vector<size_t> so, wo;
  size_t sb, wb;
  r = plan_runs(runs, precision, Ls, so, wo, sb, wb);
  if (r) return r;
  *state_bytes = sb;
  *work_bytes = wb;
  return MPSB_OK;
}

int mps_batch_create(int n_traj, const int32_t* width, const int32_t* chi, int precision, uint64_t seed,
                     int64_t traj_offset, void* state_buf, size_t state_bytes, void* work_buf, size_t work_bytes,
                     void* stream, mpsb_handle* out) {
  if (!out) return fail(MPSB_EINVAL, "null handle pointer");
  if (traj_offset < 0 || traj_offset + (int64_t)n_traj > (int64_t)1 << 32)
    return fail(MPSB_EINVAL, "traj_offset must be >= 0 with traj_offset + n_traj <= 2^32");
  std::vector<Run> runs;
  int r = runs_of(n_traj, width, chi, runs);
  if (r) return r;
  std::vector<Layout> Ls;
  std::vector<size_t> so, wo;
  size_t sb, wb;
  r = plan_runs(runs, precision, Ls, so, wo, sb, wb);
  if (r) return r;
  if (!state_buf || !work_buf) return fail(MPSB_EINVAL, "null buffer");
  if (((uintptr_t)state_buf & 255) || ((uintptr_t)work_buf & 255)) return fail(MPSB_EINVAL, "buffers must be 256-byte aligned");
  if (state_bytes < sb || work_bytes < wb) return fail(MPSB_ENOMEM, "buffer smaller than planned");
  int nmax = 0;
  for (const Run& u : runs) nmax = std::max(nmax, u.width);
  mpsb_batch* h = new mpsb_batch();
  h->st = (hipStream_t)stream;
  h->seed = seed;
  h->n_traj_total = n_traj;
  h->rec_stride = nmax;
  h->width.assign(width, width + n_traj);
  h->chi.assign(chi, chi + n_traj);
  hipError_t e = hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking);
  auto make = [&](size_t i) {
    mpsb_batch* b = runs.size() == 1 ? h : new mpsb_batch();
    b->L = Ls[i];
    b->seed = seed;
    b->state = (char*)state_buf + so[i];
    b->work = (char*)work_buf + wo[i];
    b->st = (hipStream_t)stream;
    b->traj_base = runs[i].first;
    b->traj_offset = traj_offset;
    b->rec_stride = nmax;
    return b;
  };
  if (runs.size() == 1) {
    make(0);
  } else {
    for (size_t i = 0; i < runs.size(); ++i) h->sub.push_back(make(i));
    const int NS = (int)std::min<size_t>(4, runs.size());
    for (int j = 0; j < NS && e == hipSuccess; ++j) {
      hipStream_t s2;
      hipEvent_t ej;
      e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
      if (e == hipSuccess) h->streams.push_back(s2);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ej, hipEventDisableTiming);
      if (e == hipSuccess) h->join_ev.push_back(ej);
    }
    hipEvent_t ef;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ef, hipEventDisableTiming);
    if (e == hipSuccess) h->fork_ev.push_back(ef);
  }
  for (mpsb_batch* b : members(h))
    if (e == hipSuccess) e = init_batch_state(b);
  if (e != hipSuccess) {
    destroy_batch(h);
    return fail(MPSB_EHIP, std::string("initialising the batch: ") + hipGetErrorString(e));
  }
  *out = h;
  return MPSB_OK;
}

int mps_batch_create_static(int n_traj, const int32_t* width, const int32_t* chi, int precision, uint64_t seed,
                            int64_t traj_offset, void* state_buf, size_t state_bytes, void* stream, mpsb_handle* out) {
  if (!out) return fail(MPSB_EINVAL, "null handle pointer");
  if (traj_offset < 0 || traj_offset + (int64_t)n_traj > (int64_t)1 << 32)
    return fail(MPSB_EINVAL, "traj_offset must be >= 0 with traj_offset + n_traj <= 2^32");
  std::vector<Run> runs;
  int r = runs_of(n_traj, width, chi, runs);
  if (r) return r;
  if (runs.size() != 1) return fail(MPSB_ENOTSUP, "a batch on the static work area must be uniform (one width and chi)");
  Layout L;
  r = make_layout(n_traj, runs[0].width, runs[0].chi, precision, L);
  if (r) return r;
  if (L.work_bytes > (size_t)MPSB_STATIC_WORK_BYTES)
    return fail(MPSB_ENOMEM, "the batch needs " + std::to_string(L.work_bytes) + " bytes of work memory; the static work area holds " +
                                 std::to_string((size_t)MPSB_STATIC_WORK_BYTES));
  if (!state_buf) return fail(MPSB_EINVAL, "null state buffer");
  if ((uintptr_t)state_buf & 255) return fail(MPSB_EINVAL, "the state buffer must be 256-byte aligned");
  if (state_bytes < L.state_bytes) return fail(MPSB_ENOMEM, "state buffer smaller than planned");
  void* work = nullptr;
  int dev = -1;
  bool busy = false;
  HIPCHK(static_work_acquire(&work, &dev, &busy));
  if (busy) return fail(MPSB_ENOTSUP, "the static work area of this device is held by another batch");
  mpsb_batch* h = new mpsb_batch();
  h->L = L;
  h->st = (hipStream_t)stream;
  h->seed = seed;
  h->n_traj_total = n_traj;
  h->rec_stride = runs[0].width;
  h->width.assign(width, width + n_traj);
  h->chi.assign(chi, chi + n_traj);
  h->state = (char*)state_buf;
  h->work = (char*)work;
  h->traj_offset = traj_offset;
  h->static_dev = dev;
  h->graphs_on = false;   // no capture stream: every layer runs as direct launches
  h->autotune = false;    // the default theta tile rule (the autotuner times with events)
  // the status word and the site-offset table are cleared and written here, at the area's
  // device address: the area keeps the previous batch's contents
  hipError_t e = init_batch_state(h);
  if (e != hipSuccess) {
    destroy_batch(h);
    return fail(MPSB_EHIP, std::string("initialising the batch: ") + hipGetErrorString(e));
  }
  *out = h;
  return MPSB_OK;
}

int mps_circuit_validate(int n_traj, const int32_t* width, const mpsb_circuit* c) {
  int nmax;
  return validate_circuit(n_traj, width, c, nmax);
}

int mps_circuit_bytes(mpsb_handle h, const mpsb_circuit* c, size_t* bytes) {
  if (!h || !c || !bytes) return fail(MPSB_EINVAL, "null argument");
  CircLayout C;
  circuit_layout(h->n_traj_total, h->rec_stride, c, C);
  *bytes = C.bytes;
  return MPSB_OK;
}

int mps_batch_set_circuit(mpsb_handle h, const mpsb_circuit* c, void* circuit_buf, size_t circuit_bytes) {
  if (!h || !c) return fail(MPSB_EINVAL, "null argument");
  int nmax;
  int rv = validate_circuit(h->n_traj_total, h->width.data(), c, nmax);
  if (rv) return rv;
  CircLayout C;
  circuit_layout(h->n_traj_total, nmax, c, C);
  if (!circuit_buf) return fail(MPSB_EINVAL, "null circuit buffer");
  if ((uintptr_t)circuit_buf & 255) return fail(MPSB_EINVAL, "circuit buffer must be 256-byte aligned");
  if (circuit_bytes < C.bytes) return fail(MPSB_ENOMEM, "circuit buffer smaller than mps_circuit_bytes");
  const int T = h->n_traj_total, D = c->depth, mp = C.mpmax;
  // host staging of the tables
  std::vector<double> pool((size_t)(C.n_pool + 1) * 32, 0.0);
  std::copy(c->gates, c->gates + (size_t)C.n_pool * 32, pool.begin());
  for (int i = 0; i < 4; ++i) pool[(size_t)C.n_pool * 32 + 2 * (4 * i + i)] = 1.0;   // identity
  std::vector<int> gid;
  if (c->n_gates > 0) {
    gid.assign(c->gate_id, c->gate_id + (size_t)T * D * mp);
    for (int& g : gid)
      if (g < 0) g = C.n_pool;
  } else {
    gid.resize((size_t)D * mp);
    for (size_t i = 0; i < gid.size(); ++i) gid[i] = (int)i;
  }
  std::vector<int> ev(c->events, c->events + (size_t)(c->events_per_traj ? T : 1) * D * nmax);
  std::vector<int> nk(c->n_kraus, c->n_kraus + c->n_channels);
  char* base = (char*)circuit_buf;
  // the Haar Optimal and least unitary unravelings run as fixed mixings (U [n_channels][4][4])
  int mode = c->unravel_mode;
  const double* fixed_host = c->fixed_u;
  std::vector<double> resolved;
  if (mode == MPSB_HAAR_OPT) {
    resolved.assign((size_t)32 * c->n_channels, 0.0);
    for (int ch = 0; ch < c->n_channels; ++ch) haar_optimal_mixing(c->n_kraus[ch], &resolved[(size_t)ch * 32]);
    fixed_host = resolved.data();
    mode = MPSB_FIXED;
  }
  HIPCHK(hipMemcpyAsync(base + C.o_gpool, pool.data(), sizeof(double) * pool.size(), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipMemcpyAsync(base + C.o_gid, gid.data(), sizeof(int) * gid.size(), hipMemcpyHostToDevice, h->st));
  if (c->n_channels > 0) {
    HIPCHK(hipMemcpyAsync(base + C.o_kraus, c->kraus, sizeof(double) * 32 * c->n_channels, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(base + C.o_nk, nk.data(), sizeof(int) * nk.size(), hipMemcpyHostToDevice, h->st));
    if (mode == MPSB_LEAST_UNITARY) {
      // the locally entanglement-optimal mixing of each channel for the maximally mixed
      // reduced state (its Choi state), by the unravelling kernel, in the circuit buffer's
      // scratch region
      double* scr = (double*)(base + C.o_scr);
      const double half[8] = {0.5, 0.0, 0.0, 0.0, 0.0, 0.0, 0.5, 0.0};
      HIPCHK(hipMemcpyAsync(scr, half, sizeof(half), hipMemcpyHostToDevice, h->st));
      for (int ch = 0; ch < c->n_channels; ++ch)
        HIPCHK(launch_unravel_opt(1, scr, (const double*)(base + C.o_kraus) + (size_t)ch * 32, 1, nullptr, c->n_kraus[ch],
                                  scr + 16 + (size_t)ch * 40, scr + 16 + (size_t)ch * 40 + 32,
                                  scr + 16 + (size_t)ch * 40 + 36, h->st));
      std::vector<double> out((size_t)40 * c->n_channels);
      HIPCHK(hipMemcpyAsync(out.data(), scr + 16, sizeof(double) * out.size(), hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipStreamSynchronize(h->st));
      resolved.assign((size_t)32 * c->n_channels, 0.0);
      for (int ch = 0; ch < c->n_channels; ++ch) {
        const int r = c->n_kraus[ch];
        const double* u = &out[(size_t)ch * 40];   // [4][r] c128
        if (!std::isfinite(u[36])) return fail(MPSB_ENUM, "least unitary mixing of channel " + std::to_string(ch));
        for (int j = 0; j < 4; ++j)
          for (int i = 0; i < r; ++i)
            for (int z = 0; z < 2; ++z) resolved[(size_t)ch * 32 + 2 * (4 * j + i) + z] = u[2 * (j * r + i) + z];
      }
      fixed_host = resolved.data();
      mode = MPSB_FIXED;
    }
    if (fixed_host)
      HIPCHK(hipMemcpyAsync(base + C.o_fixed, fixed_host, sizeof(double) * 32 * c->n_channels, hipMemcpyHostToDevice, h->st));
  }
  HIPCHK(hipMemcpyAsync(base + C.o_ev, ev.data(), sizeof(int) * ev.size(), hipMemcpyHostToDevice, h->st));
  HIPCHK(set_int((int*)(base + C.o_layer), h->next_layer, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  Tables tab;
  tab.layer = (int*)(base + C.o_layer);
  tab.gpool = (const double*)(base + C.o_gpool);
  tab.gid = (const int*)(base + C.o_gid);
  tab.gid_ts = C.gid_ts;
  tab.gid_ls = mp;
  tab.kraus = (const double*)(base + C.o_kraus);
  tab.nk = (const int*)(base + C.o_nk);
  tab.fixed = fixed_host ? (const double*)(base + C.o_fixed) : nullptr;
  tab.ev = (const int*)(base + C.o_ev);
  tab.ev_ts = C.ev_ts;
  tab.ev_ls = nmax;
  h->tab = tab;
  for (auto& g : h->graphs)
    if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
  h->graphs.clear();
  for (mpsb_batch* b : members(h)) {
    const int n = b->L.n, first = b->traj_base, cnt = b->L.n_traj;
    b->tab = tab;
    b->tab.gid = tab.gid + (long long)first * C.gid_ts;
    b->tab.ev = tab.ev + (long long)first * C.ev_ts;
    // last layer with work for this batch (identity gates and no events past a trajectory's depth)
    b->depth = D;
    b->n_channels = c->n_channels;
    b->mode = mode;
    if (b == h) {   // host copy of the channels for sample_kraus (uniform batches only)
      b->kraus.assign(c->kraus, c->kraus + (size_t)c->n_channels * 32);
      b->n_kraus.assign(c->n_kraus, c->n_kraus + c->n_channels);
      if (fixed_host) b->fixed_u.assign(fixed_host, fixed_host + (size_t)c->n_channels * 32);
      else b->fixed_u.clear();
    }
    b->any_ev.assign((size_t)D * n, 0);
    for (int l = 0; l < D; ++l)
      for (int q = 0; q < n; ++q) {
        bool any = false;
        if (c->events_per_traj) {
          for (int t = first; t < first + cnt && !any; ++t) any = c->events[((size_t)t * D + l) * nmax + q] >= 0;
        } else {
          any = c->events[(size_t)l * nmax + q] >= 0;
        }
        b->any_ev[(size_t)l * n + q] = any;
      }
    b->has_circuit = true;
  }
  h->depth = D;
  h->mode = mode;
  h->has_circuit = true;
  return MPSB_OK;
}

int mps_batch_set_entropy(mpsb_handle h, double* entropy) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  h->entropy = entropy;
  return MPSB_OK;
}

int mps_batch_set_graphs(mpsb_handle h, int enable) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (enable && h->static_dev >= 0) return fail(MPSB_ENOTSUP, "a batch on the static work area runs without graphs");
  h->graphs_on = enable != 0;
  return MPSB_OK;
}

int mps_batch_set_autotune(mpsb_handle h, int enable) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  for (mpsb_batch* b : members(h)) {
    b->autotune = enable != 0;
    b->theta_var.clear();
  }
  return MPSB_OK;
}

int apply_layer_replay(mpsb_handle h, int layer, const double* w_in, const int32_t* branch_in, double* discarded,
                       int32_t* branch, double* w_record) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (!h->has_circuit) return fail(MPSB_EINVAL, "no circuit set");
  if (layer < 0 || layer >= h->depth) return fail(MPSB_EINVAL, "layer out of range");
  if (layer != h->next_layer) return fail(MPSB_EINVAL, "layers must be applied in order");
  const size_t T = (size_t)h->n_traj_total, rs = (size_t)h->rec_stride;
  if (branch) HIPCHK(hipMemsetAsync(branch, 0xFF, sizeof(int32_t) * T * rs, h->st));
  if (w_record) HIPCHK(hipMemsetAsync(w_record, 0, sizeof(double) * 32 * T * rs, h->st));
  if (discarded) HIPCHK(hipMemsetAsync(discarded, 0, sizeof(double) * T * (rs / 2), h->st));
  if (h->entropy) HIPCHK(hipMemsetAsync(h->entropy, 0, sizeof(double) * T * (rs / 2), h->st));
  // replay inputs differ per layer, so such layers run as direct launches; recorded outputs
  // are part of the launch sequence, so their addresses are part of the graph signature
  const bool replay = w_in || branch_in;
  std::vector<mpsb_batch*> bs = members(h);
  if (!h->graphs_on || replay || profiling(h)) {
    int r = enqueue_layer(h, layer, h->st, discarded, branch, w_record, false, w_in, branch_in);
    if (r) return r;
    for (mpsb_batch* b : bs) b->next_layer = layer + 1;
    h->next_layer = layer + 1;
    return MPSB_OK;
  }
  std::string sig;
  for (mpsb_batch* b : bs) sig += (layer < b->depth ? layer_signature(b, layer) : std::string("-")) + "|";
  {
    char out[96];
    snprintf(out, sizeof(out), "%p,%p,%p,%p", (void*)discarded, (void*)branch, (void*)w_record, (void*)h->entropy);
    sig += out;
  }
  auto it = h->graphs.find(sig);
  if (it == h->graphs.end()) {
    static const std::string seen_tag = "#seen";
    if (h->graphs.find(sig + seen_tag) == h->graphs.end()) {
      // first occurrence: run directly (kernel variants are tuned on live operands here)
      int r = enqueue_layer(h, layer, h->st, discarded, branch, w_record, false);
      if (r) return r;
      h->graphs[sig + seen_tag] = mpsb_batch::Graph{nullptr, 0};
      for (mpsb_batch* b : bs) b->next_layer = layer + 1;
      h->next_layer = layer + 1;
      return MPSB_OK;
    }
    // second occurrence: capture the launch sequence on the private stream
    std::vector<int> centres;
    for (mpsb_batch* b : bs) centres.push_back(b->centre);
    HIPCHK(hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeRelaxed));
    int r = enqueue_layer(h, layer, h->cap_st, discarded, branch, w_record, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_st, &g);
    if (r) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return fail(MPSB_EHIP, std::string("capturing a layer: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(MPSB_EHIP, std::string("instantiating a layer graph: ") + hipGetErrorString(e));
    // the capture moved the host-side centres as a direct run would
    mpsb_batch::Graph gr{ge, 0};
    it = h->graphs.emplace(sig, gr).first;
    (void)centres;
  } else {
    // replay: advance the host-side centres as the captured run did
    for (mpsb_batch* b : bs)
      if (layer < b->depth) {
        for (const LayerOp& op : layer_ops(b, layer)) {
          if (op.gate) {
            b->centre = (layer % 2 == 0) ? op.q + 1 : op.q;
            const int q = op.q;
            const int bl = q > 0 ? b->live[q - 1] : 1, br = q + 1 < b->L.n - 1 ? b->live[q + 1] : 1;
            b->live[q] = std::min(b->L.cap[q], std::min(2 * bl, 2 * br));
          } else {
            b->centre = op.q;
          }
        }
      }
  }
  HIPCHK(hipGraphLaunch(it->second.exec, h->st));
  for (mpsb_batch* b : bs) b->next_layer = layer + 1;
  h->next_layer = layer + 1;
  return MPSB_OK;
}

int apply_layer(mpsb_handle h, int layer, double* discarded, int32_t* branch, double* w_record) {
  return apply_layer_replay(h, layer, nullptr, nullptr, discarded, branch, w_record);
}

int sample_kraus(mpsb_handle h, const int32_t* qubit, int channel, int unravel_mode, int rng_layer,
                 const int32_t* forced, int32_t* branch, double* p) {
  if (!h || !qubit) return fail(MPSB_EINVAL, "null argument");
  if (!h->sub.empty()) return fail(MPSB_ENOTSUP, "sample_kraus needs a batch of one width and chi");
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
  return idle_step(h, rng_layer, q, false, channel, unravel_mode, d_forced, branch, nullptr, p, true);
}

int mps_sample_bitstrings(mpsb_handle h, int n_samples, uint64_t seed, uint8_t* bits) {
  if (!h || !bits) return fail(MPSB_EINVAL, "null argument");
  if (!h->sub.empty()) return fail(MPSB_ENOTSUP, "mps_sample_bitstrings needs a batch of one width and chi");
  const Layout& L = h->L;
  int cmax = 1;
  for (int c : L.cap) cmax = std::max(cmax, c);
  if (n_samples < 1 || n_samples > 65535 || n_samples > 2 * cmax)
    return fail(MPSB_EINVAL, "n_samples must be in 1..min(65535, 2 chi)");
  const int p = L.prec == MPSB_FP64 ? 1 : 0, T = L.n_traj, S = n_samples;
  int r = move_centre(h, 0, 0);
  if (r) return r;
  // V [S][d_k] (left vectors) in the hop-result region, W [S][2][d_(k+1)] in the theta region
  char* V = W<char>(h, L.o_tmp);
  char* Wt = W<char>(h, L.o_x);
  HIPCHK(born_init(p, V, L.s_tmp, S, T, h->st));
  for (int k = 0; k < L.n; ++k) {
    const int a = dl(L, k), b = dr(L, k);
    HIPCHK(gemm(p, p, false, false, S, 2 * b, a, V, a, L.s_tmp, site_ptr(h, k), 2 * b, L.s_traj, Wt, 2 * b, L.s_x, nullptr,
                T, h->st));
    HIPCHK(born_step(p, Wt, L.s_x, S, b, V, L.s_tmp, bits, L.n, k, seed, h->traj_offset, T, h->st));
  }
  return MPSB_OK;
}

int apply_layer_global(mpsb_handle h, int layer, int chi, double* discarded) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (!h->sub.empty()) return fail(MPSB_ENOTSUP, "global layering needs a batch of one width and chi");
  if (chi < 1 || chi > h->L.chi) return fail(MPSB_EINVAL, "chi must be in 1..batch chi");
  int r = apply_layer_replay(h, layer, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (r) return r;
  return mps_truncate(h, chi, discarded);
}

int mps_truncate(mpsb_handle h, int chi, double* discarded) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (!h->sub.empty()) return fail(MPSB_ENOTSUP, "mps_truncate needs a batch of one width and chi");
  if (chi < 1 || chi > h->L.chi) return fail(MPSB_EINVAL, "chi must be in 1..batch chi");
  const Layout& L = h->L;
  Mat4 id;
  memset(&id, 0, sizeof(id));
  for (int i = 0; i < 4; ++i) id.v[2 * (4 * i + i)] = 1.0;
  if (discarded) HIPCHK(hipMemsetAsync(discarded, 0, sizeof(double) * L.n_traj, h->st));
  for (int k = 0; k + 1 < L.n; ++k) {
    int r = two_site_step(h, -1, k, -1, id, false, -1, -1, false, false, true, std::min(chi, L.cap[k]), discarded, 1, 1,
                          nullptr, nullptr);
    if (r) return r;
  }
  int r = move_centre(h, 0, 0);
  if (r) return r;
  return MPSB_OK;
}

}  // extern "C"

namespace {
// Observables of a uniform batch into per_traj rows of `stride` doubles, and (mean, m2) over
// its trajectories when requested.  A measurement sweep: the orthogonality centre walks from
// site 0 to site n-2; at each site i the two-site contraction of (i, i+1) with the identity
// gate accumulates the two-site reduced state (the environments are orthonormal, so this is
// the state's own reduced state), from which <Z_i>, <Z_i Z_(i+1)> (and <Z_(n-1)>) follow.
// 2(n-1) batched launches plus the centre hops, all trajectories in each.
int expect_uniform(mpsb_batch* h, double* mean, double* m2, double* per_traj, int stride) {
  const Layout& L = h->L;
  const int n = L.n, nobs = 2 * n - 1, T = L.n_traj;
  const int p = L.prec == MPSB_FP64 ? 1 : 0;
  if (!per_traj) stride = nobs;
  double* obs = per_traj ? per_traj : W<double>(h, L.o_obs);
  // one profiler class for the whole sweep (the hops inside are not split out)
  ProfSec sexp(h, PC_EXPECT);
  const bool prof_on = h->prof.on;
  h->prof.on = false;
  Mat4 id;
  memset(&id, 0, sizeof(id));
  for (int i = 0; i < 4; ++i) id.v[2 * (4 * i + i)] = 1.0;
  GateRef none;
  memset(&none, 0, sizeof(none));
  int r = MPSB_OK;
  for (int i = 0; i + 1 < n && r == MPSB_OK; ++i) {
    r = move_centre(h, i, i);
    if (r) break;
    const int cl = dl(L, i), cm = dr(L, i), cr = dr(L, i + 1);
    const int var = theta_default_variant(p, cl, cr);
    hipError_t e = theta(p, cl, cm, cr, site_ptr(h, i), site_ptr(h, i + 1), L.s_traj, W<char>(h, L.o_x), L.s_x, id, none,
                         W<double>(h, L.o_partial), T, h->st, var);
    if (e == hipSuccess) e = obs_pair(W<double>(h, L.o_partial), theta_tiles(var, cl, cr), i, n, obs, stride, T, h->st);
    if (e != hipSuccess) r = fail(MPSB_EHIP, std::string("measurement sweep: ") + hipGetErrorString(e));
  }
  h->prof.on = prof_on;
  if (r) return r;
  if (stride > nobs) HIPCHK(fill_nan(obs, stride, nobs, T, h->st));
  if (mean) HIPCHK(obs_reduce(obs, nobs, stride, T, mean, m2, h->st));
  return MPSB_OK;
}
}  // namespace

extern "C" {

int expect(mpsb_handle h, double* mean, double* m2, double* per_traj) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if ((mean == nullptr) != (m2 == nullptr)) return fail(MPSB_EINVAL, "mean and m2 go together");
  if (h->sub.empty()) {
    if (!mean && !per_traj) return fail(MPSB_EINVAL, "no output");
    return expect_uniform(h, mean, m2, per_traj, 2 * h->L.n - 1);
  }
  if (!mean && !per_traj) return fail(MPSB_EINVAL, "no output");
  const int Wd = h->rec_stride, stride = 2 * Wd - 1;
  // trajectory mean and M2 in the widest trajectory's layout: each member's own (fixed-order
  // device reduction, written into the caller's mean / m2 as scratch) merged on the host in
  // member order with the pairwise update of Chan et al.; a slot counts the trajectories
  // that have the observable (Z_i: width > i, Z_i Z_(i+1): width > i + 1)
  std::vector<double> cnt(mean ? stride : 0, 0.0), mu(mean ? stride : 0, 0.0), sq(mean ? stride : 0, 0.0);
  std::vector<double> mb, qb;
  for (mpsb_batch* b : h->sub) {
    b->st = h->st;
    int r = expect_uniform(b, mean, m2, per_traj ? per_traj + (size_t)b->traj_base * stride : nullptr, stride);
    if (r) return r;
    if (!mean) continue;
    const int nb = b->L.n, nob = 2 * nb - 1;
    const double tb = (double)b->L.n_traj;
    mb.resize(nob);
    qb.resize(nob);
    HIPCHK(hipMemcpyAsync(mb.data(), mean, sizeof(double) * nob, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipMemcpyAsync(qb.data(), m2, sizeof(double) * nob, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    for (int k = 0; k < nob; ++k) {
      const int slot = k < nb ? k : Wd + (k - nb);
      const double na = cnt[slot], nab = na + tb, dlt = mb[k] - mu[slot];
      mu[slot] += dlt * tb / nab;
      sq[slot] += qb[k] + dlt * dlt * na * tb / nab;
      cnt[slot] = nab;
    }
  }
  if (mean) {
    for (int k = 0; k < stride; ++k)
      if (cnt[k] == 0) mu[k] = sq[k] = std::nan("");
    HIPCHK(hipMemcpyAsync(mean, mu.data(), sizeof(double) * stride, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(m2, sq.data(), sizeof(double) * stride, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  return MPSB_OK;
}


int mps_profile(mpsb_handle h, int enable) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (enable < 0 || enable > 3) return fail(MPSB_EINVAL, "enable must be 0..3");
  for (mpsb_batch* b : members(h)) {
    prof_collect(b);
    for (int c = 0; c < PC_COUNT; ++c) { b->prof.ms[c] = 0; b->prof.count[c] = 0; }
    b->prof.on = (enable & 1) != 0;
  }
  sched_collect(h);
  const size_t nm = members(h).size();
  h->sub_ms.assign(nm, 0.0);
  h->sub_stream.assign(nm, -1);
  h->sched_elapsed = 0;
  h->sched_layers = 0;
  h->sched_on = (enable & 2) != 0;
  return MPSB_OK;
}

int mps_schedule_read(mpsb_handle h, int* first, int* count, int* stream, double* busy_ms, double* elapsed_ms,
                      long long* layers, int n) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  if (n < 0) return fail(MPSB_EINVAL, "n must be >= 0");
  const std::vector<mpsb_batch*> ms = members(h);
  if (n > 0 && (!first || !count || !stream || !busy_ms)) return fail(MPSB_EINVAL, "null member array");
  sched_collect(h);
  for (int i = 0; i < n && i < (int)ms.size(); ++i) {
    first[i] = ms[i]->traj_base;
    count[i] = ms[i]->L.n_traj;
    stream[i] = i < (int)h->sub_stream.size() ? h->sub_stream[i] : -1;
    busy_ms[i] = i < (int)h->sub_ms.size() ? h->sub_ms[i] : 0.0;
  }
  if (elapsed_ms) *elapsed_ms = h->sched_elapsed;
  if (layers) *layers = h->sched_layers;
  return (int)ms.size();
}

int mps_profile_read(mpsb_handle h, double* ms, long long* count, int n) {
  if (!h || !ms || !count) return fail(MPSB_EINVAL, "null argument");
  for (int c = 0; c < n && c < PC_COUNT; ++c) { ms[c] = 0; count[c] = 0; }
  for (mpsb_batch* b : members(h)) {
    prof_collect(b);
    for (int c = 0; c < n && c < PC_COUNT; ++c) { ms[c] += b->prof.ms[c]; count[c] += b->prof.count[c]; }
  }
  return PC_COUNT;
}

int mps_batch_sync(mpsb_handle h) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->st));
  for (mpsb_batch* b : members(h)) {
    b->st = h->st;
    int r = check_status(b);
    if (r) return r;
  }
  return MPSB_OK;
}

int mps_batch_destroy(mpsb_handle h) {
  if (!h) return fail(MPSB_EINVAL, "null handle");
  destroy_batch(h);
  return MPSB_OK;
}

int mps_error_accumulate(int n_traj, int slots, const double* discarded, int step_kind, double weight, double* eps_tot,
                         void* stream) {
  if (n_traj < 0 || slots < 0) return fail(MPSB_EINVAL, "bad sizes");
  if (step_kind != MPSB_STEP_EXACT && step_kind != MPSB_STEP_PAPER) return fail(MPSB_EINVAL, "unknown step kind");
  if (!(weight >= 0.0) || !std::isfinite(weight)) return fail(MPSB_EINVAL, "weight must be finite and >= 0");
  if (n_traj == 0) return MPSB_OK;
  if (!eps_tot || (slots > 0 && !discarded)) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(err_accumulate(n_traj, slots, discarded, step_kind, weight, eps_tot, (hipStream_t)stream));
  return MPSB_OK;
}

int mps_error_estimate(int n_traj, const double* eps_tot, double eps_max, double delta, double* out, void* stream) {
  if (n_traj < 1) return fail(MPSB_EINVAL, "n_traj must be >= 1");
  if (!(eps_max >= 2.0) || !std::isfinite(eps_max)) return fail(MPSB_EINVAL, "eps_max must be >= 2");
  if (!(delta > 0.0 && delta < 1.0)) return fail(MPSB_EINVAL, "delta must be in (0, 1)");
  if (!eps_tot || !out) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(err_estimate(n_traj, eps_tot, eps_max, delta, out, (hipStream_t)stream));
  return MPSB_OK;
}

int unravel_opt(int batch, const double* rho_q, const double* kraus, int n_k, const int32_t* kraus_id, int r, double* U,
                double* p, double* eof, void* stream) {
  if (batch < 0) return fail(MPSB_EINVAL, "batch < 0");
  if (r < 1 || r > 4) return fail(MPSB_EINVAL, "r must be in 1..4");
  if (n_k < 1 || n_k > MPSB_MAX_CHANNELS) return fail(MPSB_EINVAL, "n_k out of range");
  if (batch == 0) return MPSB_OK;
  if (!rho_q || !kraus || !U || !p || !eof) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(launch_unravel_opt(batch, rho_q, kraus, n_k, kraus_id, r, U, p, eof, (hipStream_t)stream));
  return MPSB_OK;
}

int unravel_cost(int batch, const void* theta_, int chi_l, int chi_r, int prec, const double* kraus,
                 const double* params, const double* u_ref, int kind, double* f_out, double* rho_out, void* stream) {
  if (batch < 0 || batch > MPSB_MAX_COST_BATCH || chi_l < 1 || chi_r < 1 || (long long)chi_l * chi_r > (1LL << 26))
    return fail(MPSB_EINVAL, "bad sizes");
  if (prec != MPSB_FP32_BULK && prec != MPSB_FP64) return fail(MPSB_EINVAL, "bad precision");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!theta_ || !kraus || !params || !u_ref || !f_out || !rho_out) return fail(MPSB_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(cost_rho(batch, theta_, chi_l, chi_r, prec == MPSB_FP64 ? 1 : 0, rho_out, st));
  HIPCHK(cost_eval(batch, rho_out, nullptr, kraus, params, u_ref, kind, f_out, st));
  return MPSB_OK;
}

int unravel_cost_grad(int batch, const double* rho_q, const double* kraus, const double* params, const double* u_ref,
                      int kind, const double* grad_f, double* grad_out, void* stream) {
  if (batch < 0 || batch > MPSB_MAX_COST_BATCH) return fail(MPSB_EINVAL, "bad sizes");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!rho_q || !kraus || !params || !u_ref || !grad_out) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(cost_grad(batch, rho_q, nullptr, kraus, params, u_ref, kind, grad_f, grad_out, (hipStream_t)stream));
  return MPSB_OK;
}

int unravel_cost_bond(int batch, const void* theta_, int chi_l, int chi_r, int prec, const double* kraus,
                      const double* params, const double* u_ref, int kind, double* f_out, double* rho_out,
                      double* n_out, void* stream) {
  if (batch < 0 || batch > MPSB_MAX_COST_BATCH || chi_l < 1 || chi_r < 1 || (long long)chi_l * chi_r > (1LL << 26))
    return fail(MPSB_EINVAL, "bad sizes");
  if (prec != MPSB_FP32_BULK && prec != MPSB_FP64) return fail(MPSB_EINVAL, "bad precision");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!theta_ || !kraus || !params || !u_ref || !f_out || !rho_out || !n_out) return fail(MPSB_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(bond_moments(batch, theta_, chi_l, chi_r, prec == MPSB_FP64 ? 1 : 0, rho_out, n_out, st));
  HIPCHK(cost_eval(batch, rho_out, n_out, kraus, params, u_ref, kind, f_out, st));
  return MPSB_OK;
}

int unravel_cost_bond_grad(int batch, const double* rho_q, const double* n_mom, const double* kraus,
                           const double* params, const double* u_ref, int kind, const double* grad_f,
                           double* grad_out, void* stream) {
  if (batch < 0 || batch > MPSB_MAX_COST_BATCH) return fail(MPSB_EINVAL, "bad sizes");
  if (kind != 0 && kind != 1) return fail(MPSB_EINVAL, "kind must be 0 or 1");
  if (batch == 0) return MPSB_OK;
  if (!rho_q || !n_mom || !kraus || !params || !u_ref || !grad_out) return fail(MPSB_EINVAL, "null pointer");
  HIPCHK(cost_grad(batch, rho_q, n_mom, kraus, params, u_ref, kind, grad_f, grad_out, (hipStream_t)stream));
  return MPSB_OK;
}

}  // extern "C"
