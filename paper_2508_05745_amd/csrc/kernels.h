// Launch wrappers of the mpsb HIP kernels (host-side declarations).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mpsb {

// Arguments of the noise-event kernels.  Channel data either travel by value (at most two
// channels: slot 0 the lower / single qubit of the launch, slot 1 the upper qubit of a gate),
// or, when ev_ids is set, come from the device circuit tables: the channel of the event on
// qubit x of trajectory t in the current layer is
//   ev_ids[t * ev_traj_stride + layer * ev_layer_stride + x]   (-1: no event),
// with its Kraus operators, their count and the fixed mixing in kraus_tab / nk_tab / fixed_tab.
// The layer is read from *layer_ptr when that is set (device layer counter), else `layer`.
// Branch draws are keyed by the global trajectory index traj_base + t.
struct EventArgs {
  int n_traj, n_qubits, layer, mode;
  int rec_stride, rec_qbase;   // record index = traj * rec_stride + (qubit - rec_qbase)
  uint64_t seed;
  int32_t* branch_out;   // [n_traj][rec_stride] or NULL
  double* w_out;         // [n_traj][rec_stride][4][4] c128 or NULL
  // replay inputs in the record layouts (NULL: choose / draw): the mixing U and the branch
  // of each event are taken from here instead
  const double* w_in;
  const int32_t* branch_in;
  int n_kraus[2];
  double kraus[2][32];
  double fixed_u[2][32];
  const int* ev_ids;
  long long ev_traj_stride;
  int ev_layer_stride;
  const double* kraus_tab;   // [n_ch][4][2][2] c128
  const int* nk_tab;         // [n_ch]
  const double* fixed_tab;   // [n_ch][4][4] c128 or NULL
  const int* layer_ptr;
  long long traj_base;   // global trajectory index of trajectory 0 (key of its branch draws)
};

// Gate of a two-site step: by value, or (pool set) pool[ids[t * traj_stride + layer *
// layer_stride + pair]] with the layer read from *layer.
struct GateRef {
  const double* pool;   // [n][4][4] c128
  const int* ids;
  long long traj_stride;
  int layer_stride, pair;
  const int* layer;
};

// active: per-batch-entry mask (NULL = all); inactive entries are left untouched.
// prec: 0 = complex64 storage / FP32 arithmetic, 1 = complex128 / FP64; gemm prec_out 2 =
// c128 output with FP64 accumulation of c64 operands; lower: only the 64 x 64 output tiles that
// hold elements on or below the diagonal are written (Hermitian products read from their lower
// triangle)
hipError_t gemm(int prec_in, int prec_out, bool conj_a, bool conj_b, int M, int N, int K, const void* A, int lda,
                long long sA, const void* B, int ldb, long long sB, void* C, int ldc, long long sC,
                const double* alpha, int batch, hipStream_t st, bool lower = false, const int* active = nullptr);
hipError_t theta(int prec, int chi_l, int chi_m, int chi_r, const void* Cs, const void* Bs, long long s_traj,
                 void* out, long long s_out, const Mat4& gate, const GateRef& gref, double* partial, int n_traj,
                 hipStream_t st, int variant = -1);
// theta kernel variants: 0 = 32 x 32 tiles, 1 = 64 x 64 tiles (FP32 only); -1 = default rule
int theta_variant_ok(int prec, int variant, int chi_l, int chi_r);
int theta_default_variant(int prec, int chi_l, int chi_r);
int theta_tiles(int variant, int chi_l, int chi_r);
// device layer counter
hipError_t set_int(int* p, int v, hipStream_t st);
hipError_t inc_int(int* p, hipStream_t st);
// batched strided copy of rows x row_elems elements between per-trajectory blocks (a kernel,
// so that it can sit in a captured graph)
hipError_t copy_blocks_k(int prec, void* dst, long long s_dst, const void* src, long long s_src, long long elems,
                         int n_traj, hipStream_t st);
hipError_t kraus_pair(int prec, int chi_l, int chi_r, void* X, long long s_traj, const double* kops, int n_traj,
                      hipStream_t st);
hipError_t scale_cast(int prec, int rows, int cols, const void* in, int ld_in, long long s_in,
                      const double* col_scale, long long s_scale, bool conj_t, void* out, int ld_out,
                      long long s_out, int n_traj, hipStream_t st);
hipError_t init_state(int prec, void* state, const long long* d_site_off, int n_sites, long long s_traj,
                      int n_traj, hipStream_t st);

size_t heev_ws_doubles(int n, int keep);
size_t heev_gws_doubles(int keep);
// phase 0: tridiagonalisation, 1: eigenvalues + inverse iteration, 2: orthonormalisation of
// the tridiagonal eigenvectors, 3: back-transformation
hipError_t heev_phase(int phase, int n, int keep, double zero_tol, void* A, long long sA, double* ws, long long sW,
                      double* gws, long long sG, double* evals, long long sE, double* kept_sum, void* Z, long long sZ,
                      int batch, hipStream_t st, const int* active = nullptr);

hipError_t launch_gate_events(const EventArgs& ea, const double* partial, int n_tiles, int q, int has_s, int has_t,
                              double* kops, int* status, hipStream_t st);
hipError_t launch_site_event(const EventArgs& ea, const double* rho1, int q, int slot, const int* forced,
                             double* kops, double* p_out, int* status, hipStream_t st);
hipError_t launch_site_event_check(const EventArgs& ea, const double* rho1, int slot, const int* forced, int* status,
                                   hipStream_t st);
// Born sampling: V = 1 for the first site; one site's draw from W = V A_k (see unravel.hip)
hipError_t born_init(int prec, void* V, long long sV, int S, int n_traj, hipStream_t st);
hipError_t born_step(int prec, const void* W, long long sW, int S, int dr, void* V, long long sV, uint8_t* bits, int n,
                     int k, uint64_t seed, long long traj_base, int n_traj, hipStream_t st);
hipError_t launch_unravel_opt(int batch, const double* rho_q, const double* kraus, int n_k, const int* kraus_id, int r,
                              double* U, double* p, double* eof, hipStream_t st);

// single-site reduced state of a site tensor [a][s][b]: rho1[traj][s][s'] (unnormalised)
hipError_t site_rdm(int prec, int chi_l, int chi_r, const void* site, long long s_traj, double* rho1, int n_traj,
                    hipStream_t st);
// apply the per-trajectory 2x2 operator (first block of kops) to the physical index of a site
hipError_t site_apply(int prec, int chi_l, int chi_r, void* site, long long s_traj, const double* kops, int n_traj,
                      hipStream_t st);
// renormalisation factors 1/sqrt(kept) and discarded weight (kept / trace)
hipError_t bond_entropy(const double* ev, long long sE, int keep, double* out, int stride, int n_traj, hipStream_t st);
hipError_t trunc_factors(const double* kept, const double* ws, long long sW, int n, double* alpha,
                         double* discarded, int disc_stride, int accumulate, int n_traj, hipStream_t st);
// untruncated splits: 1 / ||X||_F per trajectory (and a zero discarded weight unless
// accumulating), and block re-mapping between full-capacity matrices and compact live blocks
// (dst[i][j] = alpha * src[i][t * sh + b] with (t, b) = (j / dh, j % dh), live iff i < ri,
// t < 2, b < bh; conj_t reads conj(src[t * sh + b][i]); src NULL: identity on the live block;
// zero elsewhere)
hipError_t split_norm(int prec, const void* X, long long sX, long long len, double* alpha, double* discarded,
                      int disc_stride, int accumulate, int n_traj, hipStream_t st);
hipError_t remap(int prec, void* dst, long long sD, int ldd, int drows, int dcols, int dh, int ri, int bh,
                 const void* src, long long sS, int lds, int sh, bool conj_t, const double* alpha, int n_traj,
                 hipStream_t st);
// second-level truncation (cuts below the Gram's resolution): per-trajectory decision and
// masked resolved directions, elementwise difference, placement of the residual directions
hipError_t l2_prep(const double* evals, long long sE, const double* ws, long long sW, const double* kept_l1, int n,
                   int kk, double tau, const double* Z, long long sZ, double* Zr, long long sZr, int* act, int* r,
                   double* info, int n_traj, hipStream_t st);
hipError_t l2_sub(double* out, long long sO, const double* a, long long sa, const double* b, long long sb, long long len,
                  const int* act, int n_traj, hipStream_t st);
hipError_t l2_merge(const int* act, const int* r, int n, int kk, double* Z, long long sZ, const double* Z2, long long sZ2,
                    const double* ev2, long long sE, const double* info, double* alpha, double* discarded,
                    int disc_stride, int accumulate, int n_traj, hipStream_t st);
// block copies (c128) into a sub-block of a larger matrix, and accumulation
hipError_t put_block(double* dst, long long sD, int ldd, int r0, int c0, int rows, int cols, const double* src,
                     long long sS, int lds, bool conj_t, int n_traj, hipStream_t st);
hipError_t add_c128(double* acc, long long sA, const double* b, long long sB, long long len, int n_traj, hipStream_t st);
// the static work area (one per device): address of this device's area (taken once per
// device), or busy = true while another batch holds it
hipError_t static_work_acquire(void** ptr, int* device, bool* busy);
void static_work_release(int device);
// inverse square roots / square roots of hop eigenvalues (0 for dropped)
hipError_t hop_scales(const double* evals, long long sE, int n, double* inv_sqrt, double* sqrt_, int n_traj,
                      hipStream_t st);

// centre hop by Gram-Cholesky (n <= 128): Q replaces C in place, R written to Rout
hipError_t hop_chol(int prec, int n, int left_to_right, int other, const void* E, long long sE, void* C, long long sC,
                    void* Rout, long long sR, double tol, int n_traj, hipStream_t st);

hipError_t zero_cols(int prec, void* X, long long sX, int rows, int ld, int c0, int w, int n_traj, hipStream_t st);
// observables: <Z_i>, <Z_i Z_(i+1)> from the two-site reduced state of a theta step (identity
// gate), and the deterministic mean / M2 over trajectories
hipError_t obs_pair(const double* partial, int n_tiles, int i, int n, double* per_traj, int stride, int n_traj,
                    hipStream_t st);
hipError_t fill_nan(double* per_traj, int stride, int c0, int n_traj, hipStream_t st);
// certified error: per-trajectory accumulation of a layer's step errors, and the estimate
hipError_t err_accumulate(int n_traj, int slots, const double* disc, int kind, double weight, double* eps_tot,
                          hipStream_t st);
hipError_t err_estimate(int n_traj, const double* eps_tot, double eps_max, double delta, double* out, hipStream_t st);
// rows of per_traj are stride doubles apart (stride >= n_obs)
hipError_t obs_reduce(const double* per_traj, int n_obs, int stride, int n_traj, double* mean, double* m2,
                      hipStream_t st);

// unravelling cost
hipError_t cost_rho(int batch, const void* theta, int chi_l, int chi_r, int prec, double* rho, hipStream_t st);
hipError_t cost_eval(int batch, const double* rho, const double* nm, const double* kraus, const double* params,
                     const double* u_ref, int kind, double* f, hipStream_t st);
hipError_t cost_grad(int batch, const double* rho, const double* nm, const double* kraus, const double* params,
                     const double* u_ref, int kind, const double* grad_f, double* grad, hipStream_t st);
hipError_t bond_moments(int batch, const void* theta, int chi_l, int chi_r, int prec, double* rho, double* nmom,
                        hipStream_t st);

}  // namespace mpsb
