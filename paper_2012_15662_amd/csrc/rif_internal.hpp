// Internal context, workspace arena and launch helpers of librif.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <initializer_list>
#include <string>
#include <vector>

#include "rif.h"

struct rif_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  std::string err;
  // workspace arena: one device allocation, grown on demand
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_limit = 0;
  int* dflag = nullptr;       // device status word for device-side validation
  // profiling
  bool prof = false;
  std::string prof_only;      // non-empty: record only launches of this name
  struct Ev { std::string name; hipEvent_t a, b; };
  std::vector<Ev> evs;        // recorded pairs, not yet folded
  std::vector<hipEvent_t> pool;
  struct Tot { std::string name; long launches; double ms; };
  std::vector<Tot> totals;
  // tile-variant selection
  int tune_mode = 0;          // 0: heuristic, 1: measure every variant on first use of a shape
  int force_variant = -1;     // >= 0: use this variant everywhere (clamped per kernel)
  struct Tune { std::string key; int variant; std::vector<float> ms; };
  std::vector<Tune> tune;
  // second stream for the steps of a build that feed neither neighbour
  // (default priority; created on first use) and the fork/join events
  hipStream_t side = nullptr;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // rocBLAS handle of the orbital step's eigensolver (created on first use)
  void* blas = nullptr;
  // orbital-step eigensolver (rif_set_eigensolver): kind and workgroup count
  int eig_kind = 0;
  int eig_groups = 0;
  // polls of one exchanged value before a cooperative kernel gives up
  // (rif_set_wait_limit; negative: every wait gives up at once)
  long long wait_limit = 1LL << 22;
  // device address of the file-scope scratch array of rif_jk_mo_noalloc on
  // this context's device (resolved at rif_create) and its size
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
};

namespace rif {

// Bits of the device status word set by device-side validation.
enum : int { kBadOcc = 1, kBadSum = 2, kBadMap = 4, kBadCount = 8, kNonFinite = 16 };

// Fails the current call with a message.
rif_status fail(rif_ctx* c, rif_status s, const std::string& msg);
// Ensures the arena holds at least `bytes`; returns RIF_OK or RIF_ENOMEM/RIF_EHIP.
rif_status ws_reserve(rif_ctx* c, size_t bytes);

// Carves aligned sub-buffers from the arena.
struct Carve {
  size_t off = 0;
  template <class T>
  size_t take(size_t n) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + n * sizeof(T);
    return o;
  }
};

// Event-pair bracket around a launch when profiling is on.
struct ProfScope {
  rif_ctx* c;
  int idx = -1;
  ProfScope(rif_ctx* c_, const char* name);
  ~ProfScope();
};

rif_status check_launch(rif_ctx* c, const char* what);

// Chooses the tile variant of `kernel` for `shape`.  Forced variant if set;
// else with autotuning on, the first call for a key times each of the `nvar`
// variants through run(v) (every kernel overwrites its whole output, so the
// trial launches are harmless) and caches the fastest; else `heuristic`.
// Returns -1 if a trial launch failed.
int pick_variant(rif_ctx* c, const char* kernel, std::initializer_list<long> shape, int nvar, int heuristic,
                 const std::function<rif_status(int)>& run);

// ---- hot-path operations (kernels.hip) ----
// All pointers are device pointers; shapes already validated.  `prec` is the
// rif_prec mode; b_half/b_mo/Jn/Kn are double for RIF_FP64, float otherwise.
rif_status op_transform(rif_ctx* c, int prec, int nb, int na, int nw, int nmo, const double* b, const double* C,
                        void* bh, void* bmo, double* d);
rif_status op_jk_mo(rif_ctx* c, int prec, int na, int nw, const void* bmo, const double* d, double* J, double* K);
// The same on a static device array (no allocation); op_static_scratch_init
// resolves that array's device address for the context's current device.
rif_status op_static_scratch_init(rif_ctx* c);
rif_status op_jk_mo_noalloc(rif_ctx* c, int prec, int na, int nw, const void* bmo, const double* d, double* J,
                            double* K);
rif_status op_jk_ao(rif_ctx* c, int prec, int nb, int na, int nw, const double* b, const void* bh,
                    const double* d, void* Jn, void* Kn);
rif_status op_energy_grad(rif_ctx* c, int prec, int functional, int nb, int nmo, int npairs, int ncwo,
                          const int* pair_of, const double* H, const double* C, const double* occ,
                          const double* J, const double* K, const void* Jn, const void* Kn, double* energy,
                          double* lambda, double* grad);
// The FP64 half transform over any stack of symmetric n_bf x n_bf slabs:
// out[q][s*n_bf + nu] = sum_mu C[mu][q] slabs[s][mu][nu], q < n_omega, s < nslab.
rif_status op_half_slabs_f64(rif_ctx* c, int nb, long nslab, int nw, int nmo, const double* slabs, const double* C,
                             double* out);
// The conventional four-centre path of Table 1 (fourc.hip): the integrals with
// the first pair packed, eri[(mu nu)][sigma][lambda] (mu <= nu), formed from b,
// and steps 1-3 from them.
unsigned long long eri4_bytes(int nb);
rif_status op_eri4_from_b(rif_ctx* c, int nb, int na, const double* b, double* eri);
rif_status op_jk_4c(rif_ctx* c, int nb, int nw, int nmo, const double* eri, const double* C, double* Jn, double* Kn,
                    double* J, double* K);
// ON optimisation and the warm-start MLP (on_mlp.hip)
typedef rif_on_problem OnProblem;
long on_work_doubles(int nw, int npairs, int ncwo);
long mlp_n_params();
rif_status op_hpp(rif_ctx* c, int nb, int nmo, int nw, const double* H, const double* C, double* Hpp);
rif_status op_on_optimize(rif_ctx* c, int n, const OnProblem* probs);
rif_status op_on_features(rif_ctx* c, int n, const OnProblem* probs, float* X, float* T, float* M, const float* mu,
                          const float* sigma);
rif_status op_on_warmstart(rif_ctx* c, int n, const OnProblem* probs, const float* Pn);
rif_status op_mlp_forward(rif_ctx* c, int nrows, const float* X, const float* M, const float* theta, float* H,
                          float* Z, float* Pn);
rif_status op_mlp_backward(rif_ctx* c, int nrows, const float* X, const float* M, const float* T,
                           const float* theta, const float* H, const float* Z, float* dA, float* grad,
                           double* loss);
rif_status op_adam(rif_ctx* c, int n, float* theta, const float* grad, float* m, float* v, int step, float lr,
                   float b1, float b2, float eps);

// a2..a8 of one molecule in one call (inst already validated), with the small
// independent steps on the context's side stream.
rif_status op_build(rif_ctx* c, int prec, int functional, const rif_instance& in);
// b pre-split for a reduced-precision mode (layouts as in rif.h).
unsigned long long presplit_b_bytes(int nb, int na, int prec);
rif_status op_presplit_b(rif_ctx* c, int prec, int nb, int na, const double* b, void* out);
// The same energy, lambda and G without forming J^q/K^q (in.Jn/in.Kn unused).
rif_status op_build_direct(rif_ctx* c, int prec, int functional, const rif_instance& in);

// FP64 GEMM out[m][n] = sum_k A[k][m] B[k][n] (row strides lda, ldb, ldo), one pass over k.
rif_status op_gemm_kn(rif_ctx* c, int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                      double* out, long ldo);

// The same product with the tile shape chosen per problem (gemm.hip), for the
// large one-off product of the b preparation.
// lower_a: A[k][m] = 0 for k > m + 1 (those products are skipped).
rif_status op_gemm_big(rif_ctx* c, int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                       double* out, long ldo, bool lower_a = false);

// b from the three-centre integrals and the metric (prep.hip)
rif_status op_prepare_b(rif_ctx* c, int nb, int na, const double* T, const double* G, double delta, double* b,
                        int* perm, double* L, double* D, int* nraised);

// Tridiagonal reduction in one cooperative launch (eig.hip): F = Q T Q^T with
// T's diagonal in d and off-diagonal in e, Q row-major.  trd_groups: the
// workgroups for an n x n problem (`want`, or the default when 0), 0 when it
// does not fit.
int trd_groups(rif_ctx* c, int n, int want);
size_t trd_scratch_bytes(int n);
rif_status op_trd(rif_ctx* c, int n, int G, const double* F, double* Q, double* d, double* e, void* scratch,
                  int* err);   // waits bounded by c->wait_limit

// Eigen-decomposition of a symmetric tridiagonal matrix by divide and conquer
// (tdc.hip): d (n, in: diagonal, out: eigenvalues ascending), e (n-1), Z0 and
// Z1 n x n each; on return row c of Z0 is eigenvector c.  *err (cleared at
// the start) is set by a non-finite entry of T (T is then taken as zero) or a
// leaf that fails to converge.  2 <= n <= tdc_max_n().
size_t tdc_scratch_bytes(int n);
int tdc_max_n();
rif_status op_tdc(rif_ctx* c, int n, double* d, double* e, double* Z0, double* Z1, void* scratch, int* err);

// Orbital optimisation (orbital.hip)
rif_status op_maxabs(rif_ctx* c, long n, const double* x, double* part, double* out);
rif_status op_orbital_step(rif_ctx* c, int nb, int nmo, int nw, const double* lam, const double* eps_in,
                           double* C, double* eps_out, int* info);
rif_status op_optimize(rif_ctx* c, int prec, int fn, const rif_instance& in, const rif_opt_params& par, double* C,
                       double* occ, double* gamma, rif_opt_result* res, double* hist_e, double* hist_g,
                       int hist_len);
void op_orbital_release(rif_ctx* c);

// Batched builds (inst already validated); the handle is opaque to the ABI layer.
rif_status op_batch_create(rif_ctx* c, int prec, int functional, int n, const rif_instance* inst, void** out);
rif_status op_batch_run(void* handle, int use_graph);
void op_batch_destroy(void* handle);

}  // namespace rif
