// C ABI of librif: context, validation, workspace, profiling, dispatch.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rif_internal.hpp"

namespace rif {

rif_status fail(rif_ctx* c, rif_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

rif_status ws_reserve(rif_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return RIF_OK;
  if (c->ws_limit && bytes > c->ws_limit)
    return fail(c, RIF_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the limit of " +
                                   std::to_string(c->ws_limit));
  // the old arena may still be in use by queued kernels
  if (c->ws) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)1 << 20);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    c->ws = nullptr;
    return fail(c, RIF_ENOMEM, "hipMalloc of " + std::to_string(want) + " workspace bytes failed");
  }
  c->ws_bytes = want;
  return RIF_OK;
}

rif_status check_launch(rif_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, RIF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return RIF_OK;
}

int pick_variant(rif_ctx* c, const char* kernel, std::initializer_list<long> shape, int nvar, int heuristic,
                 const std::function<rif_status(int)>& run) {
  if (c->force_variant >= 0) return std::min(c->force_variant, nvar - 1);
  if (c->tune_mode == 0) return heuristic;
  std::string key = kernel;
  for (long v : shape) key += " " + std::to_string(v);
  for (auto& t : c->tune)
    if (t.key == key && t.variant < nvar) return t.variant;   // (a loaded entry may name too many)
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1; }
  rif_ctx::Tune t{key, heuristic, std::vector<float>(nvar, -1.f)};
  const bool prof = c->prof;
  c->prof = false;
  // One warm-up launch per variant (variants a kernel lacks report an error),
  // then kRounds interleaved rounds of kReps launches each; a variant's time
  // is its fastest round, so a clock still ramping up at the start does not
  // favour the variants timed last.
  constexpr int kRounds = 3, kReps = 2;
  std::vector<char> ok(nvar, 0);
  for (int v = 0; v < nvar; ++v) ok[v] = run(v) == RIF_OK;
  for (int round = 0; round < kRounds; ++round)
    for (int v = 0; v < nvar; ++v) {
      if (!ok[v]) continue;
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < kReps; ++r) run(v);
      (void)hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) { c->prof = prof; return -1; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= kReps;
      if (t.ms[v] < 0.f || ms < t.ms[v]) t.ms[v] = ms;
    }
  float best = 1e30f;
  for (int v = 0; v < nvar; ++v)
    if (ok[v] && t.ms[v] < best) { best = t.ms[v]; t.variant = v; }
  c->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->err.clear();
  c->tune.push_back(t);
  return t.variant;
}

ProfScope::ProfScope(rif_ctx* c_, const char* name) : c(c_) {
  if (!c->prof) return;
  if (!c->prof_only.empty() && c->prof_only != name) return;
  auto get = [&]() {
    hipEvent_t e;
    if (!c->pool.empty()) {
      e = c->pool.back();
      c->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      return (hipEvent_t) nullptr;
    }
    return e;
  };
  rif_ctx::Ev ev{std::string(name), get(), get()};
  if (!ev.a || !ev.b) return;
  hipEventRecord(ev.a, c->stream);
  c->evs.push_back(ev);
  idx = (int)c->evs.size() - 1;
}

ProfScope::~ProfScope() {
  if (idx >= 0) hipEventRecord(c->evs[idx].b, c->stream);
}

}  // namespace rif

using namespace rif;

static bool dims_ok(long n) { return n > 0 && n < (1L << 30); }

extern "C" {

rif_status rif_create(rif_ctx** out, int dev, void* stream) {
  if (!out) return RIF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || dev < 0 || dev >= n) return RIF_EINVAL;
  if (hipSetDevice(dev) != hipSuccess) return RIF_EHIP;
  rif_ctx* c = new rif_ctx();
  c->device = dev;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->own_stream) != hipSuccess) {
      delete c;
      return RIF_EHIP;
    }
    c->stream = c->own_stream;
  }
  if (hipMalloc(&c->dflag, sizeof(int)) != hipSuccess || hipMemset(c->dflag, 0, sizeof(int)) != hipSuccess) {
    if (c->own_stream) hipStreamDestroy(c->own_stream);
    delete c;
    return RIF_EHIP;
  }
  // the static scratch of rif_jk_mo_noalloc on this device; a failure is kept
  // (that entry point then reports it) and leaves every other call working
  if (op_static_scratch_init(c) == RIF_OK) c->err.clear();
  *out = c;
  return RIF_OK;
}

void rif_destroy(rif_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto& e : c->evs) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  if (c->ws) hipFree(c->ws);
  if (c->dflag) hipFree(c->dflag);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
  }
  for (auto e : c->ev)
    if (e) hipEventDestroy(e);
  op_orbital_release(c);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  delete c;
}

const char* rif_last_error(const rif_ctx* c) { return c ? c->err.c_str() : "null context"; }

rif_status rif_set_stream(rif_ctx* c, void* stream) {
  if (!c) return RIF_EINVAL;
  c->stream = stream ? (hipStream_t)stream : c->own_stream;
  if (!c->stream) {
    if (hipStreamCreate(&c->own_stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamCreate failed");
    c->stream = c->own_stream;
  }
  return RIF_OK;
}

rif_status rif_set_workspace_limit(rif_ctx* c, unsigned long long bytes) {
  if (!c) return RIF_EINVAL;
  c->ws_limit = (size_t)bytes;
  return RIF_OK;
}

rif_status rif_sync(rif_ctx* c) {
  if (!c) return RIF_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
  int flag = 0;
  if (hipMemcpy(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, RIF_EHIP, "reading the status word failed");
  if (flag) {
    if (hipMemset(c->dflag, 0, sizeof(int)) != hipSuccess) return fail(c, RIF_EHIP, "hipMemset failed");
    std::string m;
    if (flag & (kBadOcc | kBadSum | kBadMap | kBadCount)) m += "invalid occupations:";
    if (flag & kBadOcc) m += " an ON outside [0,1];";
    if (flag & kBadSum) m += " a pair whose ONs do not sum to 1;";
    if (flag & kBadMap) m += " a pair map entry out of range or a strong orbital g not in pair g;";
    if (flag & kBadCount) m += " a pair without exactly 1 + n_cwo orbitals;";
    if (flag & kNonFinite)
      m += std::string(m.empty() ? "" : " ") + "a non-finite energy or gradient (NaN or infinite inputs, or in "
           "RIF_FP16X3 an operand of a split product of magnitude 65504 or more);";
    return fail(c, RIF_EINVAL, m);
  }
  return RIF_OK;
}

rif_status rif_transform(rif_ctx* c, int nb, int na, int nw, int nmo, const double* b, const double* C,
                         rif_prec prec, void* bh, void* bmo, double* d) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(na) || !dims_ok(nw) || !dims_ok(nmo) || nw > nmo || nmo > nb)
    return fail(c, RIF_EINVAL, "rif_transform: need 0 < n_omega <= n_mo <= n_bf and n_aux > 0");
  if (!b || !C || !bh || !bmo || !d) return fail(c, RIF_EINVAL, "rif_transform: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_transform(c, (int)prec, nb, na, nw, nmo, b, C, bh, bmo, d);
}

rif_status rif_jk_mo(rif_ctx* c, int na, int nw, const void* bmo, const double* d, rif_prec prec, double* J,
                     double* K) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(na) || !dims_ok(nw)) return fail(c, RIF_EINVAL, "rif_jk_mo: need n_aux > 0 and n_omega > 0");
  if (!bmo || !d || !J || !K) return fail(c, RIF_EINVAL, "rif_jk_mo: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_jk_mo(c, (int)prec, na, nw, bmo, d, J, K);
}

rif_status rif_jk_mo_noalloc(rif_ctx* c, int na, int nw, const void* bmo, const double* d, rif_prec prec, double* J,
                             double* K) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(na) || !dims_ok(nw)) return fail(c, RIF_EINVAL, "rif_jk_mo_noalloc: need n_aux > 0 and n_omega > 0");
  if (!bmo || !d || !J || !K) return fail(c, RIF_EINVAL, "rif_jk_mo_noalloc: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_jk_mo_noalloc(c, (int)prec, na, nw, bmo, d, J, K);
}

rif_status rif_jk_ao_per_mo(rif_ctx* c, int nb, int na, int nw, const double* b, const void* bh,
                            const double* d, rif_prec prec, void* Jn, void* Kn) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(na) || !dims_ok(nw) || nw > nb)
    return fail(c, RIF_EINVAL, "rif_jk_ao_per_mo: need 0 < n_omega <= n_bf and n_aux > 0");
  if (!b || !bh || !d || !Jn || !Kn) return fail(c, RIF_EINVAL, "rif_jk_ao_per_mo: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_jk_ao(c, (int)prec, nb, na, nw, b, bh, d, Jn, Kn);
}

rif_status pnof_energy_grad(rif_ctx* c, rif_functional fn, int nb, int nmo, int npairs, int ncwo,
                            const int* pair_of, const double* H, const double* C, const double* occ,
                            const double* J, const double* K, const void* Jn, const void* Kn, rif_prec prec,
                            double* energy, double* lambda, double* grad) {
  if (!c) return RIF_EINVAL;
  if (fn != RIF_PNOF7 && fn != RIF_PNOF5) return fail(c, RIF_EINVAL, "pnof_energy_grad: unknown functional");
  if (!dims_ok(nb) || !dims_ok(nmo) || !dims_ok(npairs) || ncwo < 1 || ncwo > (1 << 20))
    return fail(c, RIF_EINVAL, "pnof_energy_grad: need n_bf, n_mo, n_pairs > 0 and n_cwo >= 1");
  const long nw = (long)npairs * (1 + ncwo);
  if (nw > nmo || nmo > nb) return fail(c, RIF_EINVAL, "pnof_energy_grad: need n_pairs (1 + n_cwo) <= n_mo <= n_bf");
  if (!H || !C || !occ || !J || !K || !Jn || !Kn || !energy || !lambda || !grad)
    return fail(c, RIF_EINVAL, "pnof_energy_grad: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_energy_grad(c, (int)prec, (int)fn, nb, nmo, npairs, ncwo, pair_of, H, C, occ, J, K, Jn, Kn, energy,
                        lambda, grad);
}

static rif_status check_instance(rif_ctx* c, const rif_instance* in, const char* who, bool need_ao = true) {
  if (!in) return fail(c, RIF_EINVAL, std::string(who) + ": NULL instance");
  const long nw = (long)in->n_pairs * (1 + (long)in->n_cwo);   // no int overflow for any inputs
  if (!dims_ok(in->n_bf) || !dims_ok(in->n_aux) || !dims_ok(in->n_mo) || !dims_ok(in->n_pairs) || in->n_cwo < 1 ||
      nw > in->n_mo || in->n_mo > in->n_bf)
    return fail(c, RIF_EINVAL, std::string(who) + ": need n_pairs (1 + n_cwo) <= n_mo <= n_bf, n_aux > 0");
  if (!in->b || !in->C || !in->H || !in->occ || !in->b_half || !in->b_mo || !in->d || !in->J || !in->K ||
      (need_ao && (!in->Jn || !in->Kn)) || !in->energy || !in->lambda || !in->grad)
    return fail(c, RIF_EINVAL, std::string(who) + ": NULL pointer");
  return RIF_OK;
}

rif_status rif_build(rif_ctx* c, const rif_instance* in, rif_prec prec, rif_functional fn) {
  if (!c) return RIF_EINVAL;
  rif_status st = check_instance(c, in, "rif_build");
  if (st) return st;
  if (fn != RIF_PNOF7 && fn != RIF_PNOF5) return fail(c, RIF_EINVAL, "rif_build: unknown functional");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_build(c, (int)prec, (int)fn, *in);
}

rif_status rif_prepare_b(rif_ctx* c, int nb, int na, const double* T, const double* G, double delta, double* b,
                         int* perm, double* L, double* D, int* nraised) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(na) || na > 46340 || (long)nb * nb > (1L << 30))
    return fail(c, RIF_EINVAL, "rif_prepare_b: need 0 < n_aux <= 46340 and 0 < n_bf^2 < 2^30");
  if (!T || !G || !b) return fail(c, RIF_EINVAL, "rif_prepare_b: NULL T, G or b");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_prepare_b(c, nb, na, T, G, delta, b, perm, L, D, nraised);
}

rif_status rif_orbital_step(rif_ctx* c, int nb, int nmo, int nw, const double* lam, const double* eps_in,
                            double* C, double* eps_out, int* info) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(nmo) || !dims_ok(nw) || nw > nmo || nmo > nb)
    return fail(c, RIF_EINVAL, "rif_orbital_step: need 0 < n_omega <= n_mo <= n_bf");
  if (!lam || !C || !eps_out) return fail(c, RIF_EINVAL, "rif_orbital_step: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_orbital_step(c, nb, nmo, nw, lam, eps_in, C, eps_out, info);
}

rif_status rif_set_eigensolver(rif_ctx* c, int kind, int groups) {
  if (!c) return RIF_EINVAL;
  if (kind < RIF_EIG_AUTO || kind > RIF_EIG_DC || groups < 0 || groups > 4096)
    return fail(c, RIF_EINVAL, "rif_set_eigensolver: need kind in {0, 1, 2, 3} and 0 <= groups <= 4096");
  c->eig_kind = kind;
  c->eig_groups = groups;
  return RIF_OK;
}

rif_status rif_set_wait_limit(rif_ctx* c, long long polls) {
  if (!c) return RIF_EINVAL;
  c->wait_limit = polls;
  return RIF_OK;
}

rif_status rif_pnof_optimize(rif_ctx* c, const rif_instance* in, rif_prec prec, rif_functional fn,
                             const rif_opt_params* par, double* C, double* occ, double* gamma, rif_opt_result* res,
                             double* hist_e, double* hist_g, int hist_len) {
  if (!c) return RIF_EINVAL;
  if (!in || !par || !C || !occ || !gamma || !res)
    return fail(c, RIF_EINVAL, "rif_pnof_optimize: NULL instance, params, C, occ, gamma or result");
  rif_instance w = *in;
  w.C = C;
  w.occ = occ;
  rif_status st = check_instance(c, &w, "rif_pnof_optimize", false);
  if (st) return st;
  if (fn != RIF_PNOF7 && fn != RIF_PNOF5) return fail(c, RIF_EINVAL, "rif_pnof_optimize: unknown functional");
  if (in->n_cwo > 14) return fail(c, RIF_EINVAL, "rif_pnof_optimize: the ON optimiser takes n_cwo <= 14");
  if (par->max_outer < 1 || par->max_inner < 1 || par->on_max_it < 0 || !(par->tol_grad > 0.0) ||
      !(par->tol_energy >= 0.0) || !(par->on_tol > 0.0) || (par->init_gamma != 0 && par->init_gamma != 1) ||
      hist_len < 0)
    return fail(c, RIF_EINVAL, "rif_pnof_optimize: need max_outer, max_inner >= 1, on_max_it >= 0, tolerances > 0, "
                               "init_gamma 0 or 1, hist_len >= 0");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_optimize(c, (int)prec, (int)fn, w, *par, C, occ, gamma, res, hist_e, hist_g, hist_len);
}

unsigned long long rif_presplit_b_bytes(int nb, int na, rif_prec prec) {
  if (!dims_ok(nb) || !dims_ok(na)) return 0;
  return presplit_b_bytes(nb, na, (int)prec);
}

rif_status rif_presplit_b(rif_ctx* c, int nb, int na, const double* b, rif_prec prec, void* out) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(na)) return fail(c, RIF_EINVAL, "rif_presplit_b: need n_bf > 0 and n_aux > 0");
  if (!b || !out) return fail(c, RIF_EINVAL, "rif_presplit_b: NULL pointer");
  if (prec != RIF_FP32 && prec != RIF_BF16X3 && prec != RIF_BF16X6 && prec != RIF_FP16X3)
    return fail(c, RIF_ENOTSUP, "rif_presplit_b: FP32, BF16x3, BF16x6 or FP16x3 only");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_presplit_b(c, (int)prec, nb, na, b, out);
}

rif_status rif_build_direct(rif_ctx* c, const rif_instance* in, rif_prec prec, rif_functional fn) {
  if (!c) return RIF_EINVAL;
  rif_status st = check_instance(c, in, "rif_build_direct", false);
  if (st) return st;
  if ((long)in->n_aux * in->n_pairs * (1 + (long)in->n_cwo) >= (1L << 31))
    return fail(c, RIF_EINVAL, "rif_build_direct: need n_aux * n_omega < 2^31");
  if (fn != RIF_PNOF7 && fn != RIF_PNOF5) return fail(c, RIF_EINVAL, "rif_build_direct: unknown functional");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_build_direct(c, (int)prec, (int)fn, *in);
}

unsigned long long rif_eri4_bytes(int nb) {
  if (!dims_ok(nb) || nb > 2048) return 0;
  return eri4_bytes(nb);
}

rif_status rif_eri4_from_b(rif_ctx* c, int nb, int na, const double* b, double* eri) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(na) || nb > 2048 || (long)nb * nb > (1L << 30) || (long)nb * (nb + 1) / 2 >= (1L << 31))
    return fail(c, RIF_EINVAL, "rif_eri4_from_b: need 0 < n_bf <= 2048 and n_aux > 0");
  if (!b || !eri) return fail(c, RIF_EINVAL, "rif_eri4_from_b: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_eri4_from_b(c, nb, na, b, eri);
}

rif_status rif_jk_4c(rif_ctx* c, int nb, int nw, int nmo, const double* eri, const double* C, double* Jn, double* Kn,
                     double* J, double* K) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(nw) || !dims_ok(nmo) || nw > nmo || nmo > nb || nb > 2048)
    return fail(c, RIF_EINVAL, "rif_jk_4c: need 0 < n_omega <= n_mo <= n_bf <= 2048");
  if (!eri || !C || !Jn || !Kn || !J || !K) return fail(c, RIF_EINVAL, "rif_jk_4c: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_jk_4c(c, nb, nw, nmo, eri, C, Jn, Kn, J, K);
}

struct rif_batch {
  rif_ctx* c;
  void* impl;
};

rif_status rif_batch_create(rif_ctx* c, int n, const rif_instance* inst, rif_prec prec, rif_functional fn,
                            rif_batch** out) {
  if (!c) return RIF_EINVAL;
  if (!out || n <= 0 || !inst) return fail(c, RIF_EINVAL, "rif_batch_create: need n_inst > 0, inst and out");
  *out = nullptr;
  if (fn != RIF_PNOF7 && fn != RIF_PNOF5) return fail(c, RIF_EINVAL, "rif_batch_create: unknown functional");
  for (int i = 0; i < n; ++i) {
    rif_status st = check_instance(c, &inst[i], "rif_batch_create");
    if (st) return st;
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  void* impl = nullptr;
  rif_status st = op_batch_create(c, (int)prec, (int)fn, n, inst, &impl);
  if (st) return st;
  *out = new rif_batch{c, impl};
  return RIF_OK;
}

rif_status rif_batch_run(rif_batch* b, int use_graph) {
  if (!b) return RIF_EINVAL;
  if (hipSetDevice(b->c->device) != hipSuccess) return fail(b->c, RIF_EHIP, "hipSetDevice failed");
  return op_batch_run(b->impl, use_graph);
}

void rif_batch_destroy(rif_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->c->device);
  op_batch_destroy(b->impl);
  delete b;
}

rif_status pnof7_energy_grad(rif_ctx* c, int nb, int nmo, int npairs, int ncwo, const int* pair_of,
                             const double* H, const double* C, const double* occ, const double* J,
                             const double* K, const void* Jn, const void* Kn, rif_prec prec, double* energy,
                             double* lambda, double* grad) {
  return pnof_energy_grad(c, RIF_PNOF7, nb, nmo, npairs, ncwo, pair_of, H, C, occ, J, K, Jn, Kn, prec, energy,
                          lambda, grad);
}

long rif_on_work_size(int nw, int npairs, int ncwo) {
  if (nw <= 0 || npairs <= 0 || ncwo <= 0) return 0;
  return on_work_doubles(nw, npairs, ncwo);
}

rif_status rif_hpp(rif_ctx* c, int nb, int nmo, int nw, const double* H, const double* C, double* Hpp) {
  if (!c) return RIF_EINVAL;
  if (!dims_ok(nb) || !dims_ok(nmo) || !dims_ok(nw) || nw > nmo || nmo > nb)
    return fail(c, RIF_EINVAL, "rif_hpp: need 0 < n_omega <= n_mo <= n_bf");
  if (!H || !C || !Hpp) return fail(c, RIF_EINVAL, "rif_hpp: NULL pointer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_hpp(c, nb, nmo, nw, H, C, Hpp);
}

static rif_status check_on(rif_ctx* c, int n, const rif_on_problem* p, bool need_opt, const char* who) {
  if (n <= 0 || !p) return fail(c, RIF_EINVAL, std::string(who) + ": need n_prob > 0 and a problem array");
  for (int i = 0; i < n; ++i) {
    const rif_on_problem& q = p[i];
    if (q.n_pairs <= 0 || q.n_cwo < 1 || q.n_cwo > 14 || q.n_omega != (long)q.n_pairs * (1 + q.n_cwo) || q.row0 < 0)
      return fail(c, RIF_EINVAL, std::string(who) + ": need n_omega = n_pairs (1 + n_cwo), 1 <= n_cwo <= 14");
    if (q.functional != RIF_PNOF7 && q.functional != RIF_PNOF5)
      return fail(c, RIF_EINVAL, std::string(who) + ": unknown functional");
    if (!q.Hpp || !q.J || !q.K) return fail(c, RIF_EINVAL, std::string(who) + ": NULL Hpp/J/K");
    if (need_opt && (!q.gamma || !q.occ || !q.energy || !q.iters || !q.status || !q.work || q.max_it < 0 ||
                     !(q.tol > 0.0)))
      return fail(c, RIF_EINVAL, std::string(who) + ": NULL output/work pointer, max_it < 0 or tol <= 0");
  }
  return RIF_OK;
}

rif_status rif_on_optimize(rif_ctx* c, int n, const rif_on_problem* p) {
  if (!c) return RIF_EINVAL;
  rif_status st = check_on(c, n, p, true, "rif_on_optimize");
  if (st) return st;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_on_optimize(c, n, p);
}

rif_status rif_on_features(rif_ctx* c, int n, const rif_on_problem* p, float* X, float* T, float* M,
                           const float* mu, const float* sigma) {
  if (!c) return RIF_EINVAL;
  rif_status st = check_on(c, n, p, false, "rif_on_features");
  if (st) return st;
  if (!X) return fail(c, RIF_EINVAL, "rif_on_features: NULL X");
  for (int i = 0; i < n; ++i)
    if (T && !p[i].occ) return fail(c, RIF_EINVAL, "rif_on_features: targets need occ");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_on_features(c, n, p, X, T, M, mu, sigma);
}

rif_status rif_on_warmstart(rif_ctx* c, int n, const rif_on_problem* p, const float* P) {
  if (!c) return RIF_EINVAL;
  rif_status st = check_on(c, n, p, false, "rif_on_warmstart");
  if (st) return st;
  for (int i = 0; i < n; ++i)
    if (!p[i].gamma) return fail(c, RIF_EINVAL, "rif_on_warmstart: NULL gamma");
  if (!P) return fail(c, RIF_EINVAL, "rif_on_warmstart: NULL P");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_on_warmstart(c, n, p, P);
}

long rif_mlp_n_params(void) { return mlp_n_params(); }

rif_status rif_mlp_forward(rif_ctx* c, int rows, const float* X, const float* M, const float* theta, float* H,
                           float* Z, float* P) {
  if (!c) return RIF_EINVAL;
  if (rows <= 0 || !X || !M || !theta || !H || !Z || !P) return fail(c, RIF_EINVAL, "rif_mlp_forward: bad arguments");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_mlp_forward(c, rows, X, M, theta, H, Z, P);
}

rif_status rif_mlp_backward(rif_ctx* c, int rows, const float* X, const float* M, const float* T, const float* theta,
                            const float* H, const float* Z, float* dA, float* grad, double* loss) {
  if (!c) return RIF_EINVAL;
  if (rows <= 0 || !X || !M || !T || !theta || !H || !Z || !dA || !grad || !loss)
    return fail(c, RIF_EINVAL, "rif_mlp_backward: bad arguments");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_mlp_backward(c, rows, X, M, T, theta, H, Z, dA, grad, loss);
}

rif_status rif_adam(rif_ctx* c, int n, float* theta, const float* grad, float* m, float* v, int step, float lr,
                    float b1, float b2, float eps) {
  if (!c) return RIF_EINVAL;
  if (n <= 0 || step < 1 || !theta || !grad || !m || !v) return fail(c, RIF_EINVAL, "rif_adam: bad arguments");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, RIF_EHIP, "hipSetDevice failed");
  return op_adam(c, n, theta, grad, m, v, step, lr, b1, b2, eps);
}

rif_status rif_autotune(rif_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 1) return RIF_EINVAL;
  c->tune_mode = mode;
  return RIF_OK;
}

rif_status rif_set_tile_variant(rif_ctx* c, int v) {
  if (!c || v < -1 || v > 3) return RIF_EINVAL;
  c->force_variant = v;
  return RIF_OK;
}

rif_status rif_tune_report(rif_ctx* c, char* buf, int len) {
  if (!c || !buf || len <= 0) return RIF_EINVAL;
  std::string s;
  for (auto& t : c->tune) {
    s += t.key + " -> " + std::to_string(t.variant) + " |";
    char x[32];
    for (float ms : t.ms) {
      snprintf(x, sizeof x, " %.4f", ms);
      s += x;
    }
    s += "\n";
  }
  strncpy(buf, s.c_str(), (size_t)len - 1);
  buf[len - 1] = 0;
  return RIF_OK;
}

rif_status rif_tune_load(rif_ctx* c, const char* text) {
  if (!c) return RIF_EINVAL;
  if (!text) return fail(c, RIF_EINVAL, "rif_tune_load: NULL text");
  std::vector<rif_ctx::Tune> add;
  int ln = 0;
  for (const char* p = text; *p;) {
    const char* e = strchr(p, '\n');
    const std::string line(p, e ? (size_t)(e - p) : strlen(p));
    p = e ? e + 1 : p + line.size();
    ++ln;
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    auto bad = [&]() { return fail(c, RIF_EINVAL, "rif_tune_load: line " + std::to_string(ln) + " does not parse"); };
    const size_t arrow = line.find(" -> ");
    if (arrow == std::string::npos || arrow == 0) return bad();
    const size_t bar = line.find(" |", arrow + 4);
    if (bar == std::string::npos) return bad();
    const std::string vs = line.substr(arrow + 4, bar - arrow - 4);
    char* end = nullptr;
    const long v = strtol(vs.c_str(), &end, 10);
    if (vs.empty() || *end != '\0' || v < 0) return bad();
    rif_ctx::Tune t{line.substr(0, arrow), (int)v, {}};
    const char* q = line.c_str() + bar + 2;
    while (*q) {
      while (*q == ' ' || *q == '\t' || *q == '\r') ++q;
      if (!*q) break;
      const float ms = strtof(q, &end);
      if (end == q) return bad();
      t.ms.push_back(ms);
      q = end;
    }
    if (t.ms.empty() || (size_t)v >= t.ms.size()) return bad();
    add.push_back(std::move(t));
  }
  for (auto& t : add) {
    bool found = false;
    for (auto& u : c->tune)
      if (u.key == t.key) {
        u = t;
        found = true;
      }
    if (!found) c->tune.push_back(t);
  }
  return RIF_OK;
}

rif_status rif_profile_enable(rif_ctx* c, int on) {
  if (!c) return RIF_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
  for (auto& e : c->evs) {
    c->pool.push_back(e.a);
    c->pool.push_back(e.b);
  }
  c->evs.clear();
  c->totals.clear();
  c->prof = on != 0;
  return RIF_OK;
}

rif_status rif_profile_only(rif_ctx* c, const char* name) {
  if (!c) return RIF_EINVAL;
  c->prof_only = name ? name : "";
  return RIF_OK;
}

rif_status rif_profile_report(rif_ctx* c, char* buf, int len) {
  if (!c || !buf || len <= 0) return RIF_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
  for (auto& e : c->evs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) ms = 0.f;
    auto it = std::find_if(c->totals.begin(), c->totals.end(), [&](const rif_ctx::Tot& t) { return t.name == e.name; });
    if (it == c->totals.end()) c->totals.push_back({e.name, 1, (double)ms});
    else { it->launches += 1; it->ms += ms; }
    c->pool.push_back(e.a);
    c->pool.push_back(e.b);
  }
  c->evs.clear();
  std::string s;
  char line[160];
  for (auto& t : c->totals) {
    snprintf(line, sizeof line, "%s %ld %.6f\n", t.name.c_str(), t.launches, t.ms);
    s += line;
  }
  strncpy(buf, s.c_str(), (size_t)len - 1);
  buf[len - 1] = 0;
  return RIF_OK;
}

}  // extern "C"
