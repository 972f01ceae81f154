// Host-side check of the C ABI's argument validation, built with the host
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_abi_host_sanitized.py).
// Every call below carries an invalid argument, so it must return its error
// status, with a message, before any GPU work: the program runs on a machine
// without a GPU and never creates a real context.  The context used here is a
// plain host object with no stream, workspace or device memory.
#include <limits.h>
#include <stdio.h>
#include <string.h>

#include "rif_internal.hpp"

static int n_fail = 0, n_call = 0;

static void expect(const char* what, rif_status got, rif_status want, const rif_ctx* c) {
  ++n_call;
  if (got != want) {
    printf("FAIL %s: status %d, want %d\n", what, (int)got, (int)want);
    ++n_fail;
  } else if (c && want != RIF_OK && rif_last_error(c)[0] == '\0') {
    printf("FAIL %s: no error message\n", what);
    ++n_fail;
  }
}
#define EXPECT(call, want) expect(#call, (call), (want), c)

static rif_instance good_instance(double* p, int* ip) {
  rif_instance in;
  memset(&in, 0, sizeof(in));
  in.n_bf = 40; in.n_aux = 100; in.n_pairs = 3; in.n_cwo = 2; in.n_mo = 30;
  in.b = in.C = in.H = in.occ = p;
  in.pair_of = ip;
  in.b_half = in.b_mo = in.Jn = in.Kn = p;
  in.d = in.J = in.K = in.energy = in.lambda = in.grad = p;
  return in;
}

int main() {
  rif_ctx ctx;
  rif_ctx* c = &ctx;
  double buf[16] = {0};
  double* p = buf;
  int ibuf[16] = {0};
  float fbuf[16] = {0};

  // no context
  {
    rif_ctx* c = nullptr;
    EXPECT(rif_transform(nullptr, 10, 10, 5, 5, p, p, RIF_FP64, p, p, p), RIF_EINVAL);
    EXPECT(rif_build(nullptr, nullptr, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    EXPECT(rif_create(nullptr, 0, nullptr), RIF_EINVAL);
    if (strcmp(rif_last_error(nullptr), "null context") != 0) { printf("FAIL rif_last_error(NULL)\n"); ++n_fail; }
  }
  // dimensions: zero, negative, too large, inconsistent
  EXPECT(rif_transform(c, 0, 10, 5, 5, p, p, RIF_FP64, p, p, p), RIF_EINVAL);
  EXPECT(rif_transform(c, 10, -1, 5, 5, p, p, RIF_FP64, p, p, p), RIF_EINVAL);
  EXPECT(rif_transform(c, 10, 10, 6, 5, p, p, RIF_FP64, p, p, p), RIF_EINVAL);      // n_omega > n_mo
  EXPECT(rif_transform(c, 10, 10, 5, 11, p, p, RIF_FP64, p, p, p), RIF_EINVAL);     // n_mo > n_bf
  EXPECT(rif_transform(c, INT_MAX, 10, 5, 5, p, p, RIF_FP64, p, p, p), RIF_EINVAL);
  EXPECT(rif_transform(c, 10, 10, 5, 5, nullptr, p, RIF_FP64, p, p, p), RIF_EINVAL);
  EXPECT(rif_jk_mo(c, 0, 5, p, p, RIF_FP64, p, p), RIF_EINVAL);
  EXPECT(rif_jk_mo(c, 10, 5, nullptr, p, RIF_FP64, p, p), RIF_EINVAL);
  EXPECT(rif_jk_mo_noalloc(c, 10, INT_MIN, p, p, RIF_FP64, p, p), RIF_EINVAL);
  EXPECT(rif_jk_mo_noalloc(c, 10, 5, p, p, RIF_FP64, p, nullptr), RIF_EINVAL);
  EXPECT(rif_jk_ao_per_mo(c, 10, 10, 11, p, p, p, RIF_FP64, p, p), RIF_EINVAL);     // n_omega > n_bf
  EXPECT(rif_jk_ao_per_mo(c, 10, 10, 5, p, p, p, RIF_FP64, nullptr, p), RIF_EINVAL);
  // energy and gradient
  EXPECT(pnof_energy_grad(c, (rif_functional)7, 10, 10, 2, 1, nullptr, p, p, p, p, p, p, p, RIF_FP64, p, p, p),
         RIF_EINVAL);
  EXPECT(pnof_energy_grad(c, RIF_PNOF7, 10, 10, 2, 0, nullptr, p, p, p, p, p, p, p, RIF_FP64, p, p, p), RIF_EINVAL);
  EXPECT(pnof_energy_grad(c, RIF_PNOF7, 10, 10, 2, INT_MAX, nullptr, p, p, p, p, p, p, p, RIF_FP64, p, p, p),
         RIF_EINVAL);
  EXPECT(pnof_energy_grad(c, RIF_PNOF7, 10, 10, 4, 2, nullptr, p, p, p, p, p, p, p, RIF_FP64, p, p, p),
         RIF_EINVAL);   // n_pairs (1 + n_cwo) = 12 > n_mo
  EXPECT(pnof7_energy_grad(c, 10, 10, 2, 1, nullptr, p, p, p, p, p, p, p, RIF_FP64, nullptr, p, p), RIF_EINVAL);
  // whole builds: instance checks
  {
    rif_instance in = good_instance(p, ibuf);
    EXPECT(rif_build(c, nullptr, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    in.n_cwo = INT_MAX;   // n_pairs (1 + n_cwo) must not overflow
    EXPECT(rif_build(c, &in, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    EXPECT(rif_build_direct(c, &in, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    in = good_instance(p, ibuf);
    in.n_pairs = INT_MAX;
    EXPECT(rif_build(c, &in, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    in = good_instance(p, ibuf);
    in.Kn = nullptr;
    EXPECT(rif_build(c, &in, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    in = good_instance(p, ibuf);
    EXPECT(rif_build(c, &in, RIF_FP64, (rif_functional)9), RIF_EINVAL);
    EXPECT(rif_build_direct(c, &in, RIF_FP64, (rif_functional)9), RIF_EINVAL);
    in.n_aux = 1 << 29; in.n_pairs = 12; in.n_cwo = 2; in.n_mo = 36; in.n_bf = 40;   // n_aux n_omega >= 2^31
    EXPECT(rif_build_direct(c, &in, RIF_FP64, RIF_PNOF7), RIF_EINVAL);
    rif_batch* bt = nullptr;
    in = good_instance(p, ibuf);
    EXPECT(rif_batch_create(c, 0, &in, RIF_FP64, RIF_PNOF7, &bt), RIF_EINVAL);
    EXPECT(rif_batch_create(c, 1, nullptr, RIF_FP64, RIF_PNOF7, &bt), RIF_EINVAL);
    rif_instance two[2] = {good_instance(p, ibuf), good_instance(p, ibuf)};
    two[1].n_mo = 41;   // second instance bad
    EXPECT(rif_batch_create(c, 2, two, RIF_FP64, RIF_PNOF7, &bt), RIF_EINVAL);
    if (bt) { printf("FAIL rif_batch_create left a handle\n"); ++n_fail; }
    EXPECT(rif_batch_run(nullptr, 0), RIF_EINVAL);
    rif_batch_destroy(nullptr);
  }
  // pre-split b and its size
  if (rif_presplit_b_bytes(0, 10, RIF_BF16X3) != 0 || rif_presplit_b_bytes(10, -3, RIF_BF16X3) != 0) {
    printf("FAIL rif_presplit_b_bytes accepts bad sizes\n");
    ++n_fail;
  }
  EXPECT(rif_presplit_b(c, 10, 10, p, RIF_FP64, p), RIF_ENOTSUP);
  EXPECT(rif_presplit_b(c, 10, 10, nullptr, RIF_BF16X3, p), RIF_EINVAL);
  EXPECT(rif_presplit_b(c, 10, 0, p, RIF_BF16X3, p), RIF_EINVAL);
  // four-centre path
  if (rif_eri4_bytes(0) != 0 || rif_eri4_bytes(4096) != 0 || rif_eri4_bytes(8) != 36ull * 64 * 8) {
    printf("FAIL rif_eri4_bytes\n");
    ++n_fail;
  }
  EXPECT(rif_eri4_from_b(c, 4096, 10, p, p), RIF_EINVAL);
  EXPECT(rif_eri4_from_b(c, 10, 10, p, nullptr), RIF_EINVAL);
  EXPECT(rif_jk_4c(c, 10, 11, 10, p, p, p, p, p, p), RIF_EINVAL);
  EXPECT(rif_jk_4c(c, 10, 5, 10, nullptr, p, p, p, p, p), RIF_EINVAL);
  // b preparation, orbital step, eigensolver choice, optimiser
  EXPECT(rif_prepare_b(c, 10, 46341, p, p, 0.0, p, ibuf, p, p, ibuf), RIF_EINVAL);
  EXPECT(rif_prepare_b(c, 40000, 10, p, p, 0.0, p, ibuf, p, p, ibuf), RIF_EINVAL);   // n_bf^2 > 2^30
  EXPECT(rif_prepare_b(c, 10, 10, nullptr, p, 0.0, p, ibuf, p, p, ibuf), RIF_EINVAL);
  EXPECT(rif_orbital_step(c, 10, 10, 11, p, p, p, p, ibuf), RIF_EINVAL);
  EXPECT(rif_orbital_step(c, 10, 10, 5, p, p, nullptr, p, ibuf), RIF_EINVAL);
  EXPECT(rif_set_eigensolver(c, 4, 0), RIF_EINVAL);
  EXPECT(rif_set_eigensolver(c, 3, 0), RIF_OK);
  EXPECT(rif_set_eigensolver(c, 1, 5000), RIF_EINVAL);
  EXPECT(rif_set_eigensolver(c, 2, 64), RIF_OK);
  {
    rif_instance in = good_instance(p, ibuf);
    rif_opt_params par;
    memset(&par, 0, sizeof(par));
    par.max_outer = 1; par.max_inner = 1; par.tol_grad = 1e-6; par.on_tol = 1e-8;
    rif_opt_result res;
    EXPECT(rif_pnof_optimize(c, &in, RIF_FP64, RIF_PNOF7, nullptr, p, p, p, &res, nullptr, nullptr, 0), RIF_EINVAL);
    in.n_cwo = 15; in.n_pairs = 1; in.n_mo = 16; in.n_bf = 40;
    EXPECT(rif_pnof_optimize(c, &in, RIF_FP64, RIF_PNOF7, &par, p, p, p, &res, nullptr, nullptr, 0), RIF_EINVAL);
    in = good_instance(p, ibuf);
    par.tol_grad = -1.0;
    EXPECT(rif_pnof_optimize(c, &in, RIF_FP64, RIF_PNOF7, &par, p, p, p, &res, nullptr, nullptr, 0), RIF_EINVAL);
    par.tol_grad = 1e-6;
    EXPECT(rif_pnof_optimize(c, &in, RIF_FP64, RIF_PNOF7, &par, p, p, p, &res, nullptr, nullptr, -1), RIF_EINVAL);
  }
  // ON optimiser and learned warm start
  EXPECT(rif_on_optimize(c, 0, nullptr), RIF_EINVAL);
  {
    rif_on_problem q;
    memset(&q, 0, sizeof(q));
    q.n_pairs = INT_MAX / 2; q.n_cwo = 14; q.n_omega = 15;   // n_pairs (1 + n_cwo) must not overflow
    q.Hpp = q.J = q.K = p;
    EXPECT(rif_on_optimize(c, 1, &q), RIF_EINVAL);
    q.n_pairs = 1; q.n_cwo = 15; q.n_omega = 16;   // the optimiser takes n_cwo <= 14
    EXPECT(rif_on_optimize(c, 1, &q), RIF_EINVAL);
    q.n_cwo = 2; q.n_omega = 3;
    q.functional = 5;
    EXPECT(rif_on_features(c, 1, &q, fbuf, nullptr, nullptr, nullptr, nullptr), RIF_EINVAL);
    if (rif_on_work_size(3, 1, 2) <= 0 || rif_on_work_size(0, 1, 2) != 0) {
      printf("FAIL rif_on_work_size\n");
      ++n_fail;
    }
  }
  EXPECT(rif_hpp(c, 10, 10, 11, p, p, p), RIF_EINVAL);
  EXPECT(rif_on_warmstart(c, 1, nullptr, fbuf), RIF_EINVAL);
  EXPECT(rif_mlp_forward(c, 0, fbuf, fbuf, fbuf, fbuf, fbuf, fbuf), RIF_EINVAL);
  EXPECT(rif_adam(c, -1, fbuf, fbuf, fbuf, fbuf, 1, 1e-3f, 0.9f, 0.999f, 1e-8f), RIF_EINVAL);
  // settings that need no GPU (status only: these report no message)
  expect("rif_set_tile_variant(c, 7)", rif_set_tile_variant(c, 7), RIF_EINVAL, nullptr);
  expect("rif_set_tile_variant(c, -1)", rif_set_tile_variant(c, -1), RIF_OK, nullptr);
  expect("rif_autotune(c, 5)", rif_autotune(c, 5), RIF_EINVAL, nullptr);
  expect("rif_tune_report(c, NULL, 10)", rif_tune_report(c, nullptr, 10), RIF_EINVAL, nullptr);
  expect("rif_set_workspace_limit", rif_set_workspace_limit(c, 1ull << 40), RIF_OK, nullptr);
  // tile choices loaded from a report: parse errors load nothing; a good text
  // round-trips through rif_tune_report, and a later line replaces its shape
  EXPECT(rif_tune_load(c, nullptr), RIF_EINVAL);
  EXPECT(rif_tune_load(c, "half 1 2 -> x | 0.1"), RIF_EINVAL);
  EXPECT(rif_tune_load(c, "half 1 2 -> 3 | 0.1 0.2"), RIF_EINVAL);       // no variant 3 among two
  EXPECT(rif_tune_load(c, "mo 3 -> 0 | 0.1\nhalf 1 2 0.5"), RIF_EINVAL);  // second line has no arrow
  EXPECT(rif_tune_load(c, "half 1 2 -> 1 | 0.5 0.25\n\nmo 3 -> 0 | 0.1\n"), RIF_OK);
  EXPECT(rif_tune_load(c, "half 1 2 -> 0 | 0.5 0.25"), RIF_OK);
  {
    char rep[256];
    ++n_call;
    if (rif_tune_report(c, rep, sizeof rep) != RIF_OK ||
        strcmp(rep, "half 1 2 -> 0 | 0.5000 0.2500\nmo 3 -> 0 | 0.1000\n") != 0) {
      printf("FAIL rif_tune_load round trip: %s\n", rep);
      ++n_fail;
    }
  }

  printf("%d calls, %d failures\n", n_call, n_fail);
  return n_fail ? 1 : 0;
}
