// Orbital optimisation with RI (Sec. II) and the outer/inner scheme of Fig. 1.
//
//   k_flam       F^lambda from the Lagrange multipliers (reading below)
//   k_transpose  64x64 LDS-tiled transpose (FP64)
//   k_maxabs     max |x| over an array, NaN counted as +inf (two passes)
//   op_orbital_step   F^lambda -> eigenvectors -> C <- C V.  Eigensolver: the
//                     one-launch tridiagonal reduction forming Q (eig.hip),
//                     divide and conquer on T (tdc.hip, or rocSOLVER dstedc),
//                     and C <- (C Q) Z as two GEMMs; or rocSOLVER dsyevd
//                     throughout (rif_set_eigensolver)
//   op_optimize       ON optimisation at fixed orbitals, then inner iterations
//                     (build -> max|G| -> orbital step) at fixed ONs, repeated;
//                     the builds skip J^q/K^q when no Jn/Kn buffers are given
//
// F^lambda is not printed in the paper; the reading (from the iterative
// diagonalisation work it cites): off the diagonal
//   F_pq = lambda_{hi,lo} - lambda_{lo,hi},  hi = max(p,q), lo = min(p,q),
// with lambda_ab = c_a^T F^(b) c_b (zero for b outside Omega), so F is
// symmetric and vanishes off the diagonal exactly when the orbital gradient
// G = 4 (lambda - lambda^T) does.  The diagonal is lambda_pp at the first step
// of an inner loop and the previous step's eigenvalues afterwards (aufbau
// order: eigenvectors in ascending eigenvalue order, orbital roles by index).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rif_internal.hpp"

namespace rif {

__global__ __launch_bounds__(256) void k_flam(int n, int nw, const double* __restrict__ lam,
                                              const double* __restrict__ eps, double* __restrict__ F) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)n * n) return;
  const int p = (int)(i / n), q = (int)(i - (long)p * n);
  auto L = [&](int a, int b) { return b < nw ? lam[(long)a * nw + b] : 0.0; };
  double v;
  if (p == q) {
    v = eps ? eps[p] : L(p, p);
  } else {
    const int hi = p > q ? p : q, lo = p > q ? q : p;
    v = L(hi, lo) - L(lo, hi);
  }
  F[i] = v;
}

// out[c][r] = in[r][c] for an R x Cn matrix; both sides coalesced through LDS.
__global__ __launch_bounds__(256) void k_transpose(int R, int Cn, const double* __restrict__ in, long ldi,
                                                   double* __restrict__ out, long ldo) {
  __shared__ double t[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int r = r0 + y, c = c0 + tx;
    if (r < R && c < Cn) t[y][tx] = in[(long)r * ldi + c];
  }
  __syncthreads();
  for (int y = ty; y < 64; y += 4) {
    const int c = c0 + y, r = r0 + tx;
    if (c < Cn && r < R) out[(long)c * ldo + r] = t[tx][y];
  }
}

// max |x|: each of up to kMaxBlocks workgroups writes the max of its strided
// share, then one workgroup takes the max of those (max is order-free).
constexpr int kMaxBlocks = 256;
__global__ __launch_bounds__(256) void k_maxabs(long n, const double* __restrict__ x, double* __restrict__ part,
                                                double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  if (x) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
      const double v = x[i];
      m = (v != v) ? INFINITY : fmax(m, fabs(v));
    }
  } else {
    for (int i = threadIdx.x; i < (int)n; i += 256) m = fmax(m, part[i]);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) (x ? part[blockIdx.x] : out[0]) = red[0];
}

static rif_status blas_handle(rif_ctx* c, rocblas_handle* h) {
  if (!c->blas) {
    rocblas_handle nh = nullptr;
    if (rocblas_create_handle(&nh) != rocblas_status_success)
      return fail(c, RIF_EHIP, "rocblas_create_handle failed");
    c->blas = nh;
  }
  *h = (rocblas_handle)c->blas;
  if (rocblas_set_stream(*h, c->stream) != rocblas_status_success)
    return fail(c, RIF_EHIP, "rocblas_set_stream failed");
  return RIF_OK;
}

void op_orbital_release(rif_ctx* c) {
  if (c->blas) rocblas_destroy_handle((rocblas_handle)c->blas);
  c->blas = nullptr;
}

static rif_status transpose(rif_ctx* c, int R, int Cn, const double* in, long ldi, double* out, long ldo) {
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((Cn + 63) / 64), (unsigned)((R + 63) / 64)), dim3(256), 0,
                     c->stream, R, Cn, in, ldi, out, ldo);
  return check_launch(c, "transpose");
}

rif_status op_maxabs(rif_ctx* c, long n, const double* x, double* part, double* out) {
  const int nblk = (int)std::min((long)kMaxBlocks, std::max(1L, (n + 2047) / 2048));
  hipLaunchKernelGGL(k_maxabs, dim3(nblk), dim3(256), 0, c->stream, n, x, part, out);
  hipLaunchKernelGGL(k_maxabs, dim3(1), dim3(256), 0, c->stream, (long)nblk, (const double*)nullptr, part, out);
  return check_launch(c, "maxabs");
}

__global__ void k_trd_info(const int* err, int* info) {
  if (threadIdx.x == 0 && *err != 0) *info = -1;
}
// own divide and conquer: -1 for a timed-out wait of the reduction, 1 for a
// non-finite T or a leaf that did not converge, else 0
__global__ void k_tdc_info(const int* err_trd, const int* err_dc, int* info) {
  if (threadIdx.x == 0) *info = *err_trd != 0 ? -1 : (*err_dc != 0 ? 1 : 0);
}

rif_status op_orbital_step(rif_ctx* c, int nb, int nmo, int nw, const double* lam, const double* eps_in,
                           double* C, double* eps_out, int* info) {
  const int n = nmo;
  // eigensolver: own tridiagonal reduction (forming Q), then own divide and
  // conquer (AUTO, DC) or rocSOLVER dstedc (TRD); or rocSOLVER dsyevd
  const int kind = c->eig_kind;
  const int G = kind == RIF_EIG_SYEVD || n > tdc_max_n() ? 0 : trd_groups(c, n, c->eig_groups);
  if ((kind == RIF_EIG_TRD || kind == RIF_EIG_DC) && G == 0)
    return fail(c, RIF_ENOTSUP, "tridiagonal reduction: n_mo does not fit the cooperative launch");
  const bool trd = G > 0;
  const bool own = trd && kind != RIF_EIG_TRD;
  rocblas_handle h = nullptr;
  rif_status st;
  if (!own && (st = blas_handle(c, &h))) return st;
  Carve cv;
  const size_t oF = cv.take<double>((size_t)n * n), oV = cv.take<double>((size_t)n * n);
  const size_t oCt = cv.take<double>((size_t)nb * n), oE = cv.take<double>((size_t)n), oI = cv.take<int>(1);
  size_t oQ = 0, oWt = 0, oS = 0, oErr = 0, oZ1 = 0, oDc = 0, oErrDc = 0;
  if (trd) {
    oQ = cv.take<double>((size_t)n * n);
    oWt = cv.take<double>((size_t)n * nb);
    oS = cv.take<char>(trd_scratch_bytes(n));
    oErr = cv.take<int>(1);
  }
  if (own) {
    oZ1 = cv.take<double>((size_t)n * n);
    oDc = cv.take<char>(tdc_scratch_bytes(n));
    oErrDc = cv.take<int>(1);
  }
  if ((st = ws_reserve(c, cv.off))) return st;
  auto at = [&](size_t o) { return (char*)c->ws + o; };
  int* dinfo = info ? info : (int*)at(oI);
  if (own) {
    double *F = (double*)at(oF), *E = (double*)at(oE);
    {
      ProfScope ps(c, "flam");
      hipLaunchKernelGGL(k_flam, dim3((unsigned)(((long)n * n + 255) / 256)), dim3(256), 0, c->stream, n, nw, lam,
                         eps_in, F);
      if ((st = check_launch(c, "flam"))) return st;
    }
    {
      ProfScope ps(c, "tridiagonal");
      if ((st = op_trd(c, n, G, F, (double*)at(oQ), eps_out, E, at(oS), (int*)at(oErr)))) return st;
    }
    {
      ProfScope ps(c, "eigensolver");
      // rows of F become the eigenvectors of T
      if ((st = op_tdc(c, n, eps_out, E, F, (double*)at(oZ1), at(oDc), (int*)at(oErrDc)))) return st;
      hipLaunchKernelGGL(k_tdc_info, dim3(1), dim3(64), 0, c->stream, (const int*)at(oErr), (const int*)at(oErrDc),
                         dinfo);
      if ((st = check_launch(c, "tdc_info"))) return st;
    }
    ProfScope ps(c, "rotate");
    double *V = (double*)at(oV), *Ct = (double*)at(oCt), *Wt = (double*)at(oWt);
    if ((st = transpose(c, n, n, F, n, V, n))) return st;
    if ((st = transpose(c, nb, n, C, n, Ct, nb))) return st;
    if ((st = op_gemm_kn(c, n, nb, n, (const double*)at(oQ), n, Ct, nb, Wt, nb))) return st;
    return op_gemm_kn(c, nb, n, n, Wt, nb, V, n, C, n);
  }
  // F is symmetric, so its row-major array is also its column-major one.  On
  // return, column j of the column-major F is eigenvector j of F (dsyevd) or
  // of T (dstedc, eigenvalues into eps_out, which holds T's diagonal).
  auto solve = [&](double* F, double* E) -> rocblas_status {
    if (trd) return rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, eps_out, E, F, n, dinfo);
    return rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, F, n, eps_out, E, dinfo);
  };
  // solver workspace: size query (host only), then carve it after the buffers above
  size_t wsz = 0;
  if (rocblas_start_device_memory_size_query(h) != rocblas_status_success)
    return fail(c, RIF_EHIP, "rocBLAS workspace size query failed");
  solve((double*)at(oF), (double*)at(oE));
  if (rocblas_stop_device_memory_size_query(h, &wsz) != rocblas_status_success)
    return fail(c, RIF_EHIP, "rocBLAS workspace size query failed");
  const size_t oW = cv.take<char>(wsz + 256);
  if ((st = ws_reserve(c, cv.off))) return st;   // may move the arena: addresses taken below
  double *F = (double*)at(oF), *V = (double*)at(oV), *Ct = (double*)at(oCt), *E = (double*)at(oE);
  if (!info) dinfo = (int*)at(oI);
  {
    ProfScope ps(c, "flam");
    hipLaunchKernelGGL(k_flam, dim3((unsigned)(((long)n * n + 255) / 256)), dim3(256), 0, c->stream, n, nw, lam,
                       eps_in, F);
    if ((st = check_launch(c, "flam"))) return st;
  }
  if (trd) {
    ProfScope ps(c, "tridiagonal");
    // T's diagonal goes straight to eps_out (k_flam has read eps_in, which may be the same array)
    if ((st = op_trd(c, n, G, F, (double*)at(oQ), eps_out, E, at(oS), (int*)at(oErr)))) return st;
  }
  {
    ProfScope ps(c, "eigensolver");
    if (rocblas_set_workspace(h, at(oW), wsz + 256) != rocblas_status_success)
      return fail(c, RIF_EHIP, "rocblas_set_workspace failed");
    const rocblas_status rs = solve(F, E);
    if (rs != rocblas_status_success)
      return fail(c, RIF_EHIP, std::string(trd ? "rocsolver_dstedc" : "rocsolver_dsyevd") + " failed (status " +
                                   std::to_string((int)rs) + ")");
    if (trd) {   // a timed-out wait inside the reduction reports as info = -1
      hipLaunchKernelGGL(k_trd_info, dim3(1), dim3(64), 0, c->stream, (const int*)at(oErr), dinfo);
      if ((st = check_launch(c, "trd_info"))) return st;
    }
  }
  ProfScope ps(c, "rotate");
  // V[i][j] = component i of eigenvector j (row-major), Ct = C^T
  if ((st = transpose(c, n, n, F, n, V, n))) return st;
  if ((st = transpose(c, nb, n, C, n, Ct, nb))) return st;
  if (!trd)   // C[mu][j] = sum_i Ct[i][mu] V[i][j]
    return op_gemm_kn(c, nb, n, n, Ct, nb, V, n, C, n);
  // eigenvectors of F are Q V: first Wt = (C Q)^T, Wt[c][mu] = sum_i Q[i][c] Ct[i][mu],
  // then C[mu][j] = sum_c Wt[c][mu] V[c][j]
  double* Wt = (double*)at(oWt);
  if ((st = op_gemm_kn(c, n, nb, n, (const double*)at(oQ), n, Ct, nb, Wt, nb))) return st;
  return op_gemm_kn(c, nb, n, n, Wt, nb, V, n, C, n);
}

// ---- the outer/inner loop ------------------------------------------------------

namespace {
struct DevBlock {   // loop state: its own allocation, since every op carves the arena from its start
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~DevBlock() {   // an error return may leave kernels that use it in the queue
    if (!p) return;
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
  }
};
struct HostBlock {
  void* p = nullptr;
  ~HostBlock() {
    if (p) (void)hipHostFree(p);
  }
};
struct Events {
  hipEvent_t e[6] = {};
  ~Events() {
    for (auto x : e)
      if (x) (void)hipEventDestroy(x);
  }
};
}  // namespace

rif_status op_optimize(rif_ctx* c, int prec, int fn, const rif_instance& in0, const rif_opt_params& par, double* C,
                       double* occ, double* gamma, rif_opt_result* res, double* hist_e, double* hist_g,
                       int hist_len) {
  rif_instance in = in0;
  in.C = C;
  in.occ = occ;
  const int nb = in.n_bf, na = in.n_aux, nmo = in.n_mo, np_ = in.n_pairs, nc = in.n_cwo;
  const int nw = np_ * (1 + nc);
  *res = rif_opt_result{};
  res->status = 1;

  Carve cv;
  const size_t oHpp = cv.take<double>(nw), oEps = cv.take<double>(nmo), oEon = cv.take<double>(1);
  const size_t oWork = cv.take<double>((size_t)on_work_doubles(nw, np_, nc));
  const size_t oX = cv.take<float>((size_t)np_ * 39), oT = cv.take<float>((size_t)np_ * 7);
  const size_t oGmax = cv.take<double>(1), oInfo = cv.take<int>(1), oIt = cv.take<int>(1), oSt = cv.take<int>(1);
  const size_t oPart = cv.take<double>(kMaxBlocks);
  DevBlock dev;
  dev.s = c->stream;
  if (hipMalloc(&dev.p, cv.off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, RIF_ENOMEM, "hipMalloc of the optimisation state failed");
  }
  auto D = [&](size_t o) { return (char*)dev.p + o; };
  double *Hpp = (double*)D(oHpp), *eps = (double*)D(oEps), *gmax = (double*)D(oGmax);
  int* info = (int*)D(oInfo);
  struct Stage { double gmax, energy; int info, on_iters, on_status; };
  HostBlock hb;
  if (hipHostMalloc(&hb.p, sizeof(Stage)) != hipSuccess) return fail(c, RIF_ENOMEM, "hipHostMalloc failed");
  Stage* hs = (Stage*)hb.p;
  if (hipMemsetAsync(info, 0, sizeof(int), c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipMemsetAsync failed");

  rif_on_problem prob{};
  prob.n_pairs = np_; prob.n_cwo = nc; prob.n_omega = nw; prob.functional = fn; prob.max_it = par.on_max_it;
  prob.row0 = 0; prob.tol = par.on_tol; prob.Hpp = Hpp; prob.J = in.J; prob.K = in.K; prob.pair_of = in.pair_of;
  prob.gamma = gamma; prob.occ = occ; prob.energy = (double*)D(oEon); prob.iters = (int*)D(oIt);
  prob.status = (int*)D(oSt); prob.work = (double*)D(oWork);

  Events ev;
  for (auto& e : ev.e)
    if (hipEventCreate(&e) != hipSuccess) return fail(c, RIF_EHIP, "hipEventCreate failed");
  auto lap = [&](hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return (double)ms;
  };
  auto pull = [&](const double* energy) -> rif_status {
    if (hipMemcpyAsync(&hs->gmax, gmax, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&hs->energy, energy, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&hs->info, info, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fail(c, RIF_EHIP, "reading the iteration state failed");
    return RIF_OK;
  };

  rif_status st;
  double e_prev = 0.0;
  int n_hist = 0;
  for (int outer = 0; outer < par.max_outer; ++outer) {
    // ON optimisation at the current orbitals: J, K (MO) and H_pp, then L-BFGS in gamma
    hipEventRecord(ev.e[0], c->stream);
    if ((st = op_transform(c, prec, nb, na, nw, nmo, in.b, C, in.b_half, in.b_mo, in.d))) return st;
    if ((st = op_jk_mo(c, prec, na, nw, in.b_mo, in.d, in.J, in.K))) return st;
    if ((st = op_hpp(c, nb, nmo, nw, in.H, C, Hpp))) return st;
    if (outer == 0 && par.init_gamma == 0) {   // gamma from the starting ONs
      if ((st = op_on_features(c, 1, &prob, (float*)D(oX), (float*)D(oT), nullptr, nullptr, nullptr))) return st;
      if ((st = op_on_warmstart(c, 1, &prob, (const float*)D(oT)))) return st;
    }
    if ((st = op_on_optimize(c, 1, &prob))) return st;
    hipEventRecord(ev.e[1], c->stream);
    if (hipMemcpyAsync(&hs->on_iters, prob.iters, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&hs->on_status, prob.status, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fail(c, RIF_EHIP, "reading the ON step state failed");
    res->ms_on += lap(ev.e[0], ev.e[1]);
    res->on_iters_total += hs->on_iters;
    res->on_status = hs->on_status;

    // inner iterations at the new ONs
    bool inner_ok = false, have_step = false;
    for (int inner = 0; inner < par.max_inner; ++inner) {
      hipEventRecord(ev.e[2], c->stream);
      if ((st = (in.Jn && in.Kn) ? op_build(c, prec, fn, in) : op_build_direct(c, prec, fn, in))) return st;
      if ((st = op_maxabs(c, (long)nmo * nmo, in.grad, (double*)D(oPart), gmax))) return st;
      hipEventRecord(ev.e[3], c->stream);
      if ((st = pull(in.energy))) return st;
      res->ms_build += lap(ev.e[2], ev.e[3]);
      if (have_step) res->ms_orbital += lap(ev.e[4], ev.e[5]);
      if (hs->info != 0) {
        res->status = 2;
        return fail(c, RIF_EHIP, "eigensolver did not converge (info " + std::to_string(hs->info) + ")");
      }
      res->inner_total++;
      res->energy = hs->energy;
      res->max_grad = hs->gmax;
      if (n_hist < hist_len) {
        if (hist_e) hist_e[n_hist] = hs->energy;
        if (hist_g) hist_g[n_hist] = hs->gmax;
        ++n_hist;
      }
      if (!std::isfinite(hs->energy) || !std::isfinite(hs->gmax)) {
        res->status = 3;
        res->outer = outer + 1;
        return RIF_OK;
      }
      if (hs->gmax <= par.tol_grad) {
        inner_ok = true;
        break;
      }
      hipEventRecord(ev.e[4], c->stream);
      if ((st = op_orbital_step(c, nb, nmo, nw, in.lambda, inner ? eps : nullptr, C, eps, info))) return st;
      hipEventRecord(ev.e[5], c->stream);
      have_step = true;
    }
    if (have_step && !inner_ok) {   // the loop ended on a step whose time is not yet counted
      if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
      res->ms_orbital += lap(ev.e[4], ev.e[5]);
    }
    res->outer = outer + 1;
    if (inner_ok && outer > 0 && std::fabs(res->energy - e_prev) <= par.tol_energy) {
      res->status = 0;
      break;
    }
    e_prev = res->energy;
  }
  return RIF_OK;
}

}  // namespace rif
