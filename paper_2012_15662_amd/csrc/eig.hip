// Tridiagonal reduction of the orbital step's symmetric eigenproblem in one
// launch (the diagonalisation of F^lambda, Sec. II and Fig. 1).
//
// F = Q T Q^T by Householder reflections, Q = H_0 H_1 ... H_{n-2},
// H_k = I - tau_k v_k v_k^T, v_k zero above index k+1 and one at k+1; T is
// tridiagonal with diagonal d and off-diagonal e.  Step k, with A the current
// matrix (trailing rows and columns k+1..n-1 still to be reduced):
//   x = A[k+1:, k];  beta = -sign(x_0) |x|;  tau = (beta - x_0) / beta;
//   v = (1, x_1.. / (x_0 - beta));  e_k = beta  (tau = 0 and e_k = x_0 when
//   x_1.. vanish: H_k = I)
//   p = tau A v;  w = p - (tau/2)(p^T v) v;  A <- A - v w^T - w v^T  (= H A H)
//   Q <- Q H_k, row by row: q <- q - tau (q . v) v^T.
// The rank-2 form of H A H is the textbook one (Golub and Van Loan, Sec. 8.3).
// The reduction is latency-bound at the orbital step's sizes (n of a few
// hundred: ~1 MB of FP64), so it runs as ONE cooperative launch instead of a
// few kernels per column.  Row i of F and row i of Q live in the LDS of
// workgroup i mod G for the whole reduction.  Per column k, with v_k and
// tau_k already known to every workgroup:
//   phase B  every workgroup forms p_i = tau_k (A v_k)_i for its rows and
//            publishes them, then applies H_k to its rows of Q (which needs
//            nothing from other workgroups and covers the wait for p)
//   phase C  every workgroup reads all of p, forms p^T v and w itself and
//            updates its rows of A.  The owner of row k+2 updates that row
//            first and publishes it (it is needed one column later).  Every
//            workgroup then applies H_k to row k+1, published by its owner one
//            column earlier, and forms v_{k+1} and tau_{k+1} from it itself.
// So each column waits for one exchange (p), and every workgroup forms the
// same v, w and tau: the same arithmetic in the same order on the same data.
// Q is formed here so that the back-transformation of T's eigenvectors is one
// GEMM instead of a sequence of reflector applications.
// Workgroups exchange data without barriers or cache flushes: every published
// value has its own slot per column (p_k and row k+2), filled beforehand with
// a signalling-NaN pattern that no arithmetic result takes (results of
// arithmetic on NaNs are quiet NaNs), written once with an agent-scope atomic
// store and read by polling it with agent-scope atomic loads until it no
// longer holds that pattern.  Each value carries its own readiness, so no
// ordering between different values is needed.  Every wait is bounded: past
// the poll limit, or once another workgroup has flagged a timeout, the
// workgroup flags it and returns, so every wave exits.  Within a workgroup the
// waves share out the rows (wave w takes rows t0 + w, t0 + w + 8, ..., t0 the
// first row still active) and every reduction is formed whole in each wave.
#include <algorithm>
#include <string>

#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

namespace {
constexpr int kTrdThreads = 512;   // eight waves, one row of A and Q each by default
constexpr int kTrdWaves = kTrdThreads / 64;
constexpr size_t kTrdLds = 150 * 1024;        // dynamic LDS per workgroup, at most
constexpr size_t kTrdLdsDefault = 64 * 1024;  // beyond this the kernel needs the attribute raised
constexpr unsigned long long kEmpty = 0x7FF4C0FFEE5E7F11ull;   // signalling NaN

struct TrdArgs {
  int n, G;
  const double* F;        // [n][n] symmetric
  double* Q;              // [n][n] out, row-major
  double *d, *e;          // [n], [n-1] out
  double* Rb;             // [n][n] row i of A after H_{i-2}, in row i  (slots, kEmpty at launch)
  double* Pb;             // [n][n] p_k in row k
  int* err;               // set when a wait timed out
  long long spin;         // polls of one value before giving up; < 0: give up at once
};

__device__ __forceinline__ double wave_sum(double x) { return wave_sum_dpp(x); }

__device__ __forceinline__ void put(double* p, double v) {
  __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long peek(const double* p) {
  return __hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The value of slot p once written; false past the poll limit (at once for a
// negative limit) or once another workgroup has flagged a timeout.
__device__ bool take(const double* p, unsigned long long u, double& out, const int* err, long long spin) {
  if (spin < 0) return false;
  for (long long s = 0; u == kEmpty; ++s) {
    if (s >= spin || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
    u = peek(p);
  }
  out = __longlong_as_double((long long)u);
  return true;
}
// dst[j] = slot src[j] for j in [j0, j1), two loads in flight per thread
__device__ bool take_range(const double* src, double* dst, int j0, int j1, const int* err, long long spin) {
  for (int j = j0 + (int)threadIdx.x; j < j1; j += 2 * kTrdThreads) {
    const int j2 = j + kTrdThreads;
    const unsigned long long u1 = peek(src + j), u2 = j2 < j1 ? peek(src + j2) : 0ull;
    double x;
    if (!take(src + j, u1, x, err, spin)) return false;
    dst[j] = x;
    if (j2 < j1) {
      if (!take(src + j2, u2, x, err, spin)) return false;
      dst[j2] = x;
    }
  }
  return true;
}

__global__ __launch_bounds__(kTrdThreads) void k_trd(TrdArgs a) {
  extern __shared__ double sm[];
  const int n = a.n, G = a.G, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int R = g < n ? (n - g + G - 1) / G : 0;   // rows i = g + G t, t < R
  double* rows = sm;                                // [R][n] rows of A
  double* qrows = rows + (long)R * n;               // [R][n] rows of Q
  double* vbuf = qrows + (long)R * n;               // [2][n] v_k by parity of k
  double* p = vbuf + 2L * n;                        // [n] p_k
  double* x = p + n;                                // [n] row k+1 of A
  for (long y = tid; y < (long)R * n; y += kTrdThreads) {
    const int t = (int)(y / n), j = (int)(y - (long)t * n);
    rows[y] = a.F[(long)(g + G * t) * n + j];
    qrows[y] = j == g + G * t ? 1.0 : 0.0;
  }
  for (int j = tid; j < n; j += kTrdThreads) x[j] = a.F[j];   // row 0
  __syncthreads();
  // v_k and tau_k from row k of A (x, entries k..n-1), in every workgroup
  // alike; d_k and e_k from workgroup 0.  Ends with a workgroup barrier.
  auto reflect = [&](int k) -> double {
    const int m0 = k + 1;
    double ss = 0.0;
    for (int j = k + 2 + lane; j < n; j += 64) ss += x[j] * x[j];
    ss = wave_sum(ss);
    const double alpha = x[m0];
    double beta = alpha, tau = 0.0, scale = 0.0;
    if (ss != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    double* v = vbuf + (long)(k & 1) * n;
    for (int j = m0 + tid; j < n; j += kTrdThreads) v[j] = j == m0 ? 1.0 : x[j] * scale;
    if (g == 0 && tid == 0) {
      a.d[k] = x[k];
      a.e[k] = beta;
    }
    __syncthreads();
    return tau;
  };
  double tau = n > 1 ? reflect(0) : 0.0;
  for (int k = 0; k + 1 < n; ++k) {
    const int m0 = k + 1;
    const int t0 = m0 > g ? (m0 - g + G - 1) / G : 0;   // first row of A held here at or past m0
    const double* v = vbuf + (long)(k & 1) * n;
    // phase B: p_i = tau sum_j A_ij v_j for the rows held here
    double* Pk = a.Pb + (long)k * n;
    for (int t = t0 + wv; t < R; t += kTrdWaves) {
      const double* r = rows + (long)t * n;
      double s = 0.0;
      for (int j = m0 + lane; j < n; j += 64) s += r[j] * v[j];
      s = wave_sum(s);
      if (lane == 0) put(Pk + g + G * t, tau * s);
    }
    // Q <- Q H_k on the rows of Q held here
    for (int t = wv; t < R; t += kTrdWaves) {
      double* q = qrows + (long)t * n;
      double s = 0.0;
      for (int j = m0 + lane; j < n; j += 64) s += q[j] * v[j];
      s = tau * wave_sum(s);
      for (int j = m0 + lane; j < n; j += 64) q[j] -= s * v[j];
    }
    // phase C: row k+1 before H_k (from F for k = 0), all of p
    const bool more = k + 2 < n;   // a reflector for column k+1 follows
    {
      bool ok = true;
      if (more) {
        if (k == 0) {
          for (int j = m0 + tid; j < n; j += kTrdThreads) x[j] = a.F[(long)n + j];
        } else {
          ok = take_range(a.Rb + (long)m0 * n, x, m0, n, a.err, a.spin);
        }
      }
      ok = ok && take_range(Pk, p, m0, n, a.err, a.spin);
      if (!ok) atomicExch(a.err, 1);
      if (__syncthreads_or(!ok)) return;
    }
    double pv = 0.0;
    for (int j = m0 + lane; j < n; j += 64) pv += p[j] * v[j];
    const double K = 0.5 * tau * wave_sum(pv);
    // A <- A - v w^T - w v^T with w = p - K v, on row r (its index i)
    auto update = [&](double* r, int i) {
      const double vi = v[i], wi = p[i] - K * vi;
      for (int j = m0 + lane; j < n; j += 64) {
        const double vj = v[j];
        r[j] -= vi * (p[j] - K * vj) + wi * vj;
      }
    };
    const int kp = k + 2;   // row published now, for column k+1's successor
    const int tp = kp + 1 < n && kp % G == g ? kp / G : -1;
    if (tp >= 0 && wv == tp % kTrdWaves) {
      double* r = rows + (long)tp * n;
      update(r, kp);
      for (int j = kp + lane; j < n; j += 64) put(a.Rb + (long)kp * n + j, r[j]);
    }
    for (int t = t0 + wv; t < R; t += kTrdWaves)
      if (t != tp) update(rows + (long)t * n, g + G * t);
    if (more) {
      // row k+1 after H_k, then column k+1's reflector
      for (int j = m0 + tid; j < n; j += kTrdThreads) {
        const double vj = v[j];
        x[j] -= (p[m0] - K) * vj + (p[j] - K * vj);   // v_{m0} = 1
      }
      __syncthreads();
      tau = reflect(k + 1);
    }
  }
  __syncthreads();
  for (long y = tid; y < (long)R * n; y += kTrdThreads) {
    const int t = (int)(y / n), j = (int)(y - (long)t * n);
    a.Q[(long)(g + G * t) * n + j] = qrows[y];
  }
  if ((n - 1) % G == g && tid == 0) a.d[n - 1] = rows[(long)((n - 1) / G) * n + (n - 1)];
}

// after a timed-out wait: T to zero, so the tridiagonal eigensolver that
// follows runs on a valid matrix (the step then reports the timeout)
__global__ __launch_bounds__(256) void k_trd_sanitize(int n, const int* err, double* d, double* e) {
  if (*err == 0) return;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    d[i] = 0.0;
    if (i + 1 < n) e[i] = 0.0;
  }
}

// slots to kEmpty, the timeout flag to zero
__global__ __launch_bounds__(256) void k_trd_reset(unsigned long long* slots, long count, int* err) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) slots[i] = kEmpty;
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

size_t trd_lds(int n, int G) {
  const long R = (n + G - 1) / G;
  return (size_t)(2 * R * n + 4L * n) * sizeof(double);   // rows of A and Q, v (two), p, x
}
long trd_slots(int n) { return 2L * n * n; }
}  // namespace

int trd_groups(rif_ctx* c, int n, int want) {
  if (n < 2) return 0;
  int ncu = 0, coop = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device) != hipSuccess || !coop) {
    (void)hipGetLastError();
    return 0;
  }
  // `want` workgroups if given, else one row per wave (at least 16
  // workgroups: more shorten each one's share of a column, fewer shorten the
  // waits; eight waves of one row measured best at 348, 580 and 1000 rows);
  // more if the rows do not fit the LDS budget; at most one per CU and one per
  // row
  const int gmax = std::min(ncu, n);
  int G = want > 0 ? want : std::max(std::min(16, n), (n + kTrdWaves - 1) / kTrdWaves);
  G = std::min(G, gmax);
  while (G <= gmax && trd_lds(n, G) > kTrdLds) ++G;
  return G <= gmax ? G : 0;
}

size_t trd_scratch_bytes(int n) { return (size_t)trd_slots(n) * sizeof(double); }

rif_status op_trd(rif_ctx* c, int n, int G, const double* F, double* Q, double* d, double* e, void* scratch,
                  int* err) {
  TrdArgs a{};
  a.n = n;
  a.G = G;
  a.F = F;
  a.Q = Q;
  a.d = d;
  a.e = e;
  double* s = (double*)scratch;
  a.Rb = s;
  a.Pb = s + (long)n * n;
  a.err = err;
  a.spin = c->wait_limit;
  const size_t lds = trd_lds(n, G);
  if (lds > kTrdLdsDefault) {
    const hipError_t he = hipFuncSetAttribute((const void*)k_trd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (he != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, RIF_EHIP, std::string("tridiagonal reduction: LDS attribute failed: ") + hipGetErrorString(he));
    }
  }
  const long count = trd_slots(n);
  const unsigned nblk = (unsigned)std::min(1024L, (count + 255) / 256);
  hipLaunchKernelGGL(k_trd_reset, dim3(nblk), dim3(256), 0, c->stream, (unsigned long long*)s, count, err);
  if (rif_status st = check_launch(c, "trd_reset")) return st;
  void* args[] = {&a};
  const hipError_t he =
      hipLaunchCooperativeKernel((const void*)k_trd, dim3(G), dim3(kTrdThreads), args, (unsigned)lds, c->stream);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, RIF_EHIP, std::string("cooperative launch of the tridiagonal reduction failed: ") +
                                 hipGetErrorString(he));
  }
  hipLaunchKernelGGL(k_trd_sanitize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, (const int*)err,
                     d, e);
  return check_launch(c, "trd_sanitize");
}

}  // namespace rif
