// The conventional four-centre path of Table 1 (Eqs. (3)-(5)), the baseline
// the RI path replaces.
//
//   step 0  (mu nu|sigma lambda), stored once.  Here it is formed from the
//           three-index factors, (mu nu|sigma lambda) = sum_l b^l_{mu nu} b^l_{sigma lambda}
//           (Eq. (6) with the symmetric factor of Eq. (9)), so both paths see the
//           same integrals and must agree to rounding.
//   step 1  P^q_{mu nu} = C_{mu q} C_{nu q}                       (Eq. (4))
//   step 2  J^q_{mu nu} = sum_{sigma lambda} P^q_{sigma lambda} (mu nu|sigma lambda)
//           K^q_{mu sigma} = sum_{nu lambda} P^q_{nu lambda} (mu nu|sigma lambda)
//   step 3  J_pq = sum P^p_{mu nu} J^q_{mu nu},  K_pq = sum P^p_{mu sigma} K^q_{mu sigma}
//                                                                 (Eqs. (3), (5))
//
// Storage: the integrals are kept with the first index pair packed,
// eri[(mu nu)][sigma][lambda] for mu <= nu, (mu nu) the row-major upper
// triangle index.  Each (mu nu) slab is an n_bf x n_bf matrix symmetric in
// (sigma, lambda), which is the layout the half transform reads b in.
//
// Steps 1 and 2 run as one contraction and two gathers.  With
//   Z[q][(mu nu)][sigma] = sum_lambda C_{lambda q} (mu nu|sigma lambda),
// one FP64 MFMA GEMM over every slab (the half transform's kernel with the
// slab count n_bf(n_bf+1)/2 in place of n_aux, n_bf^4 n_Omega flops),
//   J^q_{mu nu}    = sum_sigma C_{sigma q} Z[q][(mu nu)][sigma]      (k_j4c)
//   K^q_{mu sigma} = sum_nu    C_{nu q}    Z[q][pair(mu, nu)][sigma] (k_k4c)
// so P^q is never formed; both gathers stream Z from HBM.  Step 3 is the
// transform of the stacked J^q (K^q) slabs with the MO coefficients: the
// diagonal d[q][p] = c_p^T J^q c_p of that transform is J_pq.
#include <algorithm>
#include <string>

#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

namespace {

__host__ __device__ inline long pair_index(long a, long b, long n) {   // a <= b
  return a * n - a * (a - 1) / 2 + (b - a);
}

// b[l][mu][nu] -> bp[l][(mu nu)], mu <= nu.  One workgroup per (l, mu) row.
__global__ __launch_bounds__(256) void k_pack_pairs(int nb, long rows, const double* __restrict__ b,
                                                    double* __restrict__ bp) {
  const long np = (long)nb * (nb + 1) / 2;
  for (long rr = blockIdx.x; rr < rows; rr += gridDim.x) {
    const long l = rr / nb;
    const int mu = (int)(rr - l * nb);
    const double* src = b + (l * nb + mu) * nb;
    double* dst = bp + l * np + pair_index(mu, mu, nb);
    for (int nu = mu + threadIdx.x; nu < nb; nu += 256) dst[nu - mu] = src[nu];
  }
}

constexpr int kMaxNb4c = 2048;

// K^q_{mu sigma} = sum_nu C_{nu q} Z[q][pair(mu, nu)][sigma] for sigma >= mu,
// written to (mu, sigma) and mirrored to (sigma, mu).  Workgroup (mu, q),
// lanes along sigma (coalesced rows of Z); the sum over nu runs in one fixed
// order.
__global__ __launch_bounds__(256) void k_k4c(int nb, int nmo, long np, const double* __restrict__ Z,
                                             const double* __restrict__ C, double* __restrict__ Kn) {
  __shared__ double cq[kMaxNb4c];
  const int mu = blockIdx.x, q = blockIdx.y;
  for (int i = threadIdx.x; i < nb; i += 256) cq[i] = C[(long)i * nmo + q];
  __syncthreads();
  const double* Zq = Z + (long)q * np * nb;
  double* K = Kn + (long)q * nb * nb;
  for (int s = mu + (int)threadIdx.x; s < nb; s += 256) {
    double acc0 = 0.0, acc1 = 0.0;
    int nu = 0;
    for (; nu + 1 < nb; nu += 2) {
      const long p0 = nu < mu ? pair_index(nu, mu, nb) : pair_index(mu, nu, nb);
      const long p1 = nu + 1 < mu ? pair_index(nu + 1, mu, nb) : pair_index(mu, nu + 1, nb);
      acc0 = fma(cq[nu], Zq[p0 * nb + s], acc0);
      acc1 = fma(cq[nu + 1], Zq[p1 * nb + s], acc1);
    }
    if (nu < nb) {
      const long p0 = nu < mu ? pair_index(nu, mu, nb) : pair_index(mu, nu, nb);
      acc0 = fma(cq[nu], Zq[p0 * nb + s], acc0);
    }
    const double v = acc0 + acc1;
    K[(long)mu * nb + s] = v;
    if (s != mu) K[(long)s * nb + mu] = v;
  }
}

// J^q_{mu nu} = sum_sigma C_{sigma q} Z[q][(mu nu)][sigma] for nu >= mu (one
// wave per (mu nu) row, DPP wave sum), written to (mu, nu) and (nu, mu).
// Workgroup (mu, q); wave w takes nu = mu + w, mu + w + 4, ...
__global__ __launch_bounds__(256) void k_j4c(int nb, int nmo, long np, const double* __restrict__ Z,
                                             const double* __restrict__ C, double* __restrict__ Jn) {
  __shared__ double cq[kMaxNb4c];
  const int mu = blockIdx.x, q = blockIdx.y;
  for (int i = threadIdx.x; i < nb; i += 256) cq[i] = C[(long)i * nmo + q];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* Zq = Z + (long)q * np * nb;
  double* J = Jn + (long)q * nb * nb;
  for (int nu = mu + w; nu < nb; nu += 4) {
    const double* row = Zq + pair_index(mu, nu, nb) * nb;
    double acc = 0.0;
    for (int s = lane; s < nb; s += 64) acc = fma(cq[s], row[s], acc);
    const double v = wave_sum_dpp(acc);
    if (lane == 0) {
      J[(long)mu * nb + nu] = v;
      J[(long)nu * nb + mu] = v;
    }
  }
}

// out[p][q] = in[q][p] (n x n, FP64)
__global__ __launch_bounds__(256) void k_transpose_sq(int n, const double* __restrict__ in, double* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)n * n) return;
  const long p = i / n, q = i - p * n;
  out[i] = in[q * n + p];
}

}  // namespace

unsigned long long eri4_bytes(int nb) {
  const unsigned long long np = (unsigned long long)nb * (nb + 1) / 2;
  return np * (unsigned long long)nb * nb * sizeof(double);
}

rif_status op_eri4_from_b(rif_ctx* c, int nb, int na, const double* b, double* eri) {
  const long np = (long)nb * (nb + 1) / 2;
  Carve cv;
  const size_t o_bp = cv.take<double>((size_t)na * np);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  double* bp = (double*)((char*)c->ws + o_bp);
  {
    ProfScope ps(c, "eri4_pack");
    const long rows = (long)na * nb;
    hipLaunchKernelGGL(k_pack_pairs, dim3((unsigned)std::min(rows, 65536L)), dim3(256), 0, c->stream, nb, rows, b, bp);
    if ((st = check_launch(c, "eri4_pack"))) return st;
  }
  // eri[(mu nu)][sigma lambda] = sum_l bp[l][(mu nu)] b[l][sigma lambda]; a one-off
  // product, so its tile comes from the wave-quantisation model even with
  // autotuning on (timing five shapes of it would cost more than it saves)
  const int tune = c->tune_mode;
  c->tune_mode = 0;
  st = op_gemm_big(c, (int)np, nb * nb, na, bp, np, b, (long)nb * nb, eri, (long)nb * nb);
  c->tune_mode = tune;
  return st;
}

rif_status op_jk_4c(rif_ctx* c, int nb, int nw, int nmo, const double* eri, const double* C, double* Jn, double* Kn,
                    double* J, double* K) {
  if (nb > kMaxNb4c) return fail(c, RIF_EINVAL, "rif_jk_4c: n_bf above 2048");
  const long np = (long)nb * (nb + 1) / 2;
  Carve cv;
  const size_t o_z = cv.take<double>((size_t)nw * np * nb);
  const size_t o_h = cv.take<double>((size_t)nw * nw * nb);     // step 3: transform of the stacked slabs
  const size_t o_m = cv.take<double>((size_t)nw * nw * nw);
  const size_t o_d = cv.take<double>((size_t)nw * nw);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  char* ws = (char*)c->ws;
  double* Z = (double*)(ws + o_z);
  // steps 1-2: Z, then the two gathers
  if ((st = op_half_slabs_f64(c, nb, np, nw, nmo, eri, C, Z))) return st;
  {
    ProfScope ps(c, "eri4_j");
    hipLaunchKernelGGL(k_j4c, dim3((unsigned)nb, (unsigned)nw), dim3(256), 0, c->stream, nb, nmo, np, Z, C, Jn);
    if ((st = check_launch(c, "eri4_j"))) return st;
  }
  {
    ProfScope ps(c, "eri4_k");
    hipLaunchKernelGGL(k_k4c, dim3((unsigned)nb, (unsigned)nw), dim3(256), 0, c->stream, nb, nmo, np, Z, C, Kn);
    if ((st = check_launch(c, "eri4_k"))) return st;
  }
  // step 3: d[q][p] = c_p^T X^q c_p of the stacked X^q = J^q (K^q) is X_pq
  double* H = (double*)(ws + o_h);
  double* M = (double*)(ws + o_m);
  double* D = (double*)(ws + o_d);
  const unsigned g = (unsigned)(((long)nw * nw + 255) / 256);
  for (int x = 0; x < 2; ++x) {
    if ((st = op_transform(c, 0, nb, nw, nw, nmo, x ? Kn : Jn, C, H, M, D))) return st;
    hipLaunchKernelGGL(k_transpose_sq, dim3(g), dim3(256), 0, c->stream, nw, D, x ? K : J);
    if ((st = check_launch(c, "eri4_mo"))) return st;
  }
  return RIF_OK;
}

}  // namespace rif
