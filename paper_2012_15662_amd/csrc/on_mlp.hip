// Occupation-number optimisation at fixed orbitals and the learned warm start.
//
// The paper's occupancy optimisation (Sec. II) minimises Eq. (2) over the ONs
// with J, K fixed, through auxiliary variables gamma that keep the bounds and
// the pair normalisation.  Parametrisation used here, per pair g with ncwo weak
// orbitals (ascending index):
//   n_g = (1 + cos^2 gamma_g)/2,   n_{w_k} = (1 - n_g) w_k,
//   w_1 = cos^2 b_1, w_k = prod_{j<k} sin^2 b_j cos^2 b_k, w_last = prod sin^2 b_j,
//   variables [gamma_g, b_1 .. b_{ncwo-1}] at g*ncwo + j.
//
//   k_on_opt      one workgroup per problem runs L-BFGS (history 8, backtracking
//                 with Armijo or, within rounding noise, approximate Wolfe) to max|dE/dgamma| <= tol, all in FP64 with
//                 fixed-order reductions.
//   k_on_feat     per-pair features (39) and ON targets/masks for the MLP.
//   k_on_warm     MLP ON predictions -> starting gamma.
//   MLP           39 -> 128 -> 128 -> 128 -> 7 (tanh, masked softmax), FP32 on
//                 the FP32 MFMA engine: forward, backward, softmax/loss, Adam.
#include <math.h>

#include <algorithm>

#include "mfma_engine.hpp"
#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

__host__ __device__ static inline int cdiv_i(long a, long b) { return (int)((a + b - 1) / b); }

constexpr int kHist = 8;        // L-BFGS history
constexpr int kOnThreads = 256;
constexpr int kKmax = 6;         // weak slots in the features
constexpr int kNin = 3 + 5 * kKmax + kKmax;   // 39
constexpr int kNhid = 128;
constexpr int kNout = 1 + kKmax;               // 7

__device__ __forceinline__ int on_pair(const int* pair_of, int p, int npairs, int ncwo) {
  if (pair_of) return pair_of[p];
  return p < npairs ? p : npairs - 1 - (p - npairs) / ncwo;
}

// Fixed-order sum over the 256 threads of a block; every thread gets the result.
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = v;
  __syncthreads();
  for (int s = kOnThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = v;
  __syncthreads();
  for (int s = kOnThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Hyperspherical weights w[0..m-1] and their derivatives dw[k][j] = dw_k/db_j.
__device__ void weights(const double* beta, int m, double* w, double* dw /* [m][m-1] or null */) {
  double s = 1.0;
  for (int k = 0; k < m - 1; ++k) {
    const double c = cos(beta[k]);
    w[k] = s * c * c;
    const double sn = sin(beta[k]);
    s *= sn * sn;
  }
  w[m - 1] = s;
  if (!dw) return;
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m - 1; ++j) {
      double v = 0.0;
      if (k == m - 1 || j <= k) {
        v = 1.0;
        for (int i = 0; i < (k < m - 1 ? k : m - 1); ++i) {
          const double si = sin(beta[i]), ci = cos(beta[i]);
          v *= (i == j) ? 2.0 * si * ci : si * si;
        }
        if (k < m - 1) {
          const double sk = sin(beta[k]), ck = cos(beta[k]);
          v *= (j == k) ? -2.0 * ck * sk : ck * ck;
        }
      }
      dw[k * (m - 1) + j] = v;
    }
}

// Workspace of one problem, in doubles (the weak-orbital table follows as ints).
__host__ __device__ inline long on_ws_doubles(int nw, int npairs, int ncwo) {
  const long nv = (long)npairs * ncwo;
  return (2L * kHist + 5) * nv + 2L * nw + (npairs * (long)ncwo + 1) / 2 + 4;
}

struct OnView {
  int nw, npairs, ncwo, nv, functional;
  const double *Hpp, *J, *K;
  const int* pair_of;
  double *S, *Y, *x, *g, *d, *xn, *gn, *n, *dn;
  int* weak;
};

// E(x) and dE/dx for the problem; writes n, dn and gout.  Returns E.
__device__ double on_eval(const OnView& v, const double* x, double* gout, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ONs from the variables
  for (int g = tid; g < v.npairs; g += kOnThreads) {
    const double* xg = x + (long)g * v.ncwo;
    const double c = cos(xg[0]);
    const double ng = 0.5 * (1.0 + c * c);
    v.n[g] = ng;
    double w[kKmax + 8];
    weights(xg + 1, v.ncwo, w, nullptr);
    for (int k = 0; k < v.ncwo; ++k) v.n[v.weak[g * v.ncwo + k]] = (1.0 - ng) * w[k];
  }
  __syncthreads();
  // dE/dn and the energy, one wave per row p, lanes over q
  double erow = 0.0;
  for (int p = wave; p < v.nw; p += kOnThreads / 64) {
    const double np = v.n[p];
    const int gp = on_pair(v.pair_of, p, v.npairs, v.ncwo);
    const double php = sqrt(np * (1.0 - np));
    const double dphp = (1.0 - 2.0 * np) / (2.0 * fmax(php, 1e-300));
    double e = 0.0, dsum = 0.0;
    for (int q = lane; q < v.nw; q += 64) {
      const double nq = v.n[q];
      const double Jpq = v.J[(long)p * v.nw + q], Kpq = v.K[(long)p * v.nw + q];
      const int gq = on_pair(v.pair_of, q, v.npairs, v.ncwo);
      if (gp == gq) {
        if (p == q) {
          e += np * Kpq;
        } else {
          const double sg = (p >= v.npairs && q >= v.npairs) ? 1.0 : -1.0;
          e += sg * sqrt(np * nq) * Kpq;
          dsum += 2.0 * sg * 0.5 * sqrt(nq / fmax(np, 1e-300)) * Kpq;
        }
      } else {
        const double phq = sqrt(nq * (1.0 - nq));
        double bb = -np * nq, db = -nq;
        if (v.functional == RIF_PNOF7) {
          bb -= php * phq;
          db -= dphp * phq;
        }
        e += 2.0 * np * nq * Jpq + bb * Kpq;
        dsum += 2.0 * (2.0 * nq * Jpq + db * Kpq);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      e += __shfl_xor(e, off, 64);
      dsum += __shfl_xor(dsum, off, 64);
    }
    if (lane == 0) {
      v.dn[p] = 2.0 * v.Hpp[p] + v.K[(long)p * v.nw + p] + dsum;
      erow += 2.0 * np * v.Hpp[p] + e;
    }
  }
  const double E = block_sum(erow, red);  // includes the __syncthreads that publishes dn
  // chain rule to the variables, one thread per pair
  for (int g = tid; g < v.npairs; g += kOnThreads) {
    const double* xg = x + (long)g * v.ncwo;
    double* gg = gout + (long)g * v.ncwo;
    const double c = cos(xg[0]), s = sin(xg[0]);
    const double h = 0.5 * s * s, dh = c * s;
    double w[kKmax + 8], dw[(kKmax + 8) * (kKmax + 8)];
    weights(xg + 1, v.ncwo, w, dw);
    double t = -c * s * v.dn[g];
    for (int k = 0; k < v.ncwo; ++k) t += dh * w[k] * v.dn[v.weak[g * v.ncwo + k]];
    gg[0] = t;
    for (int j = 0; j < v.ncwo - 1; ++j) {
      double u = 0.0;
      for (int k = 0; k < v.ncwo; ++k) u += h * dw[k * (v.ncwo - 1) + j] * v.dn[v.weak[g * v.ncwo + k]];
      gg[1 + j] = u;
    }
  }
  __syncthreads();
  return E;
}

__device__ double dot(const double* a, const double* b, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kOnThreads) s += a[i] * b[i];
  return block_sum(s, red);
}

__global__ __launch_bounds__(kOnThreads) void k_on_opt(const OnProblem* __restrict__ probs) {
  __shared__ double red[kOnThreads];
  const OnProblem& P = probs[blockIdx.x];
  const int tid = threadIdx.x;
  OnView v;
  v.nw = P.n_omega; v.npairs = P.n_pairs; v.ncwo = P.n_cwo; v.nv = P.n_pairs * P.n_cwo;
  v.functional = P.functional;
  v.Hpp = P.Hpp; v.J = P.J; v.K = P.K; v.pair_of = P.pair_of;
  double* w = P.work;
  const int nv = v.nv;
  v.S = w; w += (long)kHist * nv;
  v.Y = w; w += (long)kHist * nv;
  double rho[kHist], alpha[kHist];  // identical in every thread (block-reduced)
  v.x = w; w += nv;
  v.g = w; w += nv;
  v.d = w; w += nv;
  v.xn = w; w += nv;
  v.gn = w; w += nv;
  v.n = w; w += v.nw;
  v.dn = w; w += v.nw;
  v.weak = (int*)w;
  // weak-orbital table (ascending index); a bad map stops the problem
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int g = tid; g < v.npairs; g += kOnThreads) {
    int k = 0;
    for (int p = v.npairs; p < v.nw; ++p)
      if (on_pair(v.pair_of, p, v.npairs, v.ncwo) == g) {
        if (k < v.ncwo) v.weak[g * v.ncwo + k] = p;
        ++k;
      }
    if (k != v.ncwo || v.ncwo > kKmax + 8) atomicOr(&bad, 1);
  }
  for (int i = tid; i < nv; i += kOnThreads) v.x[i] = P.gamma[i];
  __syncthreads();
  if (bad) {
    if (tid == 0) { *P.status = 3; *P.iters = 0; }
    return;
  }
  double E = on_eval(v, v.x, v.g, red);
  int it = 0, hist = 0, head = 0, status = 1;
  while (true) {
    double gm = 0.0;
    for (int i = tid; i < nv; i += kOnThreads) gm = fmax(gm, fabs(v.g[i]));
    gm = block_max(gm, red);
    if (gm <= P.tol) { status = 0; break; }
    if (it >= P.max_it) { status = 1; break; }
    // two-loop recursion: d = -H g
    for (int i = tid; i < nv; i += kOnThreads) v.d[i] = v.g[i];
    __syncthreads();
    for (int j = 0; j < hist; ++j) {
      const int h = (head - 1 - j + kHist) % kHist;
      const double a = rho[h] * dot(v.S + (long)h * nv, v.d, nv, red);
      alpha[h] = a;
      for (int i = tid; i < nv; i += kOnThreads) v.d[i] -= a * v.Y[(long)h * nv + i];
      __syncthreads();
    }
    double scale;
    if (hist > 0) {
      const int h = (head - 1 + kHist) % kHist;
      scale = 1.0 / (rho[h] * dot(v.Y + (long)h * nv, v.Y + (long)h * nv, nv, red));
    } else {
      scale = fmin(1.0, 1.0 / gm);
    }
    for (int i = tid; i < nv; i += kOnThreads) v.d[i] *= scale;
    __syncthreads();
    for (int j = hist - 1; j >= 0; --j) {
      const int h = (head - 1 - j + kHist) % kHist;
      const double b = rho[h] * dot(v.Y + (long)h * nv, v.d, nv, red);
      const double a = alpha[h];
      for (int i = tid; i < nv; i += kOnThreads) v.d[i] += (a - b) * v.S[(long)h * nv + i];
      __syncthreads();
    }
    for (int i = tid; i < nv; i += kOnThreads) v.d[i] = -v.d[i];
    __syncthreads();
    double gd = dot(v.g, v.d, nv, red);
    if (!(gd < 0.0)) {  // not a descent direction: restart from steepest descent
      for (int i = tid; i < nv; i += kOnThreads) v.d[i] = -v.g[i] * fmin(1.0, 1.0 / gm);
      __syncthreads();
      hist = 0;
      gd = dot(v.g, v.d, nv, red);
    }
    // Backtracking with the Armijo test, or, once the energy change is below
    // its rounding noise, the approximate Wolfe conditions on the directional
    // derivative (Hager and Zhang, 2005): 0.9 phi'(0) <= phi'(a) <= -0.8 phi'(0).
    const double epsE = 1e-12 * fabs(E);
    double step = 1.0, En = 0.0;
    bool ok = false;
    for (int ls = 0; ls < 50; ++ls) {
      for (int i = tid; i < nv; i += kOnThreads) v.xn[i] = v.x[i] + step * v.d[i];
      __syncthreads();
      En = on_eval(v, v.xn, v.gn, red);
      if (En <= E + 1e-4 * step * gd) { ok = true; break; }
      if (En <= E + epsE) {
        const double gnd = dot(v.gn, v.d, nv, red);
        if (gnd >= 0.9 * gd && gnd <= -0.8 * gd) { ok = true; break; }
      }
      step *= 0.5;
    }
    if (!ok) { status = 2; break; }
    // history update (skipped without positive curvature)
    double sy = 0.0;
    for (int i = tid; i < nv; i += kOnThreads) {
      const double si = v.xn[i] - v.x[i], yi = v.gn[i] - v.g[i];
      v.S[(long)head * nv + i] = si;
      v.Y[(long)head * nv + i] = yi;
      sy += si * yi;
    }
    sy = block_sum(sy, red);
    if (sy > 1e-300) {
      rho[head] = 1.0 / sy;
      head = (head + 1) % kHist;
      hist = hist < kHist ? hist + 1 : kHist;
    }
    for (int i = tid; i < nv; i += kOnThreads) {
      v.x[i] = v.xn[i];
      v.g[i] = v.gn[i];
    }
    __syncthreads();
    E = En;
    ++it;
  }
  // outputs: the ONs of the final point (re-evaluated so n matches x)
  E = on_eval(v, v.x, v.g, red);
  for (int i = tid; i < nv; i += kOnThreads) P.gamma[i] = v.x[i];
  for (int p = tid; p < v.nw; p += kOnThreads) P.occ[p] = v.n[p];
  if (tid == 0) {
    *P.energy = E;
    *P.iters = it;
    *P.status = status;
  }
}

// ---- features, targets and warm start ------------------------------------

// Row block of problem i starts at P.row0; one row per pair.  One wave per
// (pair g, problem): the pair's weak orbitals (ascending index, the first
// kKmax) found by a ballot over the orbitals, and each mean field
// m_x = sum_{u strong, u != g} (2 J_xu - K_xu) as a lane-parallel FP64 sum with
// a fixed-order wave reduction.
__global__ __launch_bounds__(64) void k_on_feat(const OnProblem* __restrict__ probs, float* __restrict__ X,
                                                float* __restrict__ T, float* __restrict__ M,
                                                const float* __restrict__ mu, const float* __restrict__ sigma) {
  const OnProblem& P = probs[blockIdx.y];
  const int g = blockIdx.x;
  const int nw = P.n_omega, np_ = P.n_pairs, nc = P.n_cwo;
  if (g >= np_) return;   // the whole wave
  const int lane = threadIdx.x;
  int weak[kKmax];
  int k = 0;
  for (int p0 = np_; p0 < nw && k < kKmax; p0 += 64) {
    const int p = p0 + lane;
    unsigned long long m = __ballot(p < nw && on_pair(P.pair_of, p, np_, nc) == g);
    while (m && k < kKmax) {
      weak[k++] = p0 + __ffsll((long long)m) - 1;
      m &= m - 1;
    }
  }
  auto mf = [&](int x) {
    double s = 0.0;
    for (int u = lane; u < np_; u += 64)
      if (u != g) s += 2.0 * P.J[(long)x * nw + u] - P.K[(long)x * nw + u];
    return wave_sum_dpp(s);
  };
  float f[kNin];
  for (int i = 0; i < kNin; ++i) f[i] = 0.f;
  float t[kNout], m[kNout];
  for (int i = 0; i < kNout; ++i) { t[i] = 0.f; m[i] = 0.f; }
  const int s0 = g;
  f[0] = (float)P.Hpp[s0];
  f[1] = (float)P.J[(long)s0 * nw + s0];
  f[2] = (float)mf(s0);
  t[0] = P.occ ? (float)P.occ[s0] : 0.f;
  m[0] = 1.f;
  for (int q = 0; q < k; ++q) {
    const int p = weak[q];
    f[3 + 5 * q + 0] = (float)(P.Hpp[p] - P.Hpp[s0]);
    f[3 + 5 * q + 1] = (float)P.J[(long)p * nw + p];
    f[3 + 5 * q + 2] = (float)P.K[(long)s0 * nw + p];
    f[3 + 5 * q + 3] = (float)P.J[(long)s0 * nw + p];
    f[3 + 5 * q + 4] = (float)mf(p);
    f[3 + 5 * kKmax + q] = 1.f;
    t[1 + q] = P.occ ? (float)P.occ[p] : 0.f;
    m[1 + q] = 1.f;
  }
  const long row = P.row0 + g;
  for (int i = lane; i < kNin; i += 64) {
    float z = f[i];
    if (mu && sigma && sigma[i] > 0.f) z = (z - mu[i]) / sigma[i];
    X[row * kNin + i] = z;
  }
  for (int i = lane; i < kNout; i += 64) {
    if (T) T[row * kNout + i] = t[i];
    if (M) M[row * kNout + i] = m[i];
  }
}

// Predicted pair ONs p (rows as in k_on_feat) -> starting variables gamma.
__global__ __launch_bounds__(64) void k_on_warm(const OnProblem* __restrict__ probs, const float* __restrict__ Pn) {
  const OnProblem& P = probs[blockIdx.x];
  const int nc = P.n_cwo;
  for (int g = threadIdx.x; g < P.n_pairs; g += 64) {
    const float* p = Pn + (P.row0 + g) * (long)kNout;
    const double ng = fmin(fmax((double)p[0], 0.5), 1.0);
    double* x = P.gamma + (long)g * nc;
    x[0] = acos(sqrt(fmin(fmax(2.0 * ng - 1.0, 0.0), 1.0)));
    double tot = 0.0;
    for (int k = 0; k < nc && k < kKmax; ++k) tot += fmax((double)p[1 + k], 0.0);
    double s = 1.0;
    for (int k = 0; k < nc - 1; ++k) {
      const double wk = (tot > 0.0 && k < kKmax) ? fmax((double)p[1 + k], 0.0) / tot : 1.0 / nc;
      const double c2 = s > 1e-300 ? fmin(fmax(wk / s, 0.0), 1.0) : 1.0;
      x[1 + k] = acos(sqrt(c2));
      s *= 1.0 - c2;
    }
  }
}

// ---- MLP ---------------------------------------------------------------------
// Layer GEMMs run on the FP32 MFMA engine with 64x64 tiles.  Each weight block
// is stored augmented: W_aug = [W (I x O); b (O)], so input rows carry an
// implicit trailing 1.
using MCfg = TileCfg<64, 64, 16, 32, 32>;
using ME = EngF32;

// A operand of y = x_aug W_aug: rows of x (k-contiguous) with x[row][I] = 1.
struct AugRows {
  using S = KCSrc<float, MCfg::BM, ME::BK, MCfg::NT, ME::KV>;
  static constexpr int NP = S::NP, R = S::R, RR = S::RR;
  using type = float;
  S s;
  int I;
  __device__ void init(const float* X, int nrows, int I_, int row0) {
    I = I_;
    s.init([&](int x) -> const float* { return row0 + x < nrows ? X + (long)(row0 + x) * I : nullptr; }, X, I + 1);
  }
  __device__ int xl(int p) const { return s.xl(p); }
  __device__ int kl(int p) const { return s.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return s.valid(p, i, kt); }
  __device__ void fetch(int kt, float (&r)[RR]) const {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int k = kt * ME::BK + s.kl(p);
      r[p] = k >= I ? 1.f : s.rp[p][k];
    }
  }
  __device__ double val(const float (&r)[RR], int p, int i) const { return (double)r[p + i]; }
};

// A operand of dW_aug = x_aug^T dY: element (x = i, k = row) = x[row][i], 1 for i = I.
struct AugCols {
  using S = XCSrc<float, MCfg::BM, ME::BK, MCfg::NT, ME::KV>;
  static constexpr int NP = S::NP, R = S::R, RR = S::RR;
  using type = float;
  S s;
  bool ones;
  __device__ void init(const float* X, int nrows, int I, int i0) {
    s.init(X, I, nrows, [&](int x, long& o) { o = i0 + x < I ? i0 + x : 0; return i0 + x <= I; });
    ones = (i0 + s.x == I);
  }
  __device__ int xl(int p) const { return s.xl(p); }
  __device__ int kl(int p) const { return s.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return s.valid(p, i, kt); }
  __device__ void fetch(int kt, float (&r)[RR]) const { s.fetch(kt, r); }
  __device__ double val(const float (&r)[RR], int p, int i) const { return ones ? 1.0 : (double)r[p + i]; }
};

// y[row][o] = act(x_aug W_aug), act = tanh (hidden) or identity (output)
__global__ __launch_bounds__(MCfg::NT) void k_mlp_fwd(int nrows, int I, int O, const float* __restrict__ X,
                                                      const float* __restrict__ W, float* __restrict__ Y,
                                                      int act_tanh) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<ME, MCfg>()];
  const int r0 = blockIdx.x * MCfg::BM, o0 = blockIdx.y * MCfg::BN;
  AugRows la;
  la.init(X, nrows, I, r0);
  XCSrc<float, MCfg::BN, ME::BK, MCfg::NT, ME::KV> lb;
  lb.init(W, O, I + 1, [&](int x, long& o) { o = o0 + x; return o0 + x < O; });
  ME::Acc<MCfg> acc;
  gemm_mainloop<ME, MCfg>(la, lb, cdiv_i(I + 1, ME::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    if (r0 + m < nrows && o0 + n < O) Y[(long)(r0 + m) * O + o0 + n] = act_tanh ? (float)tanh(v) : (float)v;
  });
}

// dW_aug[i][o] = sum_row x_aug[row][i] dY[row][o]
__global__ __launch_bounds__(MCfg::NT) void k_mlp_wgrad(int nrows, int I, int O, const float* __restrict__ X,
                                                        const float* __restrict__ dY, float* __restrict__ dW) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<ME, MCfg>()];
  const int i0 = blockIdx.x * MCfg::BM, o0 = blockIdx.y * MCfg::BN;
  AugCols la;
  la.init(X, nrows, I, i0);
  XCSrc<float, MCfg::BN, ME::BK, MCfg::NT, ME::KV> lb;
  lb.init(dY, O, nrows, [&](int x, long& o) { o = o0 + x; return o0 + x < O; });
  ME::Acc<MCfg> acc;
  gemm_mainloop<ME, MCfg>(la, lb, cdiv_i(nrows, ME::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    if (i0 + m <= I && o0 + n < O) dW[(long)(i0 + m) * O + o0 + n] = (float)v;
  });
}

// dA[row][i] = (sum_o dY[row][o] W[i][o]) * (1 - h[row][i]^2), h = tanh output of the layer below
__global__ __launch_bounds__(MCfg::NT) void k_mlp_dgrad(int nrows, int I, int O, const float* __restrict__ dY,
                                                        const float* __restrict__ W, const float* __restrict__ h,
                                                        float* __restrict__ dA) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<ME, MCfg>()];
  const int r0 = blockIdx.x * MCfg::BM, i0 = blockIdx.y * MCfg::BN;
  KCSrc<float, MCfg::BM, ME::BK, MCfg::NT, ME::KV> la;
  la.init([&](int x) -> const float* { return r0 + x < nrows ? dY + (long)(r0 + x) * O : nullptr; }, dY, O);
  KCSrc<float, MCfg::BN, ME::BK, MCfg::NT, ME::KV> lb;
  lb.init([&](int x) -> const float* { return i0 + x < I ? W + (long)(i0 + x) * O : nullptr; }, W, O);
  ME::Acc<MCfg> acc;
  gemm_mainloop<ME, MCfg>(la, lb, cdiv_i(O, ME::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const int r = r0 + m, i = i0 + n;
    if (r < nrows && i < I) {
      const float hv = h[(long)r * I + i];
      dA[(long)r * I + i] = (float)(v * (1.0 - (double)hv * hv));
    }
  });
}

// masked softmax of the logits, loss partial per block, dZ of the loss
__global__ __launch_bounds__(256) void k_mlp_softmax_loss(int nrows, const float* __restrict__ Z,
                                                          const float* __restrict__ T, const float* __restrict__ M,
                                                          float* __restrict__ Pout, float* __restrict__ dZ,
                                                          double* __restrict__ lpart) {
  __shared__ double red[256];
  const int row = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (row < nrows) {
    const float* z = Z + (long)row * kNout;
    const float* m = M + (long)row * kNout;
    double zmax = -1e300, p[kNout], e = 0.0;
    for (int k = 0; k < kNout; ++k)
      if (m[k] > 0.f) zmax = fmax(zmax, (double)z[k]);
    for (int k = 0; k < kNout; ++k) {
      p[k] = m[k] > 0.f ? exp((double)z[k] - zmax) : 0.0;
      e += p[k];
    }
    double dp[kNout], sdp = 0.0;
    for (int k = 0; k < kNout; ++k) {
      p[k] /= e;
      if (Pout) Pout[(long)row * kNout + k] = (float)p[k];
      if (T) {
        const double t = T[(long)row * kNout + k];
        l += m[k] * (p[k] - t) * (p[k] - t);
        dp[k] = 2.0 * m[k] * (p[k] - t) / nrows;
        sdp += dp[k] * p[k];
      }
    }
    if (T && dZ)
      for (int k = 0; k < kNout; ++k) dZ[(long)row * kNout + k] = (float)(p[k] * (dp[k] - sdp));
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && lpart) lpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(int n, const double* __restrict__ parts, double scale,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += parts[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam with bias correction (step counts from 1)
__global__ __launch_bounds__(256) void k_adam(int n, float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int step, float lr,
                                              float b1, float b2, float eps) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  th[i] -= lr * mh / (sqrtf(vh) + eps);
}

// H_pp = c_p^T H c_p: one workgroup per orbital; threads over mu read H[nu][mu]
// (H symmetric) coalesced, then a fixed-order block sum.
__global__ __launch_bounds__(256) void k_hpp(int nb, int nmo, const double* __restrict__ H,
                                             const double* __restrict__ C, double* __restrict__ Hpp) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double acc = 0.0;
  for (int mu = threadIdx.x; mu < nb; mu += 256) {
    double t = 0.0;
    for (int nu = 0; nu < nb; ++nu) t = fma(H[(long)nu * nb + mu], C[(long)nu * nmo + p], t);
    acc = fma(C[(long)mu * nmo + p], t, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) Hpp[p] = red[0];
}

// ---- host entry points --------------------------------------------------------

rif_status op_hpp(rif_ctx* c, int nb, int nmo, int nw, const double* H, const double* C, double* Hpp) {
  ProfScope ps(c, "hpp");
  hipLaunchKernelGGL(k_hpp, dim3(nw), dim3(256), 0, c->stream, nb, nmo, H, C, Hpp);
  return check_launch(c, "hpp");
}

static rif_status upload_problems(rif_ctx* c, int n, const OnProblem* probs, OnProblem** dptr) {
  const size_t bytes = sizeof(OnProblem) * (size_t)n;
  Carve cv;
  const size_t o = cv.take<OnProblem>((size_t)n);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  *dptr = (OnProblem*)((char*)c->ws + o);
  if (hipMemcpyAsync(*dptr, probs, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return fail(c, RIF_EHIP, "uploading the problem table failed");
  // the host array may be reused by the caller right after return
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipStreamSynchronize failed");
  return RIF_OK;
}

long on_work_doubles(int nw, int npairs, int ncwo) { return on_ws_doubles(nw, npairs, ncwo); }

rif_status op_on_optimize(rif_ctx* c, int n, const OnProblem* probs) {
  OnProblem* d = nullptr;
  rif_status st = upload_problems(c, n, probs, &d);
  if (st) return st;
  ProfScope ps(c, "on_opt");
  hipLaunchKernelGGL(k_on_opt, dim3(n), dim3(kOnThreads), 0, c->stream, d);
  return check_launch(c, "on_opt");
}

rif_status op_on_features(rif_ctx* c, int n, const OnProblem* probs, float* X, float* T, float* M, const float* mu,
                          const float* sigma) {
  OnProblem* d = nullptr;
  rif_status st = upload_problems(c, n, probs, &d);
  if (st) return st;
  int maxp = 1;
  for (int i = 0; i < n; ++i) maxp = std::max(maxp, probs[i].n_pairs);
  ProfScope ps(c, "on_features");
  hipLaunchKernelGGL(k_on_feat, dim3((unsigned)maxp, (unsigned)n), dim3(64), 0, c->stream, d, X, T, M, mu, sigma);
  return check_launch(c, "on_features");
}

rif_status op_on_warmstart(rif_ctx* c, int n, const OnProblem* probs, const float* Pn) {
  OnProblem* d = nullptr;
  rif_status st = upload_problems(c, n, probs, &d);
  if (st) return st;
  ProfScope ps(c, "on_warm");
  hipLaunchKernelGGL(k_on_warm, dim3(n), dim3(64), 0, c->stream, d, Pn);
  return check_launch(c, "on_warm");
}

static const long kLayerIn[4] = {kNin, kNhid, kNhid, kNhid};
static const long kLayerOut[4] = {kNhid, kNhid, kNhid, kNout};
static long layer_off(int l) {
  long o = 0;
  for (int i = 0; i < l; ++i) o += (kLayerIn[i] + 1) * kLayerOut[i];
  return o;
}
long mlp_n_params() { return layer_off(4); }

rif_status op_mlp_forward(rif_ctx* c, int nrows, const float* X, const float* M, const float* theta, float* H,
                          float* Z, float* Pn) {
  const float* in = X;
  for (int l = 0; l < 4; ++l) {
    const int I = (int)kLayerIn[l], O = (int)kLayerOut[l];
    float* out = l < 3 ? H + (long)l * nrows * kNhid : Z;
    ProfScope ps(c, "mlp_fwd");
    hipLaunchKernelGGL(k_mlp_fwd, dim3(cdiv_i(nrows, MCfg::BM), cdiv_i(O, MCfg::BN)), dim3(MCfg::NT), 0, c->stream,
                       nrows, I, O, in, theta + layer_off(l), out, l < 3 ? 1 : 0);
    rif_status st = check_launch(c, "mlp_fwd");
    if (st) return st;
    in = out;
  }
  hipLaunchKernelGGL(k_mlp_softmax_loss, dim3(cdiv_i(nrows, 256)), dim3(256), 0, c->stream, nrows, Z, nullptr, M,
                     Pn, nullptr, nullptr);
  return check_launch(c, "mlp_softmax");
}

rif_status op_mlp_backward(rif_ctx* c, int nrows, const float* X, const float* M, const float* T,
                           const float* theta, const float* H, const float* Z, float* dA, float* grad,
                           double* loss) {
  const int nb = cdiv_i(nrows, 256);
  Carve cv;
  const size_t o_lp = cv.take<double>((size_t)nb);
  const size_t o_dz = cv.take<float>((size_t)nrows * kNout);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  double* lp = (double*)((char*)c->ws + o_lp);
  float* dZ = (float*)((char*)c->ws + o_dz);
  {
    ProfScope ps(c, "mlp_loss");
    hipLaunchKernelGGL(k_mlp_softmax_loss, dim3(nb), dim3(256), 0, c->stream, nrows, Z, T, M, (float*)nullptr, dZ,
                       lp);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, nb, lp, 1.0 / nrows, loss);
  }
  if ((st = check_launch(c, "mlp_loss"))) return st;
  // dA holds two [nrows][128] ping-pong buffers
  const float* dcur = dZ;
  for (int l = 3; l >= 0; --l) {
    const int I = (int)kLayerIn[l], O = (int)kLayerOut[l];
    const float* xin = l == 0 ? X : H + (long)(l - 1) * nrows * kNhid;
    {
      ProfScope ps(c, "mlp_wgrad");
      hipLaunchKernelGGL(k_mlp_wgrad, dim3(cdiv_i(I + 1, MCfg::BM), cdiv_i(O, MCfg::BN)), dim3(MCfg::NT), 0,
                         c->stream, nrows, I, O, xin, dcur, grad + layer_off(l));
    }
    if ((st = check_launch(c, "mlp_wgrad"))) return st;
    if (l == 0) break;
    float* dnext = dA + (long)(l % 2) * nrows * kNhid;
    {
      ProfScope ps(c, "mlp_dgrad");
      hipLaunchKernelGGL(k_mlp_dgrad, dim3(cdiv_i(nrows, MCfg::BM), cdiv_i(I, MCfg::BN)), dim3(MCfg::NT), 0,
                         c->stream, nrows, I, O, dcur, theta + layer_off(l), xin, dnext);
    }
    if ((st = check_launch(c, "mlp_dgrad"))) return st;
    dcur = dnext;
  }
  return RIF_OK;
}

rif_status op_adam(rif_ctx* c, int n, float* theta, const float* grad, float* m, float* v, int step, float lr,
                   float b1, float b2, float eps) {
  ProfScope ps(c, "adam");
  hipLaunchKernelGGL(k_adam, dim3(cdiv_i(n, 256)), dim3(256), 0, c->stream, n, theta, grad, m, v, step, lr, b1, b2,
                     eps);
  return check_launch(c, "adam");
}

}  // namespace rif
