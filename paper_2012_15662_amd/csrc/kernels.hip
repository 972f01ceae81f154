// Kernels of the RI-PNOF7 hot path (gfx950), in every arithmetic mode.
//
//   half transform   Eq. (12), Table 3 step 2:  b_half[q][l][nu] = sum_mu C[mu][q] b[l][mu][nu]
//   MO transform     Eq. (13), Table 2 step 3:  b_mo[l][p][q] = sum_nu b_half[p][l][nu] C[nu][q]
//   MO J/K           Eqs. (10)-(11), Table 2 step 4 (FP64 sums over l in every mode)
//   per-MO AO J/K    Table 3 steps 3-4
//   energy           Eq. (2) with L = K (FP64)
//   Lagrangian       F^(q) c_q, lambda = C^T Y, G = 4 (lambda - lambda^T) (FP64)
//
// GEMM-shaped steps are templates over the arithmetic mode P (mfma_engine.hpp)
// and a tile shape; each supplies operand loaders describing its own layout in
// HBM.  In the FP64 mode b_half, b_mo, Jn and Kn are stored as double, in the
// other modes as float.  Sums that cross workgroups are written as partials
// and reduced in a fixed order, so every result is deterministic.
#include <math.h>

#include <type_traits>

#include "mfma_engine.hpp"
#include "rif_internal.hpp"

namespace rif {

template <int P>
using IOT = typename std::conditional<P == kF64, double, float>::type;

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This maps the hardware-linear id to a logical tile id so that
// consecutive logical tiles run on the same XCD and share its L2.
__device__ __forceinline__ long xcd_remap(long i, long n) {
  constexpr long X = 8;
  if (n < X) return i;
  const long xcd = i % X, k = i / X;
  const long base = n / X, extra = n % X;
  return xcd * base + (xcd < extra ? xcd : extra) + k;
}

__host__ __device__ static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

#define ENGINE_TYPES                          \
  using E = typename EngineOf<P>::type;       \
  using Acc = typename E::template Acc<Cfg>;  \
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<E, Cfg>()]

template <int P, class T, int BX, int NT>
using XCS = XCSrc<T, BX, EngineOf<P>::type::BK, NT, EngineOf<P>::type::KV>;
template <int P, class T, int BX, int NT>
using KCS = KCSrc<T, BX, EngineOf<P>::type::BK, NT, EngineOf<P>::type::KV>;

// ---------------------------------------------------------------------------
// Half transform.  Since b[l] is symmetric, b[l][mu][nu] = b[l][nu][mu] and the
// step is one GEMM: bh[q][r] = sum_mu C[mu][q] bflat[r][mu] with r = l*n_bf + nu.
// M = q, N = r (stores run along r, contiguous in b_half), K = mu.
template <int P, class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_half_transform(int nb, long nr, int nw, int nmo,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ C,
                                                            IOT<P>* __restrict__ bh) {
  ENGINE_TYPES;
  const int q0 = blockIdx.y * Cfg::BM;
  const long r0 = (long)blockIdx.x * Cfg::BN;
  XCS<P, double, Cfg::BM, Cfg::NT> la;
  la.init(C, nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  KCS<P, double, Cfg::BN, Cfg::NT> lb;
  lb.init([&](int x) -> const double* {
    const long r = r0 + x;
    return r < nr ? b + r * nb : nullptr;
  }, b, nb);
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(nb, E::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const int q = q0 + m;
    const long r = r0 + n;
    if (q < nw && r < nr) bh[(long)q * nr + r] = (IOT<P>)v;
  });
}

// MO transform: rows s = l*n_omega + p, bmo[s][q] = sum_nu bh[p][l][nu] C[nu][q];
// the FP64 diagonal d[l][p] = bmo[l][p][p] comes from the same epilogue.
template <int P, class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_mo_transform(int nb, int na, int nw, int nmo,
                                                          const IOT<P>* __restrict__ bh,
                                                          const double* __restrict__ C,
                                                          IOT<P>* __restrict__ bmo,
                                                          double* __restrict__ d) {
  ENGINE_TYPES;
  const long ns = (long)na * nw;
  const long s0 = (long)blockIdx.x * Cfg::BM;
  const int q0 = blockIdx.y * Cfg::BN;
  const long AB = (long)na * nb;
  KCS<P, IOT<P>, Cfg::BM, Cfg::NT> la;
  la.init([&](int x) -> const IOT<P>* {
    const long s = s0 + x;
    if (s >= ns) return nullptr;
    const long l = s / nw, p = s - l * nw;
    return bh + p * AB + l * nb;
  }, bh, nb);
  XCS<P, double, Cfg::BN, Cfg::NT> lb;
  lb.init(C, nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(nb, E::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const long s = s0 + m;
    const int q = q0 + n;
    if (s < ns && q < nw) {
      bmo[s * nw + q] = (IOT<P>)v;
      if (s % nw == q) d[s] = v;
    }
  });
}

// First block column of block row bi that holds an element with nu >= mu.
__host__ __device__ __forceinline__ int jao_first_col(int bi, int tmu, int tnu) {
  const int t = bi * tmu - (tnu - 1);
  return t <= 0 ? 0 : (t + tnu - 1) / tnu;
}

// Per-MO AO Coulomb: Jn[q][mu][nu] = sum_l d[l][q] b[l][mu][nu].
// M = q, N = a TMU x TNU block of (mu, nu), K = l.  The grid enumerates only
// blocks that touch the upper triangle, q-tile fastest, so the XCD remap
// spreads equal work over the XCDs and q-tiles sharing a b block run on one
// XCD.  Each block writes (mu <= nu) directly and (mu < nu) mirrored, so every
// element of the full matrix is written exactly once.
template <int P, class Cfg, int TNU>
__global__ __launch_bounds__(Cfg::NT) void k_jao(int nb, int na, int nw, const double* __restrict__ b,
                                                 const double* __restrict__ d,
                                                 IOT<P>* __restrict__ Jn) {
  ENGINE_TYPES;
  constexpr int TMU = Cfg::BN / TNU;
  const int nbj = (nb + TNU - 1) / TNU;
  const int nbi = (nb + TMU - 1) / TMU;
  const long nq = (nw + Cfg::BM - 1) / Cfg::BM;
  const long t = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int qt = (int)(t % nq);
  long a = t / nq;
  int bi = 0;
  for (; bi < nbi; ++bi) {
    const int n = nbj - jao_first_col(bi, TMU, TNU);
    if (a < n) break;
    a -= n;
  }
  if (bi >= nbi) return;
  const int bj = jao_first_col(bi, TMU, TNU) + (int)a;
  const int mu0 = bi * TMU, nu0 = bj * TNU;
  const int q0 = qt * Cfg::BM;
  const long B2 = (long)nb * nb;
  XCS<P, double, Cfg::BM, Cfg::NT> la;
  la.init(d, nw, na, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  XCS<P, double, Cfg::BN, Cfg::NT> lb;
  lb.init(b, B2, na, [&](int x, long& o) {
    const int mu = mu0 + x / TNU, nu = nu0 + x % TNU;
    o = (long)mu * nb + nu;
    return mu < nb && nu < nb;
  });
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const int q = q0 + m, mu = mu0 + n / TNU, nu = nu0 + n % TNU;
    if (q < nw && mu < nb && nu < nb) {
      IOT<P>* J = Jn + (long)q * B2;
      if (mu <= nu) J[(long)mu * nb + nu] = (IOT<P>)v;
      if (mu < nu) J[(long)nu * nb + mu] = (IOT<P>)v;
    }
  });
}

// Per-MO AO exchange: Kn[q] = X_q^T X_q with X_q = b_half[q] ([n_aux][n_bf]).
// Square blocks bi <= bj only, mirrored like k_jao.
template <int P, class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_kao(int nb, int na, int nw, const IOT<P>* __restrict__ bh,
                                                 IOT<P>* __restrict__ Kn) {
  static_assert(Cfg::BM == Cfg::BN, "square blocks");
  ENGINE_TYPES;
  const int nbk = (nb + Cfg::BM - 1) / Cfg::BM;
  const long nblk = (long)nbk * (nbk + 1) / 2;  // upper-triangle blocks per q
  const long t = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int q = (int)(t / nblk);
  if (q >= nw) return;
  int rem = (int)(t % nblk), bi = 0;
  while (rem >= nbk - bi) { rem -= nbk - bi; ++bi; }
  const int bj = bi + rem;
  const long AB = (long)na * nb;
  const IOT<P>* X = bh + (long)q * AB;
  const int mu0 = bi * Cfg::BM, nu0 = bj * Cfg::BN;
  XCS<P, IOT<P>, Cfg::BM, Cfg::NT> la;
  la.init(X, nb, na, [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
  XCS<P, IOT<P>, Cfg::BN, Cfg::NT> lb;
  lb.init(X, nb, na, [&](int x, long& o) { o = nu0 + x; return nu0 + x < nb; });
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem);
  const long B2 = (long)nb * nb;
  IOT<P>* K = Kn + (long)q * B2;
  acc.for_each([&](int m, int n, double v) {
    const int mu = mu0 + m, nu = nu0 + n;
    if (mu < nb && nu < nb) {
      if (mu <= nu) K[(long)mu * nb + nu] = (IOT<P>)v;
      if (mu < nu) K[(long)nu * nb + mu] = (IOT<P>)v;
    }
  });
}

// FP64 GEMM out[m][n] = sum_k A[k][m] B[k][n], both operands x-contiguous;
// used for H C_Omega and lambda = C^T Y.
template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_gemm_tn(int M, int N, int K, const double* __restrict__ A,
                                                     long lda, const double* __restrict__ B, long ldb,
                                                     double* __restrict__ out, long ldo) {
  constexpr int P = kF64;
  ENGINE_TYPES;
  const int m0 = blockIdx.x * Cfg::BM, n0 = blockIdx.y * Cfg::BN;
  XCS<P, double, Cfg::BM, Cfg::NT> la;
  la.init(A, lda, K, [&](int x, long& o) { o = m0 + x; return m0 + x < M; });
  XCS<P, double, Cfg::BN, Cfg::NT> lb;
  lb.init(B, ldb, K, [&](int x, long& o) { o = n0 + x; return n0 + x < N; });
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(K, E::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    if (m0 + m < M && n0 + n < N) out[(long)(m0 + m) * ldo + n0 + n] = v;
  });
}

// Fock-apply, split over the slabs t of the stacked operand [J^0..J^{W-1}, K^0..K^{W-1}]:
//   Ypart[s][mu][q] = sum_{t in split s} sum_nu X_t[nu][mu] coef_t[q] C[nu][q]
// with X_t = J^t (coef A[q][t]) or K^{t-W} (coef B[q][t-W]).  M = mu, N = q,
// K = (t, nu), nu padded per slab to a multiple of the slice depth.
template <int P, class Cfg>
struct FockA {  // element (mu, nu) of slab t; X_t symmetric, so read row nu
  using E = typename EngineOf<P>::type;
  using T = IOT<P>;
  using G = XCS<P, T, Cfg::BM, Cfg::NT>;
  static constexpr int NP = G::NP, R = G::R, RR = G::RR, KV = E::KV, BK = E::BK;
  using type = T;
  G g;
  const T *Jn, *Kn;
  int nb, nw, t0, nchunk, mu;
  __device__ void init(const T* Jn_, const T* Kn_, int nb_, int nw_, int t0_, int mu0) {
    Jn = Jn_; Kn = Kn_; nb = nb_; nw = nw_; t0 = t0_; nchunk = (nb + BK - 1) / BK;
    g.x = threadIdx.x % Cfg::BM; g.kg = threadIdx.x / Cfg::BM;
    mu = mu0 + g.x; g.ok = mu < nb;
  }
  __device__ int xl(int p) const { return g.xl(p); }
  __device__ int kl(int p) const { return g.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return g.ok && (kt % nchunk) * BK + g.kl(p) + i < nb; }
  __device__ void fetch(int kt, T (&r)[RR]) const {
    const int t = t0 + kt / nchunk, nu0 = (kt % nchunk) * BK;
    const T* X = (t < nw ? Jn + (long)t * nb * nb : Kn + (long)(t - nw) * nb * nb);
    const int muc = g.ok ? mu : 0;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        const int nu = nu0 + g.kl(p) + i;
        r[p * KV + i] = X[(long)(nu < nb ? nu : nb - 1) * nb + muc];
      }
  }
  __device__ double val(const T (&r)[RR], int p, int i) const { return (double)r[p * KV + i]; }
};

template <int P, class Cfg>
struct FockB {  // element (q, nu) of slab t: coef_t[q] * C[nu][q]; r[R] holds coef_t[q]
  using E = typename EngineOf<P>::type;
  using G = XCS<P, double, Cfg::BN, Cfg::NT>;
  static constexpr int NP = G::NP, R = G::R, RR = G::R + 1, KV = E::KV, BK = E::BK;
  using type = double;
  G g;
  const double *Ac, *Bc, *C;
  int nb, nw, nmo, t0, nchunk, q;
  __device__ void init(const double* Ac_, const double* Bc_, const double* C_, int nb_, int nw_, int nmo_,
                       int t0_, int q0) {
    Ac = Ac_; Bc = Bc_; C = C_; nb = nb_; nw = nw_; nmo = nmo_; t0 = t0_;
    nchunk = (nb + BK - 1) / BK;
    g.x = threadIdx.x % Cfg::BN; g.kg = threadIdx.x / Cfg::BN;
    q = q0 + g.x; g.ok = q < nw;
  }
  __device__ int xl(int p) const { return g.xl(p); }
  __device__ int kl(int p) const { return g.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return g.ok && (kt % nchunk) * BK + g.kl(p) + i < nb; }
  __device__ void fetch(int kt, double (&r)[RR]) const {
    const int t = t0 + kt / nchunk, nu0 = (kt % nchunk) * BK;
    const int qc = g.ok ? q : 0;
    r[R] = t < nw ? Ac[(long)qc * nw + t] : Bc[(long)qc * nw + (t - nw)];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        const int nu = nu0 + g.kl(p) + i;
        r[p * KV + i] = C[(long)(nu < nb ? nu : nb - 1) * nmo + qc];
      }
  }
  __device__ double val(const double (&r)[RR], int p, int i) const { return r[R] * r[p * KV + i]; }
};

template <int P, class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_fock(int nb, int nw, int nmo, int per,
                                                  const IOT<P>* __restrict__ Jn,
                                                  const IOT<P>* __restrict__ Kn,
                                                  const double* __restrict__ Ac,
                                                  const double* __restrict__ Bc,
                                                  const double* __restrict__ C,
                                                  double* __restrict__ Ypart) {
  ENGINE_TYPES;
  const int mu0 = blockIdx.x * Cfg::BM, q0 = blockIdx.y * Cfg::BN, s = blockIdx.z;
  const int t0 = s * per, t1 = min(2 * nw, t0 + per);
  FockA<P, Cfg> la;
  la.init(Jn, Kn, nb, nw, t0, mu0);
  FockB<P, Cfg> lb;
  lb.init(Ac, Bc, C, nb, nw, nmo, t0, q0);
  Acc acc;
  gemm_mainloop<E, Cfg>(la, lb, (t1 - t0) * la.nchunk, acc, smem);
  double* Y = Ypart + (long)s * nb * nw;
  acc.for_each([&](int m, int n, double v) {
    if (mu0 + m < nb && q0 + n < nw) Y[(long)(mu0 + m) * nw + q0 + n] = v;
  });
}

// MO J/K partial sums over a contiguous range of l (fixed split), then a
// fixed-order reduction over the splits.  FP64 arithmetic in every mode.
template <class T>
__global__ __launch_bounds__(256) void k_jk_mo_partial(int na, int nw, int nsplit, const T* __restrict__ bmo,
                                                       const double* __restrict__ d,
                                                       double* __restrict__ part) {
  const long w2 = (long)nw * nw;
  const long pq = (long)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (pq >= w2) return;
  const int l0 = (int)((long)na * s / nsplit), l1 = (int)((long)na * (s + 1) / nsplit);
  const int p = (int)(pq / nw), q = (int)(pq - (long)p * nw);
  double sj = 0.0, sk = 0.0;
  for (int l = l0; l < l1; ++l) {
    const double v = (double)bmo[(long)l * w2 + pq];
    sk = fma(v, v, sk);
    sj = fma(d[(long)l * nw + p], d[(long)l * nw + q], sj);
  }
  part[(2L * s) * w2 + pq] = sj;
  part[(2L * s + 1) * w2 + pq] = sk;
}

__global__ __launch_bounds__(256) void k_jk_mo_reduce(int nw, int nsplit, const double* __restrict__ part,
                                                      double* __restrict__ J, double* __restrict__ K) {
  const long w2 = (long)nw * nw;
  const long pq = (long)blockIdx.x * 256 + threadIdx.x;
  if (pq >= w2) return;
  double sj = 0.0, sk = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    sj += part[(2L * s) * w2 + pq];
    sk += part[(2L * s + 1) * w2 + pq];
  }
  J[pq] = sj;
  K[pq] = sk;
}

// Pair index of orbital p of Omega (explicit map or the default one).
__device__ __forceinline__ int pair_index(const int* pair_of, int p, int npairs, int ncwo) {
  if (pair_of) return pair_of[p];
  return p < npairs ? p : npairs - 1 - (p - npairs) / ncwo;
}

// Coefficients A, B of E = 2 sum n_p H_pp + sum (A J + B K) (Eq. (2), PNOF7 or
// PNOF5 Delta/Pi), with one energy partial per workgroup (fixed order).
__global__ __launch_bounds__(256) void k_coef(int functional, int nw, int npairs, int ncwo,
                                              const int* __restrict__ pair_of,
                                              const double* __restrict__ occ,
                                              const double* __restrict__ J, const double* __restrict__ K,
                                              double* __restrict__ Ac, double* __restrict__ Bc,
                                              double* __restrict__ epart) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const long w2 = (long)nw * nw;
  const long idx = (long)blockIdx.x * 256 + tid;
  double e = 0.0;
  if (idx < w2) {
    const int p = (int)(idx / nw), q = (int)(idx - (long)p * nw);
    const double np = occ[p], nq = occ[q];
    const int gp = pair_index(pair_of, p, npairs, ncwo), gq = pair_index(pair_of, q, npairs, ncwo);
    double a, bb;
    if (gp == gq) {
      a = 0.0;
      if (p == q) bb = np;
      else if (p >= npairs && q >= npairs) bb = sqrt(np * nq);
      else bb = -sqrt(np * nq);
    } else {
      a = 2.0 * np * nq;
      bb = -np * nq;
      if (functional == RIF_PNOF7) bb -= sqrt(np * (1.0 - np)) * sqrt(nq * (1.0 - nq));
    }
    Ac[idx] = a;
    Bc[idx] = bb;
    e = a * J[idx] + bb * K[idx];
  }
  red[tid] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) epart[blockIdx.x] = red[0];
}

// H_pp = c_p^T H c_p, the energy (coefficient partials + 2 sum n_p H_pp, fixed
// order) and the device-side validation of the occupations.  One workgroup.
__global__ __launch_bounds__(256) void k_energy(int nw, int npairs, int ncwo, int nb, int nmo, int nparts,
                                                const int* __restrict__ pair_of,
                                                const double* __restrict__ occ,
                                                const double* __restrict__ C,
                                                const double* __restrict__ HC,
                                                const double* __restrict__ epart,
                                                double* __restrict__ energy, int* __restrict__ flag) {
  constexpr int kStage = 2048;
  __shared__ double socc[kStage];
  __shared__ int spair[kStage];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const bool staged = nw <= kStage;
  if (staged) {
    for (int p = tid; p < nw; p += 256) {
      socc[p] = occ[p];
      spair[p] = pair_index(pair_of, p, npairs, ncwo);
    }
  }
  __syncthreads();
  int bad = 0;
  for (int p = tid; p < nw; p += 256) {
    const double n = staged ? socc[p] : occ[p];
    if (!(n >= 0.0 && n <= 1.0)) bad |= kBadOcc;
    const int g = staged ? spair[p] : pair_index(pair_of, p, npairs, ncwo);
    if (g < 0 || g >= npairs || (p < npairs && g != p)) bad |= kBadMap;
  }
  for (int g = tid; g < npairs; g += 256) {
    double s = 0.0;
    int cnt = 0;
    for (int p = 0; p < nw; ++p) {
      const int gp = staged ? spair[p] : pair_index(pair_of, p, npairs, ncwo);
      if (gp == g) { s += staged ? socc[p] : occ[p]; ++cnt; }
    }
    if (!(fabs(s - 1.0) <= 1e-12)) bad |= kBadSum;
    if (cnt != 1 + ncwo) bad |= kBadCount;
  }
  if (bad) atomicOr(flag, bad);

  double e = 0.0;
  for (int i = tid; i < nparts; i += 256) e += epart[i];
  // H_pp: one wave per orbital, lanes over mu, fixed-order butterfly
  const int lane = tid & 63, wave = tid >> 6;
  for (int p = wave; p < nw; p += 4) {
    double h = 0.0;
    for (int mu = lane; mu < nb; mu += 64) h = fma(C[(long)mu * nmo + p], HC[(long)mu * nw + p], h);
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
    if (lane == 0) e += 2.0 * occ[p] * h;
  }
  red[tid] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) energy[0] = red[0];
}

__global__ __launch_bounds__(256) void k_fock_reduce(int nb, int nw, int nsplit, const double* __restrict__ part,
                                                     const double* __restrict__ occ,
                                                     const double* __restrict__ HC, double* __restrict__ Y) {
  const long n = (long)nb * nw;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int q = (int)(i % nw);
  double y = occ[q] * HC[i];
  for (int s = 0; s < nsplit; ++s) y += part[(long)s * n + i];
  Y[i] = y;
}

// G[a][b] = 4 (L[a][b] - L[b][a]),  L[a][b] = lambda[a][b] for b < n_omega, else 0.
__global__ __launch_bounds__(256) void k_grad(int nmo, int nw, const double* __restrict__ lam,
                                              double* __restrict__ G) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)nmo * nmo) return;
  const int a = (int)(i / nmo), b = (int)(i - (long)a * nmo);
  const double lab = b < nw ? lam[(long)a * nw + b] : 0.0;
  const double lba = a < nw ? lam[(long)b * nw + a] : 0.0;
  G[i] = 4.0 * (lab - lba);
}

// ---------------------------------------------------------------------------
// Launchers.  Each GEMM-shaped kernel exists in four tile variants per mode:
//   0: 128x128   1: 64x64   2: 128x64   3: 64x128   (outputs per workgroup)
// pick_variant() chooses one per (kernel, mode, shape): a wave-quantisation
// model by default, or the fastest measured one when autotuning is on.

template <int BK> struct Vars;
template <> struct Vars<16> {  // FP64 / FP32 engines: 4 waves
  using V0 = TileCfg<128, 128, 16, 64, 64>;
  using V1 = TileCfg<64, 64, 16, 32, 32>;
  using V2 = TileCfg<128, 64, 16, 64, 32>;
  using V3 = TileCfg<64, 128, 16, 32, 64>;
};
template <> struct Vars<32> {  // BF16 split engines: smaller wave tiles (three accumulator sets)
  using V0 = TileCfg<128, 128, 32, 64, 32>;
  using V1 = TileCfg<64, 64, 32, 32, 32>;
  using V2 = TileCfg<128, 64, 32, 64, 32>;
  using V3 = TileCfg<64, 128, 32, 32, 64>;
};

template <int P, class F>
static decltype(auto) dispatch(int v, F&& f) {
  using VS = Vars<EngineOf<P>::type::BK>;
  switch (v) {
    case 0: return f(typename VS::V0());
    case 1: return f(typename VS::V1());
    case 2: return f(typename VS::V2());
    default: return f(typename VS::V3());
  }
}

static const char* kPrecName[4] = {"f64", "f32", "bf16x3", "bf16x6"};

// Relative time of a launch of `nwg` tiles of a variant with `wg_per_cu`
// resident workgroups per CU: whole rounds of 256*wg_per_cu tiles, each round
// as long as one tile running at 1/wg_per_cu of a CU.
static double est_cost(long nwg, int wg_per_cu, long tile_mn, double useful) {
  const long slots = 256L * wg_per_cu;
  const long rounds = (nwg + slots - 1) / slots;
  return (double)rounds * tile_mn * wg_per_cu / useful;
}
template <int P, class Cfg>
static int wg_per_cu() {
  using E = typename EngineOf<P>::type;
  const int lds = 163840 / smem_bytes<E, Cfg>();
  const int waves = 32 / Cfg::NWAVES;  // at most 8 waves per SIMD
  return std::max(1, std::min(std::min(lds, waves), 4));
}

template <class F>
static int best_of(int nvar, F&& cost) {
  double best = 1e300;
  int hv = 0;
  for (int v = 0; v < nvar; ++v) {
    const double e = cost(v);
    if (e < best) { best = e; hv = v; }
  }
  return hv;
}

template <int P>
static rif_status run_transform(rif_ctx* c, int nb, int na, int nw, int nmo, const double* b, const double* C,
                                IOT<P>* bh, IOT<P>* bmo, double* d) {
  const long nr = (long)na * nb, ns = (long)na * nw;
  auto runh = [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_half_transform<P, Cfg>), dim3(cdiv(nr, Cfg::BN), cdiv(nw, Cfg::BM)), dim3(Cfg::NT),
                         0, c->stream, nb, nr, nw, nmo, b, C, bh);
      return check_launch(c, "half_transform");
    });
  };
  int hv = best_of(4, [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const double useful = (double)nw / (cdiv(nw, Cfg::BM) * Cfg::BM);
      return est_cost((long)cdiv(nr, Cfg::BN) * cdiv(nw, Cfg::BM), wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful);
    });
  });
  int v = pick_variant(c, "half_transform", {P, nb, na, nw, nmo}, 4, hv, runh);
  if (v < 0) return RIF_EHIP;
  rif_status st;
  {
    ProfScope ps(c, "half_transform");
    if ((st = runh(v))) return st;
  }
  auto runm = [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_mo_transform<P, Cfg>), dim3(cdiv(ns, Cfg::BM), cdiv(nw, Cfg::BN)), dim3(Cfg::NT), 0,
                         c->stream, nb, na, nw, nmo, bh, C, bmo, d);
      return check_launch(c, "mo_transform");
    });
  };
  hv = best_of(4, [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const double useful = (double)nw / (cdiv(nw, Cfg::BN) * Cfg::BN);
      return est_cost((long)cdiv(ns, Cfg::BM) * cdiv(nw, Cfg::BN), wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful);
    });
  });
  v = pick_variant(c, "mo_transform", {P, nb, na, nw, nmo}, 4, hv, runm);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "mo_transform");
  return runm(v);
}

template <int P>
static rif_status run_jk_mo(rif_ctx* c, int na, int nw, const IOT<P>* bmo, const double* d, double* J, double* K) {
  const long w2 = (long)nw * nw;
  const int nx = cdiv(w2, 256);
  const int nsplit = (int)std::max(1L, std::min((long)na, (1024L + nx - 1) / nx));
  Carve cv;
  const size_t o_part = cv.take<double>(2L * nsplit * w2);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  double* part = (double*)((char*)c->ws + o_part);
  {
    ProfScope ps(c, "jk_mo_partial");
    hipLaunchKernelGGL(k_jk_mo_partial<IOT<P>>, dim3(nx, nsplit), dim3(256), 0, c->stream, na, nw, nsplit, bmo, d,
                       part);
  }
  if ((st = check_launch(c, "jk_mo_partial"))) return st;
  ProfScope ps(c, "jk_mo_reduce");
  hipLaunchKernelGGL(k_jk_mo_reduce, dim3(nx), dim3(256), 0, c->stream, nw, nsplit, part, J, K);
  return check_launch(c, "jk_mo_reduce");
}

template <int TMU, int TNU>
static long jao_active(int nb) {  // blocks that touch the upper triangle
  long n = 0;
  for (int bi = 0; bi < cdiv(nb, TMU); ++bi) n += std::max(0, cdiv(nb, TNU) - jao_first_col(bi, TMU, TNU));
  return n;
}

template <int P>
static rif_status run_jk_ao(rif_ctx* c, int nb, int na, int nw, const double* b, const IOT<P>* bh,
                            const double* d, IOT<P>* Jn, IOT<P>* Kn) {
  rif_status st;
  constexpr int TNU = 16;
  auto runj = [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const long n = jao_active<Cfg::BN / TNU, TNU>(nb) * cdiv(nw, Cfg::BM);
      hipLaunchKernelGGL((k_jao<P, Cfg, TNU>), dim3((unsigned)n), dim3(Cfg::NT), 0, c->stream, nb, na, nw, b, d, Jn);
      return check_launch(c, "jao");
    });
  };
  int hv = best_of(4, [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const long n = jao_active<Cfg::BN / TNU, TNU>(nb) * cdiv(nw, Cfg::BM);
      const double useful = (double)nw / (cdiv(nw, Cfg::BM) * Cfg::BM);
      return est_cost(n, wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful);
    });
  });
  int v = pick_variant(c, "jao", {P, nb, na, nw}, 4, hv, runj);
  if (v < 0) return RIF_EHIP;
  {
    ProfScope ps(c, "jao");
    if ((st = runj(v))) return st;
  }
  // K: square tiles only (variants 0 and 1)
  auto runk = [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      if constexpr (Cfg::BM == Cfg::BN) {
        const long nbk = cdiv(nb, Cfg::BM);
        hipLaunchKernelGGL((k_kao<P, Cfg>), dim3((unsigned)(nbk * (nbk + 1) / 2 * nw)), dim3(Cfg::NT), 0,
                           c->stream, nb, na, nw, bh, Kn);
        return check_launch(c, "kao");
      } else {
        return fail(c, RIF_ENOTSUP, "kao: non-square tile variant");
      }
    });
  };
  hv = best_of(2, [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const long nbk = cdiv(nb, Cfg::BM);
      const double useful = (double)nb * (nb + 1) / 2 / (nbk * (nbk + 1) / 2 * (double)Cfg::BM * Cfg::BM);
      return est_cost(nbk * (nbk + 1) / 2 * nw, wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful);
    });
  });
  v = pick_variant(c, "kao", {P, nb, na, nw}, 2, hv, runk);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "kao");
  return runk(v);
}

template <int P>
static rif_status run_energy_grad(rif_ctx* c, int functional, int nb, int nmo, int npairs, int ncwo,
                                  const int* pair_of, const double* H, const double* C, const double* occ,
                                  const double* J, const double* K, const IOT<P>* Jn, const IOT<P>* Kn,
                                  double* energy, double* lambda, double* grad) {
  const int nw = npairs * (1 + ncwo);
  using CS = Vars<16>::V1;
  const int slabs = 2 * nw;
  // split-K over the stacked slabs, sized so a 64x64-tile launch has >= 1024 tiles
  const int mt = cdiv(nb, 64), nt = cdiv(nw, 64);
  int nsplit = std::max(1, std::min(slabs, cdiv(1024, (long)mt * nt)));
  const int per = cdiv(slabs, nsplit);
  nsplit = cdiv(slabs, per);
  const int nparts = cdiv((long)nw * nw, 256);
  Carve cv;
  const size_t o_hc = cv.take<double>((size_t)nb * nw);
  const size_t o_a = cv.take<double>((size_t)nw * nw);
  const size_t o_b = cv.take<double>((size_t)nw * nw);
  const size_t o_yp = cv.take<double>((size_t)nsplit * nb * nw);
  const size_t o_y = cv.take<double>((size_t)nb * nw);
  const size_t o_ep = cv.take<double>((size_t)nparts);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  char* w = (char*)c->ws;
  double *HC = (double*)(w + o_hc), *Ac = (double*)(w + o_a), *Bc = (double*)(w + o_b);
  double *Yp = (double*)(w + o_yp), *Y = (double*)(w + o_y), *Ep = (double*)(w + o_ep);
  {
    ProfScope ps(c, "hc_gemm");
    hipLaunchKernelGGL(k_gemm_tn<CS>, dim3(cdiv(nb, CS::BM), cdiv(nw, CS::BN)), dim3(CS::NT), 0, c->stream,
                       nb, nw, nb, H, (long)nb, C, (long)nmo, HC, (long)nw);
  }
  if ((st = check_launch(c, "hc_gemm"))) return st;
  {
    ProfScope ps(c, "coef");
    hipLaunchKernelGGL(k_coef, dim3(nparts), dim3(256), 0, c->stream, functional, nw, npairs, ncwo, pair_of, occ,
                       J, K, Ac, Bc, Ep);
  }
  if ((st = check_launch(c, "coef"))) return st;
  {
    ProfScope ps(c, "energy");
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, c->stream, nw, npairs, ncwo, nb, nmo, nparts, pair_of, occ,
                       C, HC, Ep, energy, c->dflag);
  }
  if ((st = check_launch(c, "energy"))) return st;
  auto runf = [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_fock<P, Cfg>), dim3(cdiv(nb, Cfg::BM), cdiv(nw, Cfg::BN), nsplit), dim3(Cfg::NT), 0,
                         c->stream, nb, nw, nmo, per, Jn, Kn, Ac, Bc, C, Yp);
      return check_launch(c, "fock");
    });
  };
  const int hv = best_of(4, [&](int v) {
    return dispatch<P>(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      const long n = (long)cdiv(nb, Cfg::BM) * cdiv(nw, Cfg::BN) * nsplit;
      const double useful = (double)nb * nw / ((double)cdiv(nb, Cfg::BM) * Cfg::BM * cdiv(nw, Cfg::BN) * Cfg::BN);
      return est_cost(n, wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful);
    });
  });
  const int v = pick_variant(c, "fock", {P, nb, nw, nmo, nsplit}, 4, hv, runf);
  if (v < 0) return RIF_EHIP;
  {
    ProfScope ps(c, "fock");
    if ((st = runf(v))) return st;
  }
  {
    ProfScope ps(c, "fock_reduce");
    hipLaunchKernelGGL(k_fock_reduce, dim3(cdiv((long)nb * nw, 256)), dim3(256), 0, c->stream, nb, nw, nsplit,
                       Yp, occ, HC, Y);
  }
  if ((st = check_launch(c, "fock_reduce"))) return st;
  {
    ProfScope ps(c, "lambda_gemm");
    hipLaunchKernelGGL(k_gemm_tn<CS>, dim3(cdiv(nmo, CS::BM), cdiv(nw, CS::BN)), dim3(CS::NT), 0, c->stream,
                       nmo, nw, nb, C, (long)nmo, Y, (long)nw, lambda, (long)nw);
  }
  if ((st = check_launch(c, "lambda_gemm"))) return st;
  ProfScope ps(c, "grad");
  hipLaunchKernelGGL(k_grad, dim3(cdiv((long)nmo * nmo, 256)), dim3(256), 0, c->stream, nmo, nw, lambda, grad);
  return check_launch(c, "grad");
}

// ---- mode dispatch (the only entry points the ABI layer calls) ----
#define RIF_PREC_SWITCH(prec, call)                                              \
  switch (prec) {                                                                \
    case kF64: { constexpr int P = kF64; return call; }                          \
    case kF32: { constexpr int P = kF32; return call; }                          \
    case kBF16x3: { constexpr int P = kBF16x3; return call; }                    \
    case kBF16x6: { constexpr int P = kBF16x6; return call; }                    \
    default: return fail(c, RIF_ENOTSUP, "precision mode not available");       \
  }

rif_status op_transform(rif_ctx* c, int prec, int nb, int na, int nw, int nmo, const double* b, const double* C,
                        void* bh, void* bmo, double* d) {
  RIF_PREC_SWITCH(prec, run_transform<P>(c, nb, na, nw, nmo, b, C, (IOT<P>*)bh, (IOT<P>*)bmo, d))
}

rif_status op_jk_mo(rif_ctx* c, int prec, int na, int nw, const void* bmo, const double* d, double* J, double* K) {
  RIF_PREC_SWITCH(prec, run_jk_mo<P>(c, na, nw, (const IOT<P>*)bmo, d, J, K))
}

rif_status op_jk_ao(rif_ctx* c, int prec, int nb, int na, int nw, const double* b, const void* bh,
                    const double* d, void* Jn, void* Kn) {
  RIF_PREC_SWITCH(prec, run_jk_ao<P>(c, nb, na, nw, b, (const IOT<P>*)bh, d, (IOT<P>*)Jn, (IOT<P>*)Kn))
}

rif_status op_energy_grad(rif_ctx* c, int prec, int functional, int nb, int nmo, int npairs, int ncwo,
                          const int* pair_of, const double* H, const double* C, const double* occ,
                          const double* J, const double* K, const void* Jn, const void* Kn, double* energy,
                          double* lambda, double* grad) {
  RIF_PREC_SWITCH(prec, run_energy_grad<P>(c, functional, nb, nmo, npairs, ncwo, pair_of, H, C, occ, J, K,
                                           (const IOT<P>*)Jn, (const IOT<P>*)Kn, energy, lambda, grad))
}

}  // namespace rif
