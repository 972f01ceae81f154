// FP64 kernels of the RI-PNOF7 hot path (gfx950, v_mfma_f64_16x16x4_f64).
//
//   half transform   Eq. (12), Table 3 step 2:  b_half[q][l][nu] = sum_mu C[mu][q] b[l][mu][nu]
//   MO transform     Eq. (13), Table 2 step 3:  b_mo[l][p][q] = sum_nu b_half[p][l][nu] C[nu][q]
//   MO J/K           Eqs. (10)-(11), Table 2 step 4
//   per-MO AO J/K    Table 3 steps 3-4
//   energy           Eq. (2) with L = K
//   Lagrangian       F^(q) c_q, lambda = C^T Y, G = 4 (lambda - lambda^T)
//
// GEMM-shaped steps share the tile engine in mfma_f64.hpp; each kernel
// supplies operand loaders that describe its own layout in HBM.  Sums that
// cross workgroups are written as partials and reduced in a fixed order, so
// every result is deterministic run to run.
#include <math.h>

#include "mfma_f64.hpp"
#include "rif_internal.hpp"

namespace rif {

using CfgL = TileCfg<128, 128, 16, 64, 64>;  // large tiles, 4 waves
using CfgS = TileCfg<64, 64, 16, 32, 32>;    // small tiles, 4 waves

template <class Cfg>
using XC = XCLoader<Cfg::BM, Cfg::BK, Cfg::NT>;
template <class Cfg>
using XCn = XCLoader<Cfg::BN, Cfg::BK, Cfg::NT>;
template <class Cfg>
using KCm = KCLoader<Cfg::BM, Cfg::BK, Cfg::NT>;
template <class Cfg>
using KCn = KCLoader<Cfg::BN, Cfg::BK, Cfg::NT>;

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

// ---------------------------------------------------------------------------
// Half transform.  Since b[l] is symmetric, b[l][mu][nu] = b[l][nu][mu] and the
// step is one GEMM: bh[q][r] = sum_mu C[mu][q] bflat[r][mu] with r = l*n_bf + nu.
// M = q, N = r (so stores run along r, contiguous in b_half), K = mu.
template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_half_transform(int nb, long nr, int nw, int nmo,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ C,
                                                            double* __restrict__ bh) {
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const int q0 = blockIdx.y * Cfg::BM;
  const long r0 = (long)blockIdx.x * Cfg::BN;
  XC<Cfg> la;
  la.init(C, nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  KCn<Cfg> lb;
  lb.init([&](int x) -> const double* {
    long r = r0 + x;
    return r < nr ? b + r * nb : nullptr;
  }, b, nb);
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, cdiv(nb, Cfg::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const int q = q0 + m;
    const long r = r0 + n;
    if (q < nw && r < nr) bh[(long)q * nr + r] = v;
  });
}

// MO transform: rows s = l*n_omega + p, bmo[s][q] = sum_nu bh[p][l][nu] C[nu][q];
// the diagonal d[l][p] = bmo[l][p][p] is emitted by the same epilogue.
template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_mo_transform(int nb, int na, int nw, int nmo,
                                                          const double* __restrict__ bh,
                                                          const double* __restrict__ C,
                                                          double* __restrict__ bmo,
                                                          double* __restrict__ d) {
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const long ns = (long)na * nw;
  const long s0 = (long)blockIdx.x * Cfg::BM;
  const int q0 = blockIdx.y * Cfg::BN;
  const long AB = (long)na * nb;
  KCm<Cfg> la;
  la.init([&](int x) -> const double* {
    const long s = s0 + x;
    if (s >= ns) return nullptr;
    const long l = s / nw, p = s - l * nw;
    return bh + p * AB + l * nb;
  }, bh, nb);
  XCn<Cfg> lb;
  lb.init(C, nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, cdiv(nb, Cfg::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const long s = s0 + m;
    const int q = q0 + n;
    if (s < ns && q < nw) {
      bmo[s * nw + q] = v;
      if (s % nw == q) d[s] = v;
    }
  });
}

// MO J/K partial sums over a contiguous range of l (fixed split), then a
// fixed-order reduction over the splits.
__global__ __launch_bounds__(256) void k_jk_mo_partial(int na, int nw, int nsplit,
                                                       const double* __restrict__ bmo,
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
    const double v = bmo[(long)l * w2 + pq];
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

// Per-MO AO Coulomb: Jn[q][mu][nu] = sum_l d[l][q] b[l][mu][nu].
// M = q, N = a TMU x TNU block of (mu, nu), K = l.  Only blocks that touch the
// upper triangle run; each writes (mu<=nu) directly and (mu<nu) mirrored, so
// every element of the full matrix is written exactly once.
// First block column of block row bi that holds an element with nu >= mu.
__host__ __device__ __forceinline__ int jao_first_col(int bi, int tmu, int tnu) {
  const int t = bi * tmu - (tnu - 1);
  return t <= 0 ? 0 : (t + tnu - 1) / tnu;
}

template <class Cfg, int TNU>
__global__ __launch_bounds__(Cfg::NT) void k_jao(int nb, int na, int nw, const double* __restrict__ b,
                                                 const double* __restrict__ d,
                                                 double* __restrict__ Jn) {
  constexpr int TMU = Cfg::BN / TNU;
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const int nbj = (nb + TNU - 1) / TNU;
  const int nbi = (nb + TMU - 1) / TMU;
  const long nq = (nw + Cfg::BM - 1) / Cfg::BM;
  // The grid enumerates only blocks that touch the upper triangle, q-tile
  // fastest, so the XCD remap spreads equal work over the XCDs and q-tiles
  // that share a b block run on one XCD.
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
  XC<Cfg> la;
  la.init(d, nw, na, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  XCn<Cfg> lb;
  lb.init(b, B2, na, [&](int x, long& o) {
    const int mu = mu0 + x / TNU, nu = nu0 + x % TNU;
    o = (long)mu * nb + nu;
    return mu < nb && nu < nb;
  });
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, cdiv(na, Cfg::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    const int q = q0 + m, mu = mu0 + n / TNU, nu = nu0 + n % TNU;
    if (q < nw && mu < nb && nu < nb) {
      double* J = Jn + (long)q * B2;
      if (mu <= nu) J[(long)mu * nb + nu] = v;
      if (mu < nu) J[(long)nu * nb + mu] = v;
    }
  });
}

// Per-MO AO exchange: Kn[q] = X_q^T X_q with X_q = b_half[q] ([n_aux][n_bf]).
// Square blocks (bi <= bj) only, mirrored like k_jao.
template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_kao(int nb, int na, int nw, const double* __restrict__ bh,
                                                 double* __restrict__ Kn) {
  static_assert(Cfg::BM == Cfg::BN, "square blocks");
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const int nbk = (nb + Cfg::BM - 1) / Cfg::BM;
  const long nblk = (long)nbk * (nbk + 1) / 2;  // upper-triangle blocks per q
  const long t = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int q = (int)(t / nblk);
  if (q >= nw) return;
  int rem = (int)(t % nblk), bi = 0;
  while (rem >= nbk - bi) { rem -= nbk - bi; ++bi; }
  const int bj = bi + rem;
  const long AB = (long)na * nb;
  const double* X = bh + (long)q * AB;
  const int mu0 = bi * Cfg::BM, nu0 = bj * Cfg::BN;
  XC<Cfg> la;
  la.init(X, nb, na, [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
  XCn<Cfg> lb;
  lb.init(X, nb, na, [&](int x, long& o) { o = nu0 + x; return nu0 + x < nb; });
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, cdiv(na, Cfg::BK), acc, smem);
  const long B2 = (long)nb * nb;
  double* K = Kn + (long)q * B2;
  acc.for_each([&](int m, int n, double v) {
    const int mu = mu0 + m, nu = nu0 + n;
    if (mu < nb && nu < nb) {
      if (mu <= nu) K[(long)mu * nb + nu] = v;
      if (mu < nu) K[(long)nu * nb + mu] = v;
    }
  });
}

// Plain GEMM out[m][n] = sum_k A[k][m] B[k][n] with both operands x-contiguous
// (A = H or C, B = C or Y); used for H C_Omega and lambda = C^T Y.
template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_gemm_tn(int M, int N, int K, const double* __restrict__ A,
                                                     long lda, const double* __restrict__ B, long ldb,
                                                     double* __restrict__ out, long ldo) {
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const int m0 = blockIdx.x * Cfg::BM, n0 = blockIdx.y * Cfg::BN;
  XC<Cfg> la;
  la.init(A, lda, K, [&](int x, long& o) { o = m0 + x; return m0 + x < M; });
  XCn<Cfg> lb;
  lb.init(B, ldb, K, [&](int x, long& o) { o = n0 + x; return n0 + x < N; });
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, cdiv(K, Cfg::BK), acc, smem);
  acc.for_each([&](int m, int n, double v) {
    if (m0 + m < M && n0 + n < N) out[(long)(m0 + m) * ldo + n0 + n] = v;
  });
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

// Fock-apply, split over the slabs t of the stacked operand [J^0..J^{W-1}, K^0..K^{W-1}]:
//   Ypart[s][mu][q] = sum_{t in split s} sum_nu X_t[nu][mu] coef_t[q] C[nu][q]
// with X_t = J^t (coef A[q][t]) or K^{t-W} (coef B[q][t-W]).  M = mu, N = q,
// K = (t, nu), nu padded per slab to a multiple of BK.
template <class Cfg>
struct FockA {  // element (mu, nu) of slab t; X_t symmetric so read row nu
  XCLoader<Cfg::BM, Cfg::BK, Cfg::NT> g;
  static constexpr int R = XCLoader<Cfg::BM, Cfg::BK, Cfg::NT>::R;
  static constexpr int RR = R;
  const double *Jn, *Kn;
  int nb, nw, t0, nchunk, mu;
  bool ok;
  __device__ void init(const double* Jn_, const double* Kn_, int nb_, int nw_, int t0_, int mu0) {
    Jn = Jn_; Kn = Kn_; nb = nb_; nw = nw_; t0 = t0_; nchunk = (nb + Cfg::BK - 1) / Cfg::BK;
    g.x = threadIdx.x % Cfg::BM; g.kx = threadIdx.x / Cfg::BM;
    mu = mu0 + g.x; ok = mu < nb;
  }
  __device__ void fetch(int kt, double (&r)[R]) const {
    const int t = t0 + kt / nchunk, nu0 = (kt % nchunk) * Cfg::BK;
    const double* X = (t < nw ? Jn + (long)t * nb * nb : Kn + (long)(t - nw) * nb * nb);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int nu = nu0 + g.kx + j * g.KSTEP;
      r[j] = X[(long)(nu < nb ? nu : nb - 1) * nb + (ok ? mu : 0)];
    }
  }
  __device__ void stash(lds_f64* S, const double (&r)[R], int kt) const {
    const int nu0 = (kt % nchunk) * Cfg::BK;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int nu = nu0 + g.kx + j * g.KSTEP;
      S[(g.kx + j * g.KSTEP) * (Cfg::BM + kPadF64) + g.x] = (ok && nu < nb) ? r[j] : 0.0;
    }
  }
};

template <class Cfg>
struct FockB {  // element (q, nu) of slab t: coef_t[q] * C[nu][q]
  XCLoader<Cfg::BN, Cfg::BK, Cfg::NT> g;
  static constexpr int R = XCLoader<Cfg::BN, Cfg::BK, Cfg::NT>::R;
  const double *Ac, *Bc, *C;
  int nb, nw, nmo, t0, nchunk, q;
  bool ok;
  __device__ void init(const double* Ac_, const double* Bc_, const double* C_, int nb_, int nw_, int nmo_,
                       int t0_, int q0) {
    Ac = Ac_; Bc = Bc_; C = C_; nb = nb_; nw = nw_; nmo = nmo_; t0 = t0_;
    nchunk = (nb + Cfg::BK - 1) / Cfg::BK;
    g.x = threadIdx.x % Cfg::BN; g.kx = threadIdx.x / Cfg::BN;
    q = q0 + g.x; ok = q < nw;
  }
  // r[0..R-1] = C elements, r[R] = the slab coefficient for this column
  static constexpr int RR = R + 1;
  __device__ void fetch(int kt, double (&r)[R + 1]) const {
    const int t = t0 + kt / nchunk, nu0 = (kt % nchunk) * Cfg::BK;
    const int qc = ok ? q : 0;
    r[R] = t < nw ? Ac[(long)qc * nw + t] : Bc[(long)qc * nw + (t - nw)];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int nu = nu0 + g.kx + j * g.KSTEP;
      r[j] = C[(long)(nu < nb ? nu : nb - 1) * nmo + qc];
    }
  }
  __device__ void stash(lds_f64* S, const double (&r)[R + 1], int kt) const {
    const int nu0 = (kt % nchunk) * Cfg::BK;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int nu = nu0 + g.kx + j * g.KSTEP;
      S[(g.kx + j * g.KSTEP) * (Cfg::BN + kPadF64) + g.x] = (ok && nu < nb) ? r[R] * r[j] : 0.0;
    }
  }
};

template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_fock(int nb, int nw, int nmo, int per,
                                                  const double* __restrict__ Jn,
                                                  const double* __restrict__ Kn,
                                                  const double* __restrict__ Ac,
                                                  const double* __restrict__ Bc,
                                                  const double* __restrict__ C,
                                                  double* __restrict__ Ypart) {
  __shared__ double smem[Cfg::SMEM_DOUBLES];
  const int mu0 = blockIdx.x * Cfg::BM, q0 = blockIdx.y * Cfg::BN, s = blockIdx.z;
  const int t0 = s * per, t1 = min(2 * nw, t0 + per);
  FockA<Cfg> la;
  la.init(Jn, Kn, nb, nw, t0, mu0);
  FockB<Cfg> lb;
  lb.init(Ac, Bc, C, nb, nw, nmo, t0, q0);
  Acc<Cfg> acc;
  gemm_mainloop<Cfg>(la, lb, (t1 - t0) * la.nchunk, acc, smem);
  double* Y = Ypart + (long)s * nb * nw;
  acc.for_each([&](int m, int n, double v) {
    if (mu0 + m < nb && q0 + n < nw) Y[(long)(mu0 + m) * nw + q0 + n] = v;
  });
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
// Launchers.  Each GEMM-shaped kernel exists in a few tile variants:
//   0: 128x128 (4 waves of 64x64)   1: 64x64 (4 waves of 32x32)
//   2: 128x64  (4 waves of 64x32)   3: 64x128 (4 waves of 32x64)
// pick_variant() chooses one per (kernel, shape): a wave-quantisation
// heuristic by default, or the fastest measured one when autotuning is on.

using V0 = TileCfg<128, 128, 16, 64, 64>;
using V1 = TileCfg<64, 64, 16, 32, 32>;
using V2 = TileCfg<128, 64, 16, 64, 32>;
using V3 = TileCfg<64, 128, 16, 32, 64>;

// workgroups of each variant that fit on one CU (LDS-limited)
static const int kWgPerCu[4] = {2, 4, 2, 2};
static const int kTileM[4] = {128, 64, 128, 64};
static const int kTileN[4] = {128, 64, 64, 128};

// Relative time of a launch of `nwg` tiles of variant v: whole rounds of
// 256*k concurrent tiles, each round as long as one tile at 1/k of a CU.
static double est_cost(int v, long nwg, double useful) {
  const long slots = 256L * kWgPerCu[v];
  const long rounds = (nwg + slots - 1) / slots;
  return (double)rounds * kTileM[v] * kTileN[v] * kWgPerCu[v] / useful;
}

template <class F>
static decltype(auto) dispatch(int v, F&& f) {
  switch (v) {
    case 0: return f(V0());
    case 1: return f(V1());
    case 2: return f(V2());
    default: return f(V3());
  }
}

// ---- half transform
template <class Cfg>
static long half_tiles(int nb, int na, int nw) {
  return (long)cdiv((long)na * nb, Cfg::BN) * cdiv(nw, Cfg::BM);
}
template <class Cfg>
static void launch_half(rif_ctx* c, int nb, int na, int nw, int nmo, const double* b, const double* C,
                        double* bh) {
  const long nr = (long)na * nb;
  dim3 grid(cdiv(nr, Cfg::BN), cdiv(nw, Cfg::BM));
  hipLaunchKernelGGL(k_half_transform<Cfg>, grid, dim3(Cfg::NT), 0, c->stream, nb, nr, nw, nmo, b, C, bh);
}

rif_status f64_half_transform(rif_ctx* c, int nb, int na, int nw, int nmo, const double* b,
                              const double* C, double* bh) {
  auto run = [&](int v) {
    return dispatch(v, [&](auto cfg) {
      launch_half<decltype(cfg)>(c, nb, na, nw, nmo, b, C, bh);
      return check_launch(c, "half_transform");
    });
  };
  double best = 1e300;
  int hv = 0;
  for (int v = 0; v < 4; ++v) {
    const double useful = (double)nw / (cdiv(nw, kTileM[v]) * kTileM[v]);
    const long n = dispatch(v, [&](auto cfg) { return half_tiles<decltype(cfg)>(nb, na, nw); });
    const double e = est_cost(v, n, useful);
    if (e < best) { best = e; hv = v; }
  }
  const int v = pick_variant(c, "half_transform", {nb, na, nw, nmo}, 4, hv, run);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "half_transform");
  return run(v);
}

// ---- MO transform
template <class Cfg>
static void launch_mo(rif_ctx* c, int nb, int na, int nw, int nmo, const double* bh, const double* C,
                      double* bmo, double* d) {
  const long ns = (long)na * nw;
  dim3 grid(cdiv(ns, Cfg::BM), cdiv(nw, Cfg::BN));
  hipLaunchKernelGGL(k_mo_transform<Cfg>, grid, dim3(Cfg::NT), 0, c->stream, nb, na, nw, nmo, bh, C, bmo, d);
}

rif_status f64_mo_transform(rif_ctx* c, int nb, int na, int nw, int nmo, const double* bh,
                            const double* C, double* bmo, double* d) {
  auto run = [&](int v) {
    return dispatch(v, [&](auto cfg) {
      launch_mo<decltype(cfg)>(c, nb, na, nw, nmo, bh, C, bmo, d);
      return check_launch(c, "mo_transform");
    });
  };
  double best = 1e300;
  int hv = 0;
  for (int v = 0; v < 4; ++v) {
    const long n = (long)cdiv((long)na * nw, kTileM[v]) * cdiv(nw, kTileN[v]);
    const double useful = (double)nw / (cdiv(nw, kTileN[v]) * kTileN[v]);
    const double e = est_cost(v, n, useful);
    if (e < best) { best = e; hv = v; }
  }
  const int v = pick_variant(c, "mo_transform", {nb, na, nw, nmo}, 4, hv, run);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "mo_transform");
  return run(v);
}

rif_status f64_jk_mo(rif_ctx* c, int na, int nw, const double* bmo, const double* d, double* J,
                     double* K) {
  const long w2 = (long)nw * nw;
  const int nx = cdiv(w2, 256);
  int nsplit = (int)std::max(1L, std::min((long)na, (1024L + nx - 1) / nx));
  Carve cv;
  size_t o_part = cv.take<double>(2L * nsplit * w2);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  double* part = (double*)((char*)c->ws + o_part);
  {
    ProfScope ps(c, "jk_mo_partial");
    hipLaunchKernelGGL(k_jk_mo_partial, dim3(nx, nsplit), dim3(256), 0, c->stream, na, nw, nsplit, bmo, d, part);
  }
  if ((st = check_launch(c, "jk_mo_partial"))) return st;
  ProfScope ps(c, "jk_mo_reduce");
  hipLaunchKernelGGL(k_jk_mo_reduce, dim3(nx), dim3(256), 0, c->stream, nw, nsplit, part, J, K);
  return check_launch(c, "jk_mo_reduce");
}

// ---- per-MO AO J and K
template <class Cfg>
static long jao_active(int nb, int nw) {  // tiles that touch the upper triangle
  constexpr int TNU = 16, TMU = Cfg::BN / TNU;
  long n = 0;
  for (int bi = 0; bi < cdiv(nb, TMU); ++bi) n += std::max(0, cdiv(nb, TNU) - jao_first_col(bi, TMU, TNU));
  return n * cdiv(nw, Cfg::BM);
}

rif_status f64_jk_ao(rif_ctx* c, int nb, int na, int nw, const double* b, const double* bh,
                     const double* d, double* Jn, double* Kn) {
  rif_status st;
  auto runj = [&](int v) {
    return dispatch(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_jao<Cfg, 16>), dim3((unsigned)jao_active<Cfg>(nb, nw)), dim3(Cfg::NT), 0, c->stream,
                         nb, na, nw, b, d, Jn);
      return check_launch(c, "jao");
    });
  };
  double best = 1e300;
  int hv = 0;
  for (int v = 0; v < 4; ++v) {
    const long n = dispatch(v, [&](auto cfg) { return jao_active<decltype(cfg)>(nb, nw); });
    const double useful = (double)nw / (cdiv(nw, kTileM[v]) * kTileM[v]);
    const double e = est_cost(v, n, useful);
    if (e < best) { best = e; hv = v; }
  }
  int v = pick_variant(c, "jao", {nb, na, nw}, 4, hv, runj);
  if (v < 0) return RIF_EHIP;
  {
    ProfScope ps(c, "jao");
    if ((st = runj(v))) return st;
  }
  // K: square tiles only (variants 0 and 1)
  auto runk = [&](int v) {
    return dispatch(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      if constexpr (Cfg::BM == Cfg::BN) {
        const long nbk = cdiv(nb, Cfg::BM);
        hipLaunchKernelGGL(k_kao<Cfg>, dim3((unsigned)(nbk * (nbk + 1) / 2 * nw)), dim3(Cfg::NT), 0, c->stream,
                           nb, na, nw, bh, Kn);
        return check_launch(c, "kao");
      } else {
        return fail(c, RIF_ENOTSUP, "kao: non-square tile variant");
      }
    });
  };
  best = 1e300;
  hv = 0;
  for (int v2 = 0; v2 < 2; ++v2) {
    const long nbk = cdiv(nb, kTileM[v2]);
    const double useful = (double)nb * (nb + 1) / 2 / (nbk * (nbk + 1) / 2 * (double)kTileM[v2] * kTileM[v2]);
    const double e = est_cost(v2, nbk * (nbk + 1) / 2 * nw, useful);
    if (e < best) { best = e; hv = v2; }
  }
  v = pick_variant(c, "kao", {nb, na, nw}, 2, hv, runk);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "kao");
  return runk(v);
}

rif_status f64_energy_grad(rif_ctx* c, int functional, int nb, int nmo, int npairs, int ncwo,
                           const int* pair_of, const double* H, const double* C, const double* occ,
                           const double* J, const double* K, const double* Jn, const double* Kn,
                           double* energy, double* lambda, double* grad) {
  const int nw = npairs * (1 + ncwo);
  using CS = V1;
  const int slabs = 2 * nw;
  // split-K over the stacked slabs; sized so a variant-0/1 launch has >= 1024 tiles
  const int mt = cdiv(nb, 64), nt = cdiv(nw, 64);
  int nsplit = std::max(1, std::min(slabs, cdiv(1024, (long)mt * nt)));
  const int per = cdiv(slabs, nsplit);
  nsplit = cdiv(slabs, per);
  Carve cv;
  const size_t o_hc = cv.take<double>((size_t)nb * nw);
  const size_t o_a = cv.take<double>((size_t)nw * nw);
  const size_t o_b = cv.take<double>((size_t)nw * nw);
  const size_t o_yp = cv.take<double>((size_t)nsplit * nb * nw);
  const size_t o_y = cv.take<double>((size_t)nb * nw);
  const int nparts = cdiv((long)nw * nw, 256);
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
    return dispatch(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL(k_fock<Cfg>, dim3(cdiv(nb, Cfg::BM), cdiv(nw, Cfg::BN), nsplit), dim3(Cfg::NT), 0,
                         c->stream, nb, nw, nmo, per, Jn, Kn, Ac, Bc, C, Yp);
      return check_launch(c, "fock");
    });
  };
  double best = 1e300;
  int hv = 1;
  for (int v = 0; v < 4; ++v) {
    const long n = (long)cdiv(nb, kTileM[v]) * cdiv(nw, kTileN[v]) * nsplit;
    const double useful = (double)nb * nw / (cdiv(nb, kTileM[v]) * kTileM[v] * (double)cdiv(nw, kTileN[v]) * kTileN[v]);
    const double e = est_cost(v, n, useful);
    if (e < best) { best = e; hv = v; }
  }
  const int v = pick_variant(c, "fock", {nb, nw, nmo, nsplit}, 4, hv, runf);
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

}  // namespace rif
