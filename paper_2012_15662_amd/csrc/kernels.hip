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

#include <atomic>
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
// pieces per operand in the split modes (0: the mode does not split)
template <int P>
constexpr int kPieces = P == kBF16x3 ? 2 : P == kBF16x6 ? 3 : P == kF16x3 ? 2 : 0;
// The mode's split of two values into its pieces (the staging path's arithmetic).
template <int P, int NPC>
__device__ __forceinline__ void split_mode(double d0, double d1, unsigned (&pc)[NPC]) {
  if constexpr (P == kF16x3) split_pair_f16(d0, d1, pc);
  else split_pair<NPC>(d0, d1, pc);
}
template <int P, int BX, int NT>
using PCS = PieceSrc<kPieces<P> ? kPieces<P> : 1, BX, 32, NT>;
template <int P, int BX, int NT>
using PDMA = PieceDma<kPieces<P> ? kPieces<P> : 1, BX, NT>;
// Which split-mode operands come from piece planes (measured): C_Omega in the
// MO transform in both modes; C_Omega in the half transform and d in J^q only
// with two pieces (with three, the 16-wave tiles spill under the 128-VGPR cap
// and staging the FP64 values directly is faster).
template <int P>
constexpr bool kPlanesMo = kPieces<P> > 0;
template <int P>
constexpr bool kPlanesHalfJao = kPieces<P> == 2;
constexpr int round32(int k) { return (k + 31) / 32 * 32; }
// Slices of global loads in flight in the two-piece modes' GEMMs whose
// operands are read without splitting VALU work or fit the register budget
// with a second load set (pre-split half transform and J^q, MO transform,
// K^q): two, since one slice's MFMA work is shorter than a load's latency.
// Elsewhere, and with three pieces, the second set would spill.
template <int P>
constexpr int kDeep = kPieces<P> == 2 ? 2 : 1;

// ---------------------------------------------------------------------------
// Per-step argument blocks.  Each step is written once as a tile function
// (a tile = one workgroup's share of the step, indexed by a linear id);
// single-molecule kernels map blockIdx to a tile, grouped kernels walk a
// work-list of tiles that spans many molecules (rif_batch_*).  The same tile
// code and tile shape give bitwise-identical results in both.

// Split-BF16 modes read C_Omega (half, mo) and d (J^q) as piece planes made once
// per call by the psplit step (PSplitArgs): row q of C_Omega^T or d^T, k
// contiguous, row length `ld`, planes `ps` elements apart.
struct Planes { const unsigned short* p; long ps; int ld; };
// Bs / bf: b given pre-split (bf16 piece planes with rows r = l*n_bf + nu, or
// an FP32 copy in b's layout); unset (null) means b is split on load.
// dma: FP64 operands staged by direct global -> LDS loads in the 128 x 128
// tile (set when every row of b and C starts 16-byte aligned and n_omega is even).
struct HalfArgs {
  int nb, nw, nmo; long nr; const double* b; const double* C; void* bh; Planes Cs; Planes Bs; const float* bf;
  int dma;
};
inline int half_dma_ok(int nb, int nmo, int nw, const double* b, const double* C) {
  return nb % 2 == 0 && nmo % 2 == 0 && nw % 2 == 0 && ((uintptr_t)b | (uintptr_t)C) % 16 == 0;
}
// b pre-split once per call: element (r, mu) = b[r*n_bf + mu] (row r = l*n_bf + nu;
// b symmetric) into the mode's pieces, rows zero-filled from n_bf up to ld;
// FP32 mode: a float copy.
struct BSplitArgs { const double* b; long nr; int nb, ld; void* out; long ps; };
// dma: FP64 128 x 128 tiles stage b_half and C_Omega by direct global -> LDS
// loads (even n_bf and n_mo, 16-byte aligned b_half and C).
struct MoArgs { int nb, na, nw, nmo; const void* bh; const double* C; void* bmo; double* d; Planes Cs; int dma; };
// Bj: b pre-split for J^q (piece planes with rows r = mu*n_bf + nu and
// k = l contiguous), or unset (split on load).
// dma: FP64 operands staged by direct global -> LDS loads in the 128 x 128
// tile (rows of b and d 16-byte aligned).
struct JaoArgs { int nb, na, nw; const double* b; const double* d; void* Jn; Planes Ds; Planes Bj; int dma; };
// Pre-split of X (element (x, k) at X[k*sk + x]) into NPC bf16 planes
// out[s*ps + x*ld + k], zero from k = K up to ld.
struct PSplitArgs { const double* X; long sk; int nx, K, ld; unsigned short* out; long ps; };
// dma: FP64 b_half staged by direct global -> LDS loads (rows 16-byte aligned).
struct KaoArgs { int nb, na, nw; const void* bh; void* Kn; int dma; };
// Split over k: out + s*ostride receives the partial product over
// k in [s*kc, min(K, (s+1)*kc)), s < ksplit.
struct GemmArgs {
  int M, N, K;
  const double* A; long lda;
  const double* B; long ldb;
  double* out; long ldo;
  int ksplit, kc; long ostride;
};
// dma: FP64 128 x 128 tiles stage J^q/K^q and C by direct global -> LDS loads
// (even n_bf, n_omega and n_mo, 16-byte aligned Jn, Kn and C).
struct FockArgs {
  int nb, nw, nmo, nsplit;
  const void *Jn, *Kn;
  const double *Ac, *Bc, *C;
  double* Yp;
  int dma;
};
struct JkArgs { int na, nw, nsplit; const void* bmo; const double* d; double* part; double* J; double* K; };
struct CoefArgs {
  int functional, nw, npairs, ncwo;
  const int* pair_of;
  const double *occ, *J, *K;
  double *Ac, *Bc, *Ep;
};
struct EnergyArgs {
  int nw, npairs, ncwo, nb, nmo, nparts;
  const int* pair_of;
  const double *occ, *C, *HC, *Ep;
  double* energy;
  int* flag;
};
struct FockRedArgs { int nb, nw, nsplit; const double *Yp, *occ, *HC; double* Y; };
// Gradient without per-MO AO matrices: Y[nu][q] = sum_{k=(r,l)} bh[r][l][nu] X[k][q] with
// X = Bt[q][r] * (r == q ? Zt[l][q] : bmo[l][r][q]), k = r*n_aux + l, split over k
// into nsplit ranges of kc; Zt, Bt (the mode's storage type) from k_ydz.
struct YdzArgs { int na, nw; const double *Ac, *Bc, *d; void *Zt, *Bt; };
struct YdArgs { int nb, na, nw, nsplit; long kc; const void *bh, *bmo, *Zt, *Bt; double* Yp; };
struct GradArgs { int nmo, nw, lsplit; const double* lp; double *lam, *G; int* flag; };

// Runs a tile's main loop, main(mma), and stores through store(m, n, v).  With
// kTrim (the grouped kernels, whose one tile shape serves molecules of every
// n_omega), in FP64 and FP32 a tile with at most half of its M fragment rows
// live (fim fragment rows of n_omega left in the last q-tile) trims each
// wave's fragment rows to the live ones under a balanced wave plan: the rows
// it computes are bitwise those of the full tile, and the rows it skips hold
// q >= n_omega, which are never stored.  Single-molecule launches pick their
// tile shape per molecule and run whole tiles: there trimming measured
// slower (those tiles stay load-bound with more rows live).
template <int P, class Cfg, bool kTrim, class Main, class Store>
__device__ __forceinline__ void run_q_rows(int fim, typename EngineOf<P>::type::template Acc<Cfg>& acc, Main&& main,
                                           Store&& store) {
  using E = typename EngineOf<P>::type;
  if constexpr (kTrim && (P == kF64 || P == kF32)) {
    if (2 * fim <= Cfg::BM / 16) {
      const WavePlan w = make_wave_plan<Cfg>([&](int I, int) { return I < fim; });
      with_rows<Cfg::TM>(w.ni, [&](auto rows) {
        constexpr int NI = decltype(rows)::value;
        main([&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
          E::template mma_rows<Cfg, NI>(SA, SB, c, w);
        });
      });
      acc.for_each(w, store);
      return;
    }
  }
  main([&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
    E::template mma<Cfg>(SA, SB, c, regular_plan<Cfg>());
  });
  acc.for_each(store);
}

// Half transform, Eq. (12): bh[q][r] = sum_mu C[mu][q] b[l][mu][nu] with the
// output column r = l*n_bf + nu flattened over (l, nu).  M = q, N = r (loads of
// b and stores of b_half both run along nu), K = mu.  Tiles: q-tile fastest.
template <int P, class Cfg>
__host__ __device__ inline long half_tiles(const HalfArgs& a) {
  return (long)cdiv(a.nw, Cfg::BM) * cdiv(a.nr, Cfg::BN);
}
template <int P, class Cfg, bool kBPre, bool kTrim>
__device__ void half_tile_with(const HalfArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  const int nqt = cdiv(a.nw, Cfg::BM);
  const int q0 = (int)(t % nqt) * Cfg::BM;
  const long r0 = (t / nqt) * Cfg::BN;
  const int nb = a.nb, nw = a.nw;
  const long nr = a.nr, B2 = (long)nb * nb;
  IOT<P>* bh = (IOT<P>*)a.bh;
  typename E::template Acc<Cfg> acc;
  auto slab_off = [&](int x, long& o) {   // column r = l*n_bf + nu of b at k = mu = 0
    const long r = r0 + x, l = r / nb;
    o = l * B2 + (r - l * nb);
    return r < nr;
  };
  auto store = [&](int m, int n, double v) {
    const int q = q0 + m;
    const long r = r0 + n;
    if (q < nw && r < nr) bh[(long)q * nr + r] = (IOT<P>)v;
  };
  const int fim = cdiv(nw - q0, 16);   // live fragment rows
  if constexpr (P == kF64 && !kBPre && Cfg::BM == 128 && Cfg::BN == 128) {
    if (a.dma) {
      XcDma64<Cfg::NT, E::BK, E::PAD> la, lb;
      la.init(a.C, a.nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
      lb.init(a.b, nb, nb, slab_off);
      if constexpr (kTrim) {
        run_q_rows<P, Cfg, kTrim>(fim, acc, [&](auto mma) {
          gemm_mainloop_dma_with<E, Cfg, 2>(la, lb, cdiv(nb, E::BK), acc, smem, false, mma);
        }, store);
      } else {
        gemm_mainloop_dma<E, Cfg, 2>(la, lb, cdiv(nb, E::BK), acc, smem);
        acc.for_each(store);
      }
      return;
    }
  }
  if constexpr (kBPre && kPieces<P> > 0) {
    // A: C_Omega^T (x = q, k = mu) from its per-call piece planes; B: column
    // r = l*n_bf + nu, piece-plane row r of the pre-split b (k = mu
    // contiguous, b symmetric).  Both staged by direct global -> LDS loads.
    PDMA<P, Cfg::BM, Cfg::NT> la;
    la.init(a.Cs.p, a.Cs.ps, a.Cs.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
    PDMA<P, Cfg::BN, Cfg::NT> lb;
    lb.init(a.Bs.p, a.Bs.ps, a.Bs.ld, [&](int x, long& o) { o = r0 + x; return r0 + x < nr; });
    gemm_mainloop_dma<E, Cfg>(la, lb, cdiv(nb, E::BK), acc, smem);
  } else {
    // A: C_Omega^T (x = q, k = mu), from piece planes in the two-piece modes
    typename std::conditional<kPlanesHalfJao<P>, PCS<P, Cfg::BM, Cfg::NT>, XCS<P, double, Cfg::BM, Cfg::NT>>::type la;
    if constexpr (kPlanesHalfJao<P>)
      la.init(a.Cs.p, a.Cs.ps, a.Cs.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
    else
      la.init(a.C, a.nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
    // B: column r = l*n_bf + nu of b[l][mu][nu] at k = mu: x-contiguous within
    // a slab (FP64 b, or FP32 mode's pre-made float copy at b's offsets)
    using LB = typename std::conditional<kBPre, XCS<P, float, Cfg::BN, Cfg::NT>, XCS<P, double, Cfg::BN, Cfg::NT>>::type;
    LB lb;
    if constexpr (kBPre)
      lb.init(a.bf, nb, nb, slab_off);
    else
      lb.init(a.b, nb, nb, slab_off);
    if constexpr (kTrim && kPieces<P> == 0) {
      run_q_rows<P, Cfg, kTrim>(fim, acc, [&](auto mma) {
        gemm_mainloop_with<E, Cfg>(la, lb, cdiv(nb, E::BK), acc, smem, false, mma);
      }, store);
      return;
    } else {
      gemm_mainloop<E, Cfg>(la, lb, cdiv(nb, E::BK), acc, smem);
    }
  }
  acc.for_each(store);
}
// Separate kernels for b split on load (half) and pre-split (halfp), so each
// keeps its own register budget.
template <int P, class Cfg>
__device__ void half_tile(const HalfArgs& a, long t, char* smem) { half_tile_with<P, Cfg, false, false>(a, t, smem); }
// The single-molecule pre-split half transform in the split modes runs
// persistent workgroups (one per resident slot, tiles strided by the grid),
// whose direct loads run ahead into the next tile while a tile's epilogue
// stores: each workgroup holds all of a CU's LDS, so a workgroup per tile left
// every tile boundary with the load pipe empty.  Results are bitwise those of
// one workgroup per tile (the same slices in the same order).
template <int P, class Cfg>
__device__ void halfp_persistent(const HalfArgs& a, long first, char* smem) {
  using E = typename EngineOf<P>::type;
  using LA = PDMA<P, Cfg::BM, Cfg::NT>;
  using LB = PDMA<P, Cfg::BN, Cfg::NT>;
  const int nb = a.nb, nw = a.nw;
  const long nr = a.nr;
  const int nqt = cdiv(nw, Cfg::BM);
  IOT<P>* bh = (IOT<P>*)a.bh;
  gemm_persistent_dma<E, Cfg, 0, LA, LB>(
      first, (long)gridDim.x, half_tiles<P, Cfg>(a), cdiv(nb, E::BK), smem,
      [&](long t, LA& la, LB& lb) {
        const int q0 = (int)(t % nqt) * Cfg::BM;
        const long r0 = (t / nqt) * Cfg::BN;
        la.init(a.Cs.p, a.Cs.ps, a.Cs.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
        lb.init(a.Bs.p, a.Bs.ps, a.Bs.ld, [&](int x, long& o) { o = r0 + x; return r0 + x < nr; });
      },
      [&](long t, const typename E::template Acc<Cfg>& acc) {
        const int q0 = (int)(t % nqt) * Cfg::BM;
        const long r0 = (t / nqt) * Cfg::BN;
        acc.for_each([&](int m, int n, double v) {
          const int q = q0 + m;
          const long r = r0 + n;
          if (q < nw && r < nr) bh[(long)q * nr + r] = (IOT<P>)v;
        });
      });
}
template <int P, class Cfg>
__device__ void halfp_tile(const HalfArgs& a, long t, char* smem) {
  if constexpr (kPieces<P> > 0)
    halfp_persistent<P, Cfg>(a, t, smem);
  else
    half_tile_with<P, Cfg, true, false>(a, t, smem);
}
template <int P, class Cfg>
__device__ void half_g_tile(const HalfArgs& a, long t, char* smem) { half_tile_with<P, Cfg, false, true>(a, t, smem); }
template <int P, class Cfg>
__device__ void halfp_g_tile(const HalfArgs& a, long t, char* smem) { half_tile_with<P, Cfg, true, true>(a, t, smem); }
template <int P, class Cfg>
__host__ __device__ inline long halfp_tiles(const HalfArgs& a) { return half_tiles<P, Cfg>(a); }
template <int P>
inline bool b_presplit(const HalfArgs& a) {
  return P != kF64 && (kPieces<P> > 0 ? a.Bs.p != nullptr : a.bf != nullptr);
}

// MO transform: rows s = l*n_omega + p, bmo[s][q] = sum_nu bh[p][l][nu] C[nu][q];
// the FP64 diagonal d[l][p] = bmo[l][p][p] comes from the same epilogue.
template <int P, class Cfg>
__host__ __device__ inline long mo_tiles(const MoArgs& a) {
  return (long)cdiv(a.nw, Cfg::BN) * cdiv((long)a.na * a.nw, Cfg::BM);
}
// FP64 slice of MFMAs with A in the swizzled [x][k] layout of KcDma64 and B in
// the engine's padded [k][x] layout.  Lane group kr of MFMA step (h, m) takes
// k = 2(kr + 4h) + m, so each lane reads its two A values of a step pair as
// one 16-byte chunk (eight lanes of one k group read eight rows' chunks in
// distinct bank slots); B is read at the same k.  Every k of the slice is
// summed once per slice, in a fixed order.
template <class Cfg>
__device__ __forceinline__ void mma_xk_f64(const lds_char* SA, const lds_char* SB,
                                           typename EngF64::template Acc<Cfg>& acc) {
  using E = EngF64;
  const lds_f64* As = (const lds_f64*)SA;
  const lds_f64* Bs = (const lds_f64*)SB;
  const int lane = threadIdx.x & 63, kr = lane >> 4, xc = lane & 15;
  int wm0, wn0;
  wave_origin(Cfg::WAVES_N, Cfg::WM, Cfg::WN, wm0, wn0);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = kr + 4 * h;   // chunk: k = 2c, 2c + 1
    double a0[Cfg::TM], a1[Cfg::TM];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i) {
      const int x = wm0 + i * 16 + xc;
      const lds_f64* q = As + x * 16 + 2 * (c ^ (x & 7));
      a0[i] = q[0];
      a1[i] = q[1];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double b[Cfg::TN];
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j) b[j] = Bs[(2 * c + m) * (Cfg::BN + E::PAD) + wn0 + j * 16 + xc];
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j)
          acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(m ? a1[i] : a0[i], b[j], acc.v[i][j], 0, 0, 0);
    }
  }
}

template <int P, class Cfg>
__device__ void mo_tile(const MoArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  const int nb = a.nb, na = a.na, nw = a.nw;
  const int nqt = cdiv(nw, Cfg::BN);
  const int q0 = (int)(t % nqt) * Cfg::BN;
  const long s0 = (t / nqt) * Cfg::BM;
  const long ns = (long)na * nw;
  const long AB = (long)na * nb;
  const IOT<P>* bh = (const IOT<P>*)a.bh;
  IOT<P>* bmo = (IOT<P>*)a.bmo;
  double* d = a.d;
  if constexpr (P == kF64 && Cfg::BM == 128 && Cfg::BN == 128) {
    if (a.dma) {   // b_half rows into the swizzled [x][k] layout, C_Omega into [k][x], both by direct loads
      KcDma64<Cfg::NT, E::BK, Cfg::BM> la;
      la.init([&](int x) -> const double* {
        const long s = s0 + x;
        if (s >= ns) return nullptr;
        const long l = s / nw, p = s - l * nw;
        return (const double*)bh + p * AB + l * nb;
      }, (const double*)bh, nb);
      XcDma64<Cfg::NT, E::BK, E::PAD> lb;
      lb.init(a.C, a.nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
      typename E::template Acc<Cfg> acc;
      gemm_mainloop_dma_with<E, Cfg, 2>(la, lb, cdiv(nb, E::BK), acc, smem, false,
                                        [&](const lds_char* SA, const lds_char* SB,
                                            typename E::template Acc<Cfg>& c) { mma_xk_f64<Cfg>(SA, SB, c); });
      acc.for_each([&](int m, int n, double v) {
        const long s = s0 + m;
        const int q = q0 + n;
        if (s < ns && q < nw) {
          bmo[s * nw + q] = v;
          if (s % nw == q) d[s] = v;
        }
      });
      return;
    }
  }
  KCS<P, IOT<P>, Cfg::BM, Cfg::NT> la;
  la.init([&](int x) -> const IOT<P>* {
    const long s = s0 + x;
    if (s >= ns) return nullptr;
    const long l = s / nw, p = s - l * nw;
    return bh + p * AB + l * nb;
  }, bh, nb);
  // B: C_Omega (x = q, k = nu), from piece planes in the split modes
  typename std::conditional<kPlanesMo<P>, PCS<P, Cfg::BN, Cfg::NT>, XCS<P, double, Cfg::BN, Cfg::NT>>::type lb;
  if constexpr (kPlanesMo<P>)
    lb.init(a.Cs.p, a.Cs.ps, a.Cs.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  else
    lb.init(a.C, a.nmo, nb, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  typename E::template Acc<Cfg> acc;
  gemm_mainloop<E, Cfg, kDeep<P>>(la, lb, cdiv(nb, E::BK), acc, smem);
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
constexpr int kJaoTNU = 16;
__host__ __device__ inline long jao_active(int nb, int tmu, int tnu) {  // blocks touching the upper triangle
  long n = 0;
  const int nbi = cdiv(nb, tmu), nbj = cdiv(nb, tnu);
  for (int bi = 0; bi < nbi; ++bi) {
    const int f = jao_first_col(bi, tmu, tnu);
    n += nbj > f ? nbj - f : 0;
  }
  return n;
}

// Per-MO AO Coulomb: Jn[q][mu][nu] = sum_l d[l][q] b[l][mu][nu].
// M = q, N = a TMU x TNU block of (mu, nu), K = l.  Tiles enumerate only
// blocks that touch the upper triangle, q-tile fastest (tiles sharing a b
// block are adjacent).  Each block writes (mu <= nu) directly and (mu < nu)
// mirrored, so every element of the full matrix is written exactly once.
template <int P, class Cfg>
__host__ __device__ inline long jao_tiles(const JaoArgs& a) {
  return jao_active(a.nb, Cfg::BN / kJaoTNU, kJaoTNU) * cdiv(a.nw, Cfg::BM);
}
template <int P, class Cfg, bool kTrim = false>
__device__ void jao_tile(const JaoArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  constexpr int TNU = kJaoTNU, TMU = Cfg::BN / TNU;
  const int nb = a.nb, na = a.na, nw = a.nw;
  const int nbj = cdiv(nb, TNU), nbi = cdiv(nb, TMU);
  const long nq = cdiv(nw, Cfg::BM);
  const int qt = (int)(t % nq);
  long r = t / nq;
  int bi = 0;
  for (; bi < nbi; ++bi) {
    const int n = nbj - jao_first_col(bi, TMU, TNU);
    if (r < n) break;
    r -= n;
  }
  if (bi >= nbi) return;
  const int bj = jao_first_col(bi, TMU, TNU) + (int)r;
  const int mu0 = bi * TMU, nu0 = bj * TNU;
  const int q0 = qt * Cfg::BM;
  const long B2 = (long)nb * nb;
  auto b_off = [&](int x, long& o) {   // element (mu, nu) of the block in slab l = 0
    const int mu = mu0 + x / TNU, nu = nu0 + x % TNU;
    o = (long)mu * nb + nu;
    return mu < nb && nu < nb;
  };
  typename E::template Acc<Cfg> acc;
  IOT<P>* Jn = (IOT<P>*)a.Jn;
  auto store = [&](int m, int n, double v) {
    const int q = q0 + m, mu = mu0 + n / TNU, nu = nu0 + n % TNU;
    if (q < nw && mu < nb && nu < nb) {
      IOT<P>* J = Jn + (long)q * B2;
      if (mu <= nu) J[(long)mu * nb + nu] = (IOT<P>)v;
      if (mu < nu) J[(long)nu * nb + mu] = (IOT<P>)v;
    }
  };
  const int fim = cdiv(nw - q0, 16);   // live fragment rows
  bool staged = false;
  if constexpr (P == kF64 && Cfg::BM == 128 && Cfg::BN == 128) {
    if (a.dma) {   // both operands by direct global -> LDS loads
      XcDma64<Cfg::NT, E::BK, E::PAD> la, lb;
      la.init(a.d, nw, na, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
      lb.init(a.b, B2, na, b_off);
      if constexpr (kTrim) {
        run_q_rows<P, Cfg, kTrim>(fim, acc, [&](auto mma) {
          gemm_mainloop_dma_with<E, Cfg, 2>(la, lb, cdiv(na, E::BK), acc, smem, false, mma);
        }, store);
        return;
      } else {
        gemm_mainloop_dma<E, Cfg, 2>(la, lb, cdiv(na, E::BK), acc, smem);
        staged = true;
      }
    }
  }
  if (!staged) {
    // A: d^T (x = q, k = l), from piece planes in the split modes
    typename std::conditional<kPlanesHalfJao<P>, PCS<P, Cfg::BM, Cfg::NT>, XCS<P, double, Cfg::BM, Cfg::NT>>::type la;
    if constexpr (kPlanesHalfJao<P>)
      la.init(a.Ds.p, a.Ds.ps, a.Ds.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
    else
      la.init(a.d, nw, na, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
    XCS<P, double, Cfg::BN, Cfg::NT> lb;
    lb.init(a.b, B2, na, b_off);
    if constexpr (kTrim && kPieces<P> == 0) {
      run_q_rows<P, Cfg, kTrim>(fim, acc, [&](auto mma) {
        gemm_mainloop_with<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem, false, mma);
      }, store);
      return;
    } else {
      gemm_mainloop<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem);
    }
  }
  acc.for_each(store);
}

template <int P, class Cfg>
__device__ void jao_g_tile(const JaoArgs& a, long t, char* smem) { jao_tile<P, Cfg, true>(a, t, smem); }

// The same J^q tile with b read as pre-split piece planes (split modes):
// B element (x = (mu, nu) of the block, k = l) at plane row mu*n_bf + nu, and
// d^T from its piece planes, so neither operand is split here; both are staged
// by direct global -> LDS loads.  The pieces are the staging path's own split
// of the same values, so the results are bitwise those of jao_tile.
template <int P, class Cfg>
__host__ __device__ inline long jaop_tiles(const JaoArgs& a) { return jao_tiles<P, Cfg>(a); }
template <int P, class Cfg>
__device__ void jaop_one_tile(const JaoArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  constexpr int TNU = kJaoTNU, TMU = Cfg::BN / TNU;
  const int nb = a.nb, na = a.na, nw = a.nw;
  const int nbj = cdiv(nb, TNU), nbi = cdiv(nb, TMU);
  const long nq = cdiv(nw, Cfg::BM);
  const int qt = (int)(t % nq);
  long r = t / nq;
  int bi = 0;
  for (; bi < nbi; ++bi) {
    const int n = nbj - jao_first_col(bi, TMU, TNU);
    if (r < n) break;
    r -= n;
  }
  if (bi >= nbi) return;
  const int bj = jao_first_col(bi, TMU, TNU) + (int)r;
  const int mu0 = bi * TMU, nu0 = bj * TNU;
  const int q0 = qt * Cfg::BM;
  const long B2 = (long)nb * nb;
  static_assert(kPieces<P> > 0, "J^q from piece planes in the split modes only");
  PDMA<P, Cfg::BM, Cfg::NT> la;
  la.init(a.Ds.p, a.Ds.ps, a.Ds.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
  PDMA<P, Cfg::BN, Cfg::NT> lb;
  lb.init(a.Bj.p, a.Bj.ps, a.Bj.ld, [&](int x, long& o) {
    const int mu = mu0 + x / TNU, nu = nu0 + x % TNU;
    o = (long)mu * nb + nu;
    return mu < nb && nu < nb;
  });
  typename E::template Acc<Cfg> acc;
  gemm_mainloop_dma<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem);
  IOT<P>* Jn = (IOT<P>*)a.Jn;
  acc.for_each([&](int m, int n, double v) {
    const int q = q0 + m, mu = mu0 + n / TNU, nu = nu0 + n % TNU;
    if (q < nw && mu < nb && nu < nb) {
      IOT<P>* J = Jn + (long)q * B2;
      if (mu <= nu) J[(long)mu * nb + nu] = (IOT<P>)v;
      if (mu < nu) J[(long)nu * nb + mu] = (IOT<P>)v;
    }
  });
}

// The single-molecule J^q from piece planes runs persistent workgroups like
// the pre-split half transform (one per resident slot, loads running ahead
// into the next tile).  Workgroups are dispatched round-robin over the 8 XCDs;
// those of one XCD take a contiguous eighth of the tile list, so tiles that
// share b blocks run on one L2.  Bitwise the results of jaop_one_tile (the
// grouped kernel's per-tile form).
template <int P, class Cfg>
__device__ void jaop_persistent(const JaoArgs& a, char* smem) {
  using E = typename EngineOf<P>::type;
  using LA = PDMA<P, Cfg::BM, Cfg::NT>;
  using LB = PDMA<P, Cfg::BN, Cfg::NT>;
  constexpr int TNU = kJaoTNU, TMU = Cfg::BN / TNU;
  const int nb = a.nb, na = a.na, nw = a.nw;
  const int nbj = cdiv(nb, TNU), nbi = cdiv(nb, TMU);
  const long nq = cdiv(nw, Cfg::BM);
  const long B2 = (long)nb * nb;
  const long n = jaop_tiles<P, Cfg>(a), G = gridDim.x, w = blockIdx.x;
  long first = w, step = G, end = n;
  if (G % 8 == 0 && n >= G) {
    const long x = w % 8;
    first = x * n / 8 + w / 8;
    step = G / 8;
    end = (x + 1) * n / 8;
  }
  auto decode = [&](long t, int& q0, int& mu0, int& nu0) {
    q0 = (int)(t % nq) * Cfg::BM;
    long r = t / nq;
    int bi = 0;
    for (; bi < nbi; ++bi) {
      const int m = nbj - jao_first_col(bi, TMU, TNU);
      if (r < m) break;
      r -= m;
    }
    mu0 = bi * TMU;   // bi == nbi only past the list: then nothing is stored
    nu0 = (bi < nbi ? jao_first_col(bi, TMU, TNU) + (int)r : 0) * TNU;
  };
  IOT<P>* Jn = (IOT<P>*)a.Jn;
  gemm_persistent_dma<E, Cfg, 0, LA, LB>(
      first, step, end, cdiv(na, E::BK), smem,
      [&](long t, LA& la, LB& lb) {
        int q0, mu0, nu0;
        decode(t, q0, mu0, nu0);
        la.init(a.Ds.p, a.Ds.ps, a.Ds.ld, [&](int x, long& o) { o = q0 + x; return q0 + x < nw; });
        lb.init(a.Bj.p, a.Bj.ps, a.Bj.ld, [&](int x, long& o) {
          const int mu = mu0 + x / TNU, nu = nu0 + x % TNU;
          o = (long)mu * nb + nu;
          return mu < nb && nu < nb;
        });
      },
      [&](long t, const typename E::template Acc<Cfg>& acc) {
        int q0, mu0, nu0;
        decode(t, q0, mu0, nu0);
        acc.for_each([&](int m, int nn, double v) {
          const int q = q0 + m, mu = mu0 + nn / TNU, nu = nu0 + nn % TNU;
          if (q < nw && mu < nb && nu < nb) {
            IOT<P>* J = Jn + (long)q * B2;
            if (mu <= nu) J[(long)mu * nb + nu] = (IOT<P>)v;
            if (mu < nu) J[(long)nu * nb + mu] = (IOT<P>)v;
          }
        });
      });
}
template <int P, class Cfg>
__device__ void jaop_tile(const JaoArgs& a, long, char* smem) { jaop_persistent<P, Cfg>(a, smem); }

// Per-MO AO exchange: Kn[q] = X_q^T X_q with X_q = b_half[q] ([n_aux][n_bf]).
// Square blocks bi <= bj only (the blocks of one q adjacent), mirrored like J.
// A block with every 16x16 fragment needed runs the regular wave layout.  In
// FP64/FP32, a block on the diagonal (fragments I <= J only) or on the ragged
// edge trims each wave's fragment rows to the live ones under a balanced wave
// plan, and a diagonal block stages its single operand panel once.
template <int P, class Cfg>
__host__ __device__ inline long kao_tiles(const KaoArgs& a) {
  const long nbk = cdiv(a.nb, Cfg::BM);
  return nbk * (nbk + 1) / 2 * a.nw;
}
template <int P, class Cfg>
__device__ void kao_tile(const KaoArgs& a, long t, char* smem) {
  static_assert(Cfg::BM == Cfg::BN, "square blocks");
  using E = typename EngineOf<P>::type;
  const int nb = a.nb, na = a.na, nw = a.nw;
  const int nbk = cdiv(nb, Cfg::BM);
  const long nblk = (long)nbk * (nbk + 1) / 2;
  const int q = (int)(t / nblk);
  if (q >= nw) return;
  int rem = (int)(t % nblk), bi = 0;
  while (rem >= nbk - bi) { rem -= nbk - bi; ++bi; }
  const int bj = bi + rem;
  const long AB = (long)na * nb;
  const IOT<P>* X = (const IOT<P>*)a.bh + (long)q * AB;
  const int mu0 = bi * Cfg::BM, nu0 = bj * Cfg::BN;
  XCS<P, IOT<P>, Cfg::BM, Cfg::NT> la;
  la.init(X, nb, na, [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
  XCS<P, IOT<P>, Cfg::BN, Cfg::NT> lb;
  lb.init(X, nb, na, [&](int x, long& o) { o = nu0 + x; return nu0 + x < nb; });
  typename E::template Acc<Cfg> acc;
  const long B2 = (long)nb * nb;
  IOT<P>* K = (IOT<P>*)a.Kn + (long)q * B2;
  auto store = [&](int m, int n, double v) {
    const int mu = mu0 + m, nu = nu0 + n;
    if (mu < nb && nu < nb) {
      if (mu <= nu) K[(long)mu * nb + nu] = (IOT<P>)v;
      if (mu < nu) K[(long)nu * nb + mu] = (IOT<P>)v;
    }
  };
  constexpr int FB = Cfg::BM / 16;
  const int fim = min(FB, cdiv(nb - mu0, 16)), fjm = min(FB, cdiv(nb - nu0, 16));
  const bool diag = bi == bj;
  if constexpr (P == kF64 && Cfg::BM == 64) {
    if (a.dma) {   // unpadded rows, three stages (two slices in flight), three workgroups per CU
      using E2 = EngF64T<16, 0>;
      XcDma64<Cfg::NT, E2::BK, E2::PAD, 64> da, db;
      da.init((const double*)X, nb, na, [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
      db.init((const double*)X, nb, na, [&](int x, long& o) { o = nu0 + x; return nu0 + x < nb; });
      typename E2::template Acc<Cfg> acc2;
      if (!diag && fim == FB && fjm == FB) {
        gemm_mainloop_dma<E2, Cfg, 3>(da, db, cdiv(na, E2::BK), acc2, smem);
        acc2.for_each(store);
        return;
      }
      const WavePlan w =
          make_wave_plan<Cfg>([&](int I, int J) { return I < fim && J < fjm && (!diag || I <= J); });
      with_rows<Cfg::TM>(w.ni, [&](auto rows) {
        constexpr int NI = decltype(rows)::value;
        gemm_mainloop_dma_with<E2, Cfg, 3>(da, db, cdiv(na, E2::BK), acc2, smem, diag,
                                           [&](const lds_char* SA, const lds_char* SB,
                                               typename E2::template Acc<Cfg>& c) {
                                             E2::template mma_rows<Cfg, NI>(SA, SB, c, w);
                                           });
      });
      acc2.for_each(w, store);
      return;
    }
  }
  if constexpr (P == kF64 && Cfg::BM == 128) {
    if (a.dma) {   // b_half by direct global -> LDS loads; a diagonal block stages one panel
      XcDma64<Cfg::NT, E::BK, E::PAD, Cfg::BM> da, db;
      da.init((const double*)X, nb, na, [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
      db.init((const double*)X, nb, na, [&](int x, long& o) { o = nu0 + x; return nu0 + x < nb; });
      if (!diag && fim == FB && fjm == FB) {
        gemm_mainloop_dma<E, Cfg, 2>(da, db, cdiv(na, E::BK), acc, smem);
        acc.for_each(store);
        return;
      }
      const WavePlan w =
          make_wave_plan<Cfg>([&](int I, int J) { return I < fim && J < fjm && (!diag || I <= J); });
      with_rows<Cfg::TM>(w.ni, [&](auto rows) {
        constexpr int NI = decltype(rows)::value;
        gemm_mainloop_dma_with<E, Cfg, 2>(da, db, cdiv(na, E::BK), acc, smem, diag,
                                          [&](const lds_char* SA, const lds_char* SB,
                                              typename E::template Acc<Cfg>& c) {
                                            E::template mma_rows<Cfg, NI>(SA, SB, c, w);
                                          });
      });
      acc.for_each(w, store);
      return;
    }
  }
  // The split-BF16 engines (VALU-bound by operand splitting, and short of
  // registers for the extra loop copies) always compute whole blocks.
  constexpr bool kPlan = P == kF64 || P == kF32;
  if (!kPlan || (!diag && fim == FB && fjm == FB)) {
    gemm_mainloop<E, Cfg, kDeep<P>>(la, lb, cdiv(na, E::BK), acc, smem);
    acc.for_each(store);
    return;
  }
  if constexpr (kPlan) {
    const WavePlan w =
        make_wave_plan<Cfg>([&](int I, int J) { return I < fim && J < fjm && (!diag || I <= J); });
    with_rows<Cfg::TM>(w.ni, [&](auto rows) {
      constexpr int NI = decltype(rows)::value;
      gemm_mainloop_with<E, Cfg>(la, lb, cdiv(na, E::BK), acc, smem, diag,
                                 [&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
                                   E::template mma_rows<Cfg, NI>(SA, SB, c, w);
                                 });
    });
    acc.for_each(w, store);
  }
}

// FP64 GEMM out[m][n] = sum_k A[k][m] B[k][n], both operands x-contiguous;
// used for H C_Omega and lambda = C^T Y.  These are small (n_bf x n_omega
// outputs), so the k range is split into ksplit parts written to separate
// partial outputs, which their consumers add in a fixed order.
template <int P, class Cfg>
__host__ __device__ inline long gemm_tiles(const GemmArgs& a) {
  return (long)cdiv(a.M, Cfg::BM) * cdiv(a.N, Cfg::BN) * a.ksplit;
}
template <int P, class Cfg>
__device__ void gemm_tile(const GemmArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  const int nmt = cdiv(a.M, Cfg::BM), nnt = cdiv(a.N, Cfg::BN);
  const int m0 = (int)(t % nmt) * Cfg::BM, n0 = (int)((t / nmt) % nnt) * Cfg::BN;
  const int s = (int)(t / ((long)nmt * nnt));
  const int k0 = s * a.kc, kn = min(a.kc, a.K - k0);
  const int M = a.M, N = a.N;
  XCS<P, double, Cfg::BM, Cfg::NT> la;
  la.init(a.A + (long)k0 * a.lda, a.lda, kn, [&](int x, long& o) { o = m0 + x; return m0 + x < M; });
  XCS<P, double, Cfg::BN, Cfg::NT> lb;
  lb.init(a.B + (long)k0 * a.ldb, a.ldb, kn, [&](int x, long& o) { o = n0 + x; return n0 + x < N; });
  typename E::template Acc<Cfg> acc;
  gemm_mainloop<E, Cfg>(la, lb, cdiv(kn, E::BK), acc, smem);
  double* out = a.out + s * a.ostride;
  acc.for_each([&](int m, int n, double v) {
    if (m0 + m < M && n0 + n < N) out[(long)(m0 + m) * a.ldo + n0 + n] = v;
  });
}

// Fock-apply over the stacked operand [J^0..J^{W-1}, K^0..K^{W-1}]:
//   Ypart[s][mu][q] = sum_{(t, nu) in split s} X_t[nu][mu] coef_t[q] C[nu][q]
// with X_t = J^t (coef A[q][t]) or K^{t-W} (coef B[q][t-W]).  M = mu, N = q,
// K = (t, nu), nu padded per slab to a multiple of the slice depth; the K
// slices (slab-major) are split into nsplit near-equal ranges, so a split may
// start or end inside a slab.  The loaders start at global slice g0.
template <int P, class Cfg>
struct FockA {  // element (mu, nu) of slab t; X_t symmetric, so read row nu
  using E = typename EngineOf<P>::type;
  using T = IOT<P>;
  using G = XCS<P, T, Cfg::BM, Cfg::NT>;
  static constexpr int NP = G::NP, R = G::R, RR = G::RR, KV = E::KV, BK = E::BK;
  using type = T;
  G g;
  const T *Jn, *Kn;
  int nb, nw, g0, nchunk, mu;
  __device__ void init(const T* Jn_, const T* Kn_, int nb_, int nw_, int g0_, int mu0) {
    Jn = Jn_; Kn = Kn_; nb = nb_; nw = nw_; g0 = g0_; nchunk = (nb + BK - 1) / BK;
    g.x = threadIdx.x % Cfg::BM; g.kg = threadIdx.x / Cfg::BM;
    mu = mu0 + g.x; g.ok = mu < nb;
  }
  __device__ int xl(int p) const { return g.xl(p); }
  __device__ int kl(int p) const { return g.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return g.ok && ((g0 + kt) % nchunk) * BK + g.kl(p) + i < nb; }
  __device__ void fetch(int kt, T (&r)[RR]) const {
    const int t = (g0 + kt) / nchunk, nu0 = ((g0 + kt) % nchunk) * BK;
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
  int nb, nw, nmo, g0, nchunk, q;
  __device__ void init(const double* Ac_, const double* Bc_, const double* C_, int nb_, int nw_, int nmo_,
                       int g0_, int q0) {
    Ac = Ac_; Bc = Bc_; C = C_; nb = nb_; nw = nw_; nmo = nmo_; g0 = g0_;
    nchunk = (nb + BK - 1) / BK;
    g.x = threadIdx.x % Cfg::BN; g.kg = threadIdx.x / Cfg::BN;
    q = q0 + g.x; g.ok = q < nw;
  }
  __device__ int xl(int p) const { return g.xl(p); }
  __device__ int kl(int p) const { return g.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return g.ok && ((g0 + kt) % nchunk) * BK + g.kl(p) + i < nb; }
  __device__ void fetch(int kt, double (&r)[RR]) const {
    const int t = (g0 + kt) / nchunk, nu0 = ((g0 + kt) % nchunk) * BK;
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

// FP64 Fock operands by direct global -> LDS loads (128 x 128 tiles, one
// 128-column k-row per wave load into the engine's padded [k][x] layout).
// Slice g of the stacked slabs holds rows nu0 .. nu0+15 of slab t = g / nchunk
// (nu0 = 16 (g mod nchunk)); rows at or past n_bf read zeros.  A: element
// (mu, nu) of slab t read as row nu of X_t (J^t or K^t, symmetric); B: row nu
// of C (x = q), scaled by the slab's coefficient at MFMA time.
template <int NT>
struct FockDma {
  static constexpr int NW = NT / 64, BK = 16, UPW = BK / NW, STRIDE = (128 + EngF64::PAD) * 8;
  static_assert(BK % NW == 0, "k rows per wave");
  const double *J, *K, *C;   // A: J, K (slabs of B2); B: C (J == nullptr)
  long B2, ld;
  int nb, nw, g0, nchunk, col;
  __device__ int count() const { return UPW; }
  __device__ void issue(int kt, lds_char* S) const {
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int g = g0 + kt, t = g / nchunk, nu0 = (g - t * nchunk) * BK;
    const double* base = J ? (t < nw ? J + (long)t * B2 : K + (long)(t - nw) * B2) : C;
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
      const int r = w + j * NW, nu = nu0 + r;
      const double* src = nu < nb ? base + (long)nu * ld + col : kDmaZeros + 2 * lane;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(S + r * STRIDE), 16, 0, 0);
    }
  }
};

template <int P, class Cfg>
__host__ __device__ inline long fock_tiles(const FockArgs& a) {
  return (long)cdiv(a.nb, Cfg::BM) * cdiv(a.nw, Cfg::BN) * a.nsplit;
}
template <int P, class Cfg>
__device__ void fock_tile(const FockArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  const int nb = a.nb, nw = a.nw;
  const int nmt = cdiv(nb, Cfg::BM), nnt = cdiv(nw, Cfg::BN);
  const int mu0 = (int)(t % nmt) * Cfg::BM;
  const int q0 = (int)((t / nmt) % nnt) * Cfg::BN;
  const int s = (int)(t / ((long)nmt * nnt));
  const long S = 2L * nw * cdiv(nb, E::BK);   // slices over all slabs
  const int g0 = (int)(S * s / a.nsplit), g1 = (int)(S * (s + 1) / a.nsplit);
  if constexpr (P == kF64 && Cfg::BM == 128 && Cfg::BN == 128) {
    if (a.dma) {
      const int lane = (int)(threadIdx.x & 63), nchunk = cdiv(nb, E::BK);
      FockDma<Cfg::NT> la{(const double*)a.Jn, (const double*)a.Kn, nullptr, (long)nb * nb, nb,
                          nb, nw, g0, nchunk, mu0 + 2 * lane < nb ? mu0 + 2 * lane : 0};
      FockDma<Cfg::NT> lb{nullptr, nullptr, a.C, 0, a.nmo, nb, nw, g0, nchunk, q0 + 2 * lane < nw ? q0 + 2 * lane : 0};
      typename E::template Acc<Cfg> acc;
      int kt = 0, tc = -1;
      double cq[Cfg::TN];
      int wm0, wn0;
      wave_origin(Cfg::WAVES_N, Cfg::WM, Cfg::WN, wm0, wn0);
      const int kr = lane >> 4, xc = lane & 15;
      // B element (q, nu) = coef_t[q] * C[nu][q], the product the register
      // path stages; the coefficients change once per slab
      gemm_mainloop_dma_with<E, Cfg, 2>(la, lb, g1 - g0, acc, smem, false,
                                        [&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
        const int t = (g0 + kt++) / nchunk;
        if (t != tc) {
          tc = t;
#pragma unroll
          for (int j = 0; j < Cfg::TN; ++j) {
            const int q = q0 + wn0 + j * 16 + xc;
            cq[j] = q < nw ? (t < nw ? a.Ac[(long)q * nw + t] : a.Bc[(long)q * nw + (t - nw)]) : 0.0;
          }
        }
        const lds_f64* As = (const lds_f64*)SA;
        const lds_f64* Bs = (const lds_f64*)SB;
#pragma unroll
        for (int kk = 0; kk < E::BK; kk += 4) {
          double av[Cfg::TM], bv[Cfg::TN];
#pragma unroll
          for (int i = 0; i < Cfg::TM; ++i) av[i] = As[(kk + kr) * (Cfg::BM + E::PAD) + wm0 + i * 16 + xc];
#pragma unroll
          for (int j = 0; j < Cfg::TN; ++j) bv[j] = cq[j] * Bs[(kk + kr) * (Cfg::BN + E::PAD) + wn0 + j * 16 + xc];
#pragma unroll
          for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
            for (int j = 0; j < Cfg::TN; ++j)
              c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c.v[i][j], 0, 0, 0);
        }
      });
      double* Y = a.Yp + (long)s * nb * nw;
      acc.for_each([&](int m, int n, double v) {
        if (mu0 + m < nb && q0 + n < nw) Y[(long)(mu0 + m) * nw + q0 + n] = v;
      });
      return;
    }
  }
  FockA<P, Cfg> la;
  la.init((const IOT<P>*)a.Jn, (const IOT<P>*)a.Kn, nb, nw, g0, mu0);
  FockB<P, Cfg> lb;
  lb.init(a.Ac, a.Bc, a.C, nb, nw, a.nmo, g0, q0);
  typename E::template Acc<Cfg> acc;
  gemm_mainloop<E, Cfg>(la, lb, g1 - g0, acc, smem);
  double* Y = a.Yp + (long)s * nb * nw;
  acc.for_each([&](int m, int n, double v) {
    if (mu0 + m < nb && q0 + n < nw) Y[(long)(mu0 + m) * nw + q0 + n] = v;
  });
}

// ---- gradient without per-MO AO matrices ---------------------------------------
// Since b is symmetric, J^(r) c_q = sum_l d_lr bh[q][l] and
// K^(r) c_q = sum_l bmo[l][r][q] bh[r][l], so
//   Y[:, q] - n_q H c_q = sum_l a_lq bh[q][l] + sum_{r,l} B_qr bmo[l][r][q] bh[r][l],
// a_lq = sum_r A_qr d_lr: one contraction over k = (r, l) of b_half with
// coefficients built from b_mo, with the Coulomb part on the r = q terms:
//   Zt[l][q] = B_qq d_lq + a_lq,  Bt[q][r] = B_qr (r != q), 1 (r == q).
// Tiles 0 .. n_aux-1: one per l, d[l][:] staged in LDS, threads over q;
// then the Bt tiles, 256 entries each.
constexpr int kYdzLds = 4096;   // n_omega up to this many read d from LDS
template <int P, class Cfg>
__host__ __device__ inline long ydz_tiles(const YdzArgs& a) {
  return (long)a.na + cdiv((long)a.nw * a.nw, 256);
}
template <int P, class Cfg>
__device__ void ydz_tile(const YdzArgs& a, long t, char* smem) {
  const int nw = a.nw;
  if (t < a.na) {
    const int l = (int)t;
    const double* dl = a.d + (long)l * nw;
    double* ds = (double*)smem;
    const bool in_lds = nw <= kYdzLds;
    if (in_lds)
      for (int r = threadIdx.x; r < nw; r += 256) ds[r] = dl[r];
    __syncthreads();
    const double* dr = in_lds ? ds : dl;
    for (int q = threadIdx.x; q < nw; q += 256) {
      // A is symmetric (bitwise: its entries are products of commuting
      // factors), so row r read along q is coalesced
      double s = a.Bc[(long)q * nw + q] * dr[q];
#pragma unroll 8
      for (int r = 0; r < nw; ++r) s = fma(a.Ac[(long)r * nw + q], dr[r], s);
      ((IOT<P>*)a.Zt)[(long)l * nw + q] = (IOT<P>)s;
    }
  } else {
    const long j = (t - a.na) * 256 + threadIdx.x;
    if (j < (long)nw * nw) {
      const int q = (int)(j / nw), r = (int)(j - (long)q * nw);
      ((IOT<P>*)a.Bt)[j] = (IOT<P>)(q == r ? 1.0 : a.Bc[j]);
    }
  }
}

template <int P, class Cfg>
struct YdB {  // element (q, k): value in r[i], coefficient Bt[q][r] in r[R + i]
  using E = typename EngineOf<P>::type;
  using T = IOT<P>;
  using G = XCS<P, T, Cfg::BN, Cfg::NT>;
  static constexpr int NP = G::NP, R = G::R, RR = 2 * G::R, KV = E::KV, BK = E::BK;
  using type = T;
  G g;
  const T *bmo, *Zt, *Bt;
  int na, nw, q;
  long k0, kend;
  double inv_na;
  __device__ void init(const T* bmo_, const T* Zt_, const T* Bt_, int na_, int nw_, long k0_, long kend_, int q0) {
    bmo = bmo_; Zt = Zt_; Bt = Bt_; na = na_; nw = nw_; k0 = k0_; kend = kend_;
    inv_na = 1.0 / na;
    g.x = threadIdx.x % Cfg::BN; g.kg = threadIdx.x / Cfg::BN;
    q = q0 + g.x; g.ok = q < nw;
  }
  __device__ int xl(int p) const { return g.xl(p); }
  __device__ int kl(int p) const { return g.kl(p); }
  __device__ bool valid(int p, int i, int kt) const { return g.ok && k0 + (long)kt * BK + g.kl(p) + i < kend; }
  __device__ void fetch(int kt, T (&r)[RR]) const {
    const int qc = g.ok ? q : 0;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        long k = k0 + (long)kt * BK + g.kl(p) + i;
        k = k < kend ? k : kend - 1;
        const int kk = (int)k;   // k < n_aux * n_omega < 2^31
        // r = kk / n_aux from the reciprocal (off by at most one), then exact
        int rr = (int)((double)kk * inv_na), l = kk - rr * na;
        if (l < 0) { --rr; l += na; } else if (l >= na) { ++rr; l -= na; }
        const T* src = rr == qc ? Zt + (long)l * nw + qc : bmo + ((long)l * nw + rr) * nw + qc;
        r[p * KV + i] = *src;
        r[R + p * KV + i] = Bt[(long)qc * nw + rr];
      }
  }
  __device__ double val(const T (&r)[RR], int p, int i) const {
    return (double)r[R + p * KV + i] * (double)r[p * KV + i];
  }
};

template <int P, class Cfg>
__host__ __device__ inline long yd_tiles(const YdArgs& a) {
  return (long)cdiv(a.nb, Cfg::BM) * cdiv(a.nw, Cfg::BN) * a.nsplit;
}
template <int P, class Cfg>
__device__ void yd_tile(const YdArgs& a, long t, char* smem) {
  using E = typename EngineOf<P>::type;
  using T = IOT<P>;
  const int nb = a.nb, nw = a.nw;
  const int nmt = cdiv(nb, Cfg::BM), nnt = cdiv(nw, Cfg::BN);
  const int mu0 = (int)(t % nmt) * Cfg::BM;
  const int q0 = (int)((t / nmt) % nnt) * Cfg::BN;
  const int s = (int)(t / ((long)nmt * nnt));
  const long K = (long)a.na * nw, k0 = (long)s * a.kc, k1 = min(K, k0 + a.kc);
  // A: b_half as [(r, l)][nu] (x = nu), rows k0 .. k1 of this split
  XCS<P, T, Cfg::BM, Cfg::NT> la;
  la.init((const T*)a.bh + k0 * nb, nb, (int)(k1 - k0), [&](int x, long& o) { o = mu0 + x; return mu0 + x < nb; });
  YdB<P, Cfg> lb;
  lb.init((const T*)a.bmo, (const T*)a.Zt, (const T*)a.Bt, a.na, nw, k0, k1, q0);
  typename E::template Acc<Cfg> acc;
  gemm_mainloop<E, Cfg>(la, lb, (int)cdiv(k1 - k0, (long)E::BK), acc, smem);
  double* Y = a.Yp + (long)s * nb * nw;
  acc.for_each([&](int m, int n, double v) {
    if (mu0 + m < nb && q0 + n < nw) Y[(long)(mu0 + m) * nw + q0 + n] = v;
  });
}

// ---- pre-split of the small reused operands (split modes) -------------------
// One thread per pair of k of one row; same split arithmetic as the staging
// path (split_mode), so a pre-split operand gives the same pieces.
template <int P, class Cfg>
__host__ __device__ inline long psplit_tiles(const PSplitArgs& a) { return cdiv((long)a.nx * (a.ld / 2), 256); }
template <int P, class Cfg>
__device__ void psplit_tile(const PSplitArgs& a, long t, char*) {
  constexpr int NPC = kPieces<P> ? kPieces<P> : 1;
  const long i = t * 256 + threadIdx.x;
  const int hl = a.ld / 2;
  if (i >= (long)a.nx * hl) return;
  const int x = (int)(i / hl), k = 2 * (int)(i - (long)x * hl);
  const double d0 = k < a.K ? a.X[(long)k * a.sk + x] : 0.0;
  const double d1 = k + 1 < a.K ? a.X[(long)(k + 1) * a.sk + x] : 0.0;
  unsigned pc[NPC];
  split_mode<P>(d0, d1, pc);
#pragma unroll
  for (int s = 0; s < NPC; ++s) *(unsigned*)(a.out + s * a.ps + (long)x * a.ld + k) = pc[s];
}

template <int P, class Cfg>
__host__ __device__ inline long bsplit_tiles(const BSplitArgs& a) {
  return cdiv(a.nr * (kPieces<P> > 0 ? a.ld / 2 : a.nb), 256);
}
template <int P, class Cfg>
__device__ void bsplit_tile(const BSplitArgs& a, long t, char*) {
  const long i = t * 256 + threadIdx.x;
  if constexpr (kPieces<P> > 0) {
    constexpr int NPC = kPieces<P>;
    const int hl = a.ld / 2;
    if (i >= a.nr * hl) return;
    const long x = i / hl;
    const int k = 2 * (int)(i - x * hl);
    const double* row = a.b + x * a.nb;
    const double d0 = k < a.nb ? row[k] : 0.0;
    const double d1 = k + 1 < a.nb ? row[k + 1] : 0.0;
    unsigned pc[NPC];
    split_mode<P>(d0, d1, pc);
    unsigned short* out = (unsigned short*)a.out;
#pragma unroll
    for (int s = 0; s < NPC; ++s) *(unsigned*)(out + s * a.ps + x * a.ld + k) = pc[s];
  } else {
    if (i < a.nr * a.nb) ((float*)a.out)[i] = (float)a.b[i];
  }
}

// b pre-split for J^q: plane s, row r = mu*n_bf + nu (every mu, nu), k = l
// contiguous; element (r, l) is piece s of b[l][mu][nu], zero from l = n_aux up
// to ld (a multiple of 32).  64 x 64 (r, l) tiles transposed through LDS: b is
// read along r, the pieces written along l, each pair (l, l+1) split by the
// staging path's arithmetic.
struct BSplitJArgs { const double* b; long nrow; int na, ld; unsigned short* out; long ps; };
template <int P>
__global__ __launch_bounds__(256) void k_bsplitj(BSplitJArgs a) {
  constexpr int NPC = kPieces<P>;
  __shared__ double t[64][65];
  const long r0 = (long)blockIdx.x * 64;
  const int l0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int l = l0 + y;
    const long r = r0 + tx;
    t[y][tx] = (l < a.na && r < a.nrow) ? a.b[(long)l * a.nrow + r] : 0.0;
  }
  __syncthreads();
  const int pl = threadIdx.x & 31, ry = threadIdx.x >> 5;
  const int l = l0 + 2 * pl;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int y = ry + 8 * j;
    const long r = r0 + y;
    if (r >= a.nrow || l >= a.ld) continue;
    unsigned pc[NPC];
    split_mode<P>(t[2 * pl][y], t[2 * pl + 1][y], pc);
#pragma unroll
    for (int s = 0; s < NPC; ++s) *(unsigned*)(a.out + s * a.ps + r * a.ld + l) = pc[s];
  }
}

// ---- element-wise and reduction steps (256-thread tiles) -------------------

// MO J/K partial sums over a contiguous range of l (fixed split), then a
// fixed-order reduction over the splits.  FP64 arithmetic in every mode.
template <int P, class Cfg>
__host__ __device__ inline long jkp_tiles(const JkArgs& a) { return (long)cdiv((long)a.nw * a.nw, 256) * a.nsplit; }
template <int P, class Cfg>
__device__ void jkp_tile(const JkArgs& a, long t, char*) {
  const long w2 = (long)a.nw * a.nw;
  const long nx = cdiv(w2, 256);
  const long pq = (t % nx) * 256 + threadIdx.x;
  const int s = (int)(t / nx);
  if (pq >= w2) return;
  const int nw = a.nw, na = a.na, nsplit = a.nsplit;
  const int l0 = (int)((long)na * s / nsplit), l1 = (int)((long)na * (s + 1) / nsplit);
  const int p = (int)(pq / nw), q = (int)(pq - (long)p * nw);
  const IOT<P>* bmo = (const IOT<P>*)a.bmo;
  double sj = 0.0, sk = 0.0;
#pragma unroll 8
  for (int l = l0; l < l1; ++l) {
    const double v = (double)bmo[(long)l * w2 + pq];
    sk = fma(v, v, sk);
    sj = fma(a.d[(long)l * nw + p], a.d[(long)l * nw + q], sj);
  }
  a.part[(2L * s) * w2 + pq] = sj;
  a.part[(2L * s + 1) * w2 + pq] = sk;
}

template <int P, class Cfg>
__host__ __device__ inline long jkr_tiles(const JkArgs& a) { return cdiv((long)a.nw * a.nw, 256); }
template <int P, class Cfg>
__device__ void jkr_tile(const JkArgs& a, long t, char*) {
  const long w2 = (long)a.nw * a.nw;
  const long pq = t * 256 + threadIdx.x;
  if (pq >= w2) return;
  double sj = 0.0, sk = 0.0;
  for (int s = 0; s < a.nsplit; ++s) {
    sj += a.part[(2L * s) * w2 + pq];
    sk += a.part[(2L * s + 1) * w2 + pq];
  }
  a.J[pq] = sj;
  a.K[pq] = sk;
}

// Pair index of orbital p of Omega (explicit map or the default one).
__device__ __forceinline__ int pair_index(const int* pair_of, int p, int npairs, int ncwo) {
  if (pair_of) return pair_of[p];
  return p < npairs ? p : npairs - 1 - (p - npairs) / ncwo;
}

// Coefficients A, B of E = 2 sum n_p H_pp + sum (A J + B K) (Eq. (2), PNOF7 or
// PNOF5 Delta/Pi), with one energy partial per tile (fixed order).
template <int P, class Cfg>
__host__ __device__ inline long coef_tiles(const CoefArgs& a) { return cdiv((long)a.nw * a.nw, 256); }
template <int P, class Cfg>
__device__ void coef_tile(const CoefArgs& a, long t, char* smem) {
  double* red = (double*)smem;
  const int tid = threadIdx.x;
  const int nw = a.nw, npairs = a.npairs, ncwo = a.ncwo;
  const long w2 = (long)nw * nw;
  const long idx = t * 256 + tid;
  double e = 0.0;
  if (idx < w2) {
    const int p = (int)(idx / nw), q = (int)(idx - (long)p * nw);
    const double np = a.occ[p], nq = a.occ[q];
    const int gp = pair_index(a.pair_of, p, npairs, ncwo), gq = pair_index(a.pair_of, q, npairs, ncwo);
    double aa, bb;
    if (gp == gq) {
      aa = 0.0;
      if (p == q) bb = np;
      else if (p >= npairs && q >= npairs) bb = sqrt(np * nq);
      else bb = -sqrt(np * nq);
    } else {
      aa = 2.0 * np * nq;
      bb = -np * nq;
      if (a.functional == RIF_PNOF7) bb -= sqrt(np * (1.0 - np)) * sqrt(nq * (1.0 - nq));
    }
    a.Ac[idx] = aa;
    a.Bc[idx] = bb;
    e = aa * a.J[idx] + bb * a.K[idx];
  }
  red[tid] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) a.Ep[t] = red[0];
}

// H_pp = c_p^T H c_p, the energy (coefficient partials + 2 sum n_p H_pp, fixed
// order) and the device-side validation of the occupations.  One 1024-thread
// tile; H_pp has lanes along p (coalesced rows of C and HC) and the 16 waves
// over mu, combined in wave order.
constexpr int kEnergyThreads = 1024;
template <int P, class Cfg>
__host__ __device__ inline long energy_tiles(const EnergyArgs&) { return 1; }
template <int P, class Cfg>
__device__ void energy_tile(const EnergyArgs& a, long, char* smem) {
  constexpr int kStage = 2048, NT = kEnergyThreads, NWV = NT / 64;
  double* socc = (double*)smem;
  int* spair = (int*)(socc + kStage);
  double* red = (double*)(spair + kStage);   // NT doubles
  const int tid = threadIdx.x;
  const int nw = a.nw, npairs = a.npairs, ncwo = a.ncwo;
  const bool staged = nw <= kStage;
  if (staged) {
    for (int p = tid; p < nw; p += NT) {
      socc[p] = a.occ[p];
      spair[p] = pair_index(a.pair_of, p, npairs, ncwo);
    }
  }
  __syncthreads();
  int bad = 0;
  for (int p = tid; p < nw; p += NT) {
    const double n = staged ? socc[p] : a.occ[p];
    if (!(n >= 0.0 && n <= 1.0)) bad |= kBadOcc;
    const int g = staged ? spair[p] : pair_index(a.pair_of, p, npairs, ncwo);
    if (g < 0 || g >= npairs || (p < npairs && g != p)) bad |= kBadMap;
  }
  for (int g = tid; g < npairs; g += NT) {
    double s = 0.0;
    int cnt = 0;
    for (int p = 0; p < nw; ++p) {
      const int gp = staged ? spair[p] : pair_index(a.pair_of, p, npairs, ncwo);
      if (gp == g) { s += staged ? socc[p] : a.occ[p]; ++cnt; }
    }
    if (!(fabs(s - 1.0) <= 1e-12)) bad |= kBadSum;
    if (cnt != 1 + ncwo) bad |= kBadCount;
  }
  if (bad) atomicOr(a.flag, bad);

  double e = 0.0;
  for (int i = tid; i < a.nparts; i += NT) e += a.Ep[i];
  const int lane = tid & 63, wave = tid >> 6;
  for (int p0 = 0; p0 < nw; p0 += 64) {
    const int p = p0 + lane;
    double h = 0.0;
    if (p < nw) {
#pragma unroll 4
      for (int mu = wave; mu < a.nb; mu += NWV) h = fma(a.C[(long)mu * a.nmo + p], a.HC[(long)mu * nw + p], h);
    }
    red[tid] = h;
    __syncthreads();
    if (wave == 0 && p < nw) {
      double hp = 0.0;
      for (int w = 0; w < NWV; ++w) hp += red[w * 64 + lane];
      e += 2.0 * (staged ? socc[p] : a.occ[p]) * hp;
    }
    __syncthreads();
  }
  red[tid] = e;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    a.energy[0] = red[0];
    if (!isfinite(red[0])) atomicOr(a.flag, kNonFinite);   // reported by rif_sync
  }
  __syncthreads();
}
constexpr int kEnergySmem = 2048 * 8 + 2048 * 4 + kEnergyThreads * 8;

// Y[mu][q] = n_q HC[mu][q] + sum_s Ypart[s][mu][q] (fixed order)
template <int P, class Cfg>
__host__ __device__ inline long fred_tiles(const FockRedArgs& a) { return cdiv((long)a.nb * a.nw, 256); }
template <int P, class Cfg>
__device__ void fred_tile(const FockRedArgs& a, long t, char*) {
  const long n = (long)a.nb * a.nw;
  const long i = t * 256 + threadIdx.x;
  if (i >= n) return;
  const int q = (int)(i % a.nw);
  double y = a.occ[q] * a.HC[i];
#pragma unroll 8
  for (int s = 0; s < a.nsplit; ++s) y += a.Yp[(long)s * n + i];
  a.Y[i] = y;
}

// lambda = sum of its k-split partials (fixed order), written out for b < n_omega;
// G[a][b] = 4 (L[a][b] - L[b][a]),  L[a][b] = lambda[a][b] for b < n_omega, else 0.
template <int P, class Cfg>
__host__ __device__ inline long grad_tiles(const GradArgs& a) { return cdiv((long)a.nmo * a.nmo, 256); }
template <int P, class Cfg>
__device__ void grad_tile(const GradArgs& a, long t, char*) {
  const int nmo = a.nmo, nw = a.nw;
  const long i = t * 256 + threadIdx.x;
  if (i >= (long)nmo * nmo) return;
  const int r = (int)(i / nmo), c = (int)(i - (long)r * nmo);
  const long ls = (long)nmo * nw;
  auto lam = [&](int x, int y) {   // lambda[x][y], y < nw
    double v = 0.0;
    for (int s = 0; s < a.lsplit; ++s) v += a.lp[s * ls + (long)x * nw + y];
    return v;
  };
  const double lab = c < nw ? lam(r, c) : 0.0;
  const double lba = r < nw ? lam(c, r) : 0.0;
  if (c < nw) a.lam[(long)r * nw + c] = lab;
  const double g = 4.0 * (lab - lba);
  a.G[i] = g;
  if (!isfinite(g)) atomicOr(a.flag, kNonFinite);   // reported by rif_sync
}

// ---- kernel wrappers ---------------------------------------------------------
// k_<step>: one molecule, tile = (XCD-remapped) blockIdx.x.
// k_<step>_g: persistent over a work-list spanning molecules: tile t of the
// list belongs to molecule i with off[i] <= t < off[i+1]; workgroups stride the
// list by gridDim.x.

__device__ __forceinline__ int find_owner(const long* __restrict__ off, int n, long t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

#define RIF_STEP_KERNELS(NAME, ARGS, SMEM_BYTES, NTHREADS, REMAP, WPE, GWPE, GTILE)                \
  template <int P, class Cfg>                                                                      \
  __global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(WPE))) void k_##NAME(  \
      ARGS a) {                                                                                    \
    __shared__ __attribute__((aligned(16))) char smem[SMEM_BYTES];                                 \
    const long t = REMAP ? xcd_remap(blockIdx.x, (long)gridDim.x) : (long)blockIdx.x;              \
    NAME##_tile<P, Cfg>(a, t, smem);                                                               \
  }                                                                                                \
  template <int P, class Cfg>                                                                      \
  __global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(GWPE))) void k_##NAME##_g( \
      const ARGS* __restrict__ a, const long* __restrict__ off, int n, long total) {               \
    __shared__ __attribute__((aligned(16))) char smem[SMEM_BYTES];                                 \
    for (long t = blockIdx.x; t < total; t += gridDim.x) {                                         \
      const int i = find_owner(off, n, t);                                                         \
      GTILE<P, Cfg>(a[i], t - off[i], smem);                                                       \
    }                                                                                              \
  }

// Single-molecule GEMM tiles keep two workgroups per CU where the engine's
// accumulators allow it: FP64 8-wave tiles are held to 128 VGPRs (4 waves per
// SIMD); FP32 (FP32 partial and FP64 folded accumulators) and split-BF16
// (three accumulator sets) 8-wave tiles to 256.  The grouped kernels (which
// also carry the work-list search) are left to the compiler (GWPE 1), except
// the half transform and J^q, whose trimmed q-tiles (GTILE) would otherwise
// take FP64 past 128 VGPRs and one workgroup per CU, and Fock, whose
// direct-staged path would.
template <int P, class Cfg>
constexpr int gemm_wpe() {
  return Cfg::NT == 1024 ? 4 : Cfg::NT == 512 ? (P == kF64 ? 4 : 2) : 1;
}
#define GEMM_SMEM smem_bytes<typename EngineOf<P>::type, Cfg>()
#define GEMM_WPE (gemm_wpe<P, Cfg>())
RIF_STEP_KERNELS(half, HalfArgs, GEMM_SMEM, Cfg::NT, false, GEMM_WPE, GEMM_WPE, half_g_tile)
// the pre-split half transform and J^q stage piece planes directly (split modes)
#define GEMM_SMEM_DMA \
  (kPieces<P> > 0 ? smem_bytes_dma<typename EngineOf<P>::type, Cfg>() : smem_bytes<typename EngineOf<P>::type, Cfg>())
RIF_STEP_KERNELS(halfp, HalfArgs, GEMM_SMEM_DMA, Cfg::NT, false, GEMM_WPE, GEMM_WPE, halfp_g_tile)
RIF_STEP_KERNELS(mo, MoArgs, GEMM_SMEM, Cfg::NT, false, GEMM_WPE, 1, mo_tile)
RIF_STEP_KERNELS(jao, JaoArgs, GEMM_SMEM, Cfg::NT, true, GEMM_WPE, GEMM_WPE, jao_g_tile)
RIF_STEP_KERNELS(jaop, JaoArgs, GEMM_SMEM_DMA, Cfg::NT, false, GEMM_WPE, 1, jaop_one_tile)
// the FP64 64x64 K^q tile: three unpadded direct-load stages
#define KAO_SMEM (P == kF64 && Cfg::BM == 64 ? 3 * 2 * EngF64T<16, 0>::template stage_bytes<64>() : GEMM_SMEM)
RIF_STEP_KERNELS(kao, KaoArgs, KAO_SMEM, Cfg::NT, true, GEMM_WPE, 1, kao_tile)
RIF_STEP_KERNELS(gemm, GemmArgs, GEMM_SMEM, Cfg::NT, false, GEMM_WPE, 1, gemm_tile)
RIF_STEP_KERNELS(fock, FockArgs, GEMM_SMEM, Cfg::NT, false, GEMM_WPE, GEMM_WPE, fock_tile)
RIF_STEP_KERNELS(yd, YdArgs, GEMM_SMEM, Cfg::NT, false, GEMM_WPE, 1, yd_tile)
RIF_STEP_KERNELS(ydz, YdzArgs, kYdzLds * 8, 256, false, 1, 1, ydz_tile)
RIF_STEP_KERNELS(jkp, JkArgs, 16, 256, false, 1, 1, jkp_tile)
RIF_STEP_KERNELS(jkr, JkArgs, 16, 256, false, 1, 1, jkr_tile)
RIF_STEP_KERNELS(coef, CoefArgs, 256 * 8, 256, false, 1, 1, coef_tile)
RIF_STEP_KERNELS(energy, EnergyArgs, kEnergySmem, kEnergyThreads, false, 1, 1, energy_tile)
RIF_STEP_KERNELS(fred, FockRedArgs, 16, 256, false, 1, 1, fred_tile)
RIF_STEP_KERNELS(grad, GradArgs, 16, 256, false, 1, 1, grad_tile)
RIF_STEP_KERNELS(psplit, PSplitArgs, 16, 256, false, 1, 1, psplit_tile)
RIF_STEP_KERNELS(bsplit, BSplitArgs, 16, 256, false, 1, 1, bsplit_tile)

// ---------------------------------------------------------------------------
// Launchers.  Each GEMM-shaped step exists in four tile variants per mode:
//   0: 128x128   1: 64x64   2: 128x64   3: 64x128 (FP64/FP32) or a second
//   128x128 wave layout (split engines)   (outputs per workgroup)
// pick_variant() chooses one per (step, mode, shape): a wave-quantisation
// model by default, or the fastest measured one when autotuning is on.

template <int BK> struct Vars;
template <> struct Vars<16> {  // FP64 / FP32 engines: 8 waves (measured ~10% over 4 at these shapes)
  using V0 = TileCfg<128, 128, 16, 64, 32>;
  using V1 = TileCfg<64, 64, 16, 32, 16>;
  using V2 = TileCfg<128, 64, 16, 32, 32>;
  using V3 = TileCfg<64, 128, 16, 32, 32>;
};
// Split engines: 128x128 as 16 waves of 32x32 (four waves per SIMD) or 8 waves
// of 64x32 (fewer fragment reads from LDS per MFMA, two waves per SIMD), then
// the 4-wave 64x64 and 128x64 tiles.
template <> struct Vars<32> {
  using V0 = TileCfg<128, 128, 32, 32, 32>;
  using V1 = TileCfg<64, 64, 32, 32, 32>;
  using V2 = TileCfg<128, 64, 32, 64, 32>;
  using V3 = TileCfg<128, 128, 32, 64, 32>;
};
struct Cfg256 { static constexpr int NT = 256; };  // element-wise steps
struct CfgEnergy { static constexpr int NT = kEnergyThreads; };

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

// Relative time of `nwg` tiles with `wg_per_cu` resident workgroups per CU:
// whole rounds of 256*wg_per_cu tiles, each round as long as one tile running
// at 1/wg_per_cu of a CU.
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

// Fraction of each tile that lands on real outputs, per step (for the model).
template <class Cfg> static double useful_half(const HalfArgs& a) { return (double)a.nw / (cdiv(a.nw, Cfg::BM) * Cfg::BM); }
template <class Cfg> static double useful_halfp(const HalfArgs& a) { return useful_half<Cfg>(a); }
template <class Cfg> static double useful_mo(const MoArgs& a) { return (double)a.nw / (cdiv(a.nw, Cfg::BN) * Cfg::BN); }
template <class Cfg> static double useful_jao(const JaoArgs& a) { return (double)a.nw / (cdiv(a.nw, Cfg::BM) * Cfg::BM); }
template <class Cfg> static double useful_jaop(const JaoArgs& a) { return useful_jao<Cfg>(a); }
template <class Cfg> static double useful_kao(const KaoArgs& a) {
  const long nbk = cdiv(a.nb, Cfg::BM);
  return (double)a.nb * (a.nb + 1) / 2 / (nbk * (nbk + 1) / 2 * (double)Cfg::BM * Cfg::BM);
}
template <class Cfg> static double useful_yd(const YdArgs& a) {
  return (double)a.nb * a.nw / ((double)cdiv(a.nb, Cfg::BM) * Cfg::BM * cdiv(a.nw, Cfg::BN) * Cfg::BN);
}
template <class Cfg> static double useful_fock(const FockArgs& a) {
  return (double)a.nb * a.nw / ((double)cdiv(a.nb, Cfg::BM) * Cfg::BM * cdiv(a.nw, Cfg::BN) * Cfg::BN);
}

// Launch grid of a single-molecule step: one workgroup per tile, except the
// persistent pre-split half transform and J^q of the split modes (one per
// resident slot, from the compiled kernel's occupancy).
#define RIF_TILE_GRID(NAME, ARGS) \
  template <int P, class Cfg>     \
  static long NAME##_grid(const ARGS& a) { return NAME##_tiles<P, Cfg>(a); }
RIF_TILE_GRID(half, HalfArgs)
RIF_TILE_GRID(mo, MoArgs)
RIF_TILE_GRID(jao, JaoArgs)
RIF_TILE_GRID(kao, KaoArgs)
RIF_TILE_GRID(fock, FockArgs)
template <int P, class Cfg, class KernelOf>
static long resident_grid(long n, KernelOf kernel_of) {
  static std::atomic<int> per_cu{0};   // queried once per kernel; threads may race to store the same value
  int v = per_cu.load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kernel_of(), Cfg::NT, 0) != hipSuccess || v < 1) {
      (void)hipGetLastError();
      v = 1;
    }
    per_cu.store(v, std::memory_order_relaxed);
  }
  return std::min(n, 256L * v);
}
template <int P, class Cfg>
static long halfp_grid(const HalfArgs& a) {
  const long n = halfp_tiles<P, Cfg>(a);
  if constexpr (kPieces<P> > 0)
    return resident_grid<P, Cfg>(n, [] { return (const void*)&k_halfp<P, Cfg>; });
  return n;
}
// every J^q from piece planes is persistent (the kernel exists in the split modes only)
template <int P, class Cfg>
static long jaop_grid(const JaoArgs& a) {
  return resident_grid<P, Cfg>(jaop_tiles<P, Cfg>(a), [] { return (const void*)&k_jaop<P, Cfg>; });
}

// Single-molecule launch of a GEMM-shaped step with variant selection.
#define RIF_GEMM_STEP(NAME, ARGS, LABEL, NVAR, ...)                                                     \
  template <int P>                                                                                      \
  static rif_status step_##NAME(rif_ctx* c, const ARGS& a) {                                            \
    auto run = [&](int v) {                                                                             \
      return dispatch<P>(v, [&](auto cfg) {                                                             \
        using Cfg = decltype(cfg);                                                                      \
        if constexpr (NVAR == 2 && Cfg::BM != Cfg::BN) {                                                \
          return fail(c, RIF_ENOTSUP, LABEL ": non-square tile variant");                               \
        } else {                                                                                        \
          hipLaunchKernelGGL((k_##NAME<P, Cfg>), dim3((unsigned)NAME##_grid<P, Cfg>(a)), dim3(Cfg::NT),  \
                             0, c->stream, a);                                                          \
          return check_launch(c, LABEL);                                                                \
        }                                                                                               \
      });                                                                                               \
    };                                                                                                  \
    const int hv = best_of(NVAR, [&](int v) {                                                           \
      return dispatch<P>(v, [&](auto cfg) {                                                             \
        using Cfg = decltype(cfg);                                                                      \
        return est_cost(NAME##_tiles<P, Cfg>(a), wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN,                \
                        useful_##NAME<Cfg>(a));                                                         \
      });                                                                                               \
    });                                                                                                 \
    const int v = pick_variant(c, LABEL, {P, __VA_ARGS__}, NVAR, hv, run);                              \
    if (v < 0) return RIF_EHIP;                                                                         \
    ProfScope ps(c, LABEL);                                                                             \
    return run(v);                                                                                      \
  }

RIF_GEMM_STEP(half, HalfArgs, "half_transform", 4, a.nb, a.nr, a.nw, a.nmo)
RIF_GEMM_STEP(halfp, HalfArgs, "half_transform_presplit", 4, a.nb, a.nr, a.nw, a.nmo)
template <int P>
static rif_status step_half_any(rif_ctx* c, const HalfArgs& a) {
  if constexpr (P != kF64)
    if (b_presplit<P>(a)) return step_halfp<P>(c, a);
  return step_half<P>(c, a);
}
RIF_GEMM_STEP(mo, MoArgs, "mo_transform", 4, a.nb, a.na, a.nw, a.nmo)
RIF_GEMM_STEP(jao, JaoArgs, "jao", 4, a.nb, a.na, a.nw)
RIF_GEMM_STEP(jaop, JaoArgs, "jao_presplit", 4, a.nb, a.na, a.nw)
// J^q from the pre-split b where the build has it (split modes), else split on load.
template <int P>
static rif_status step_jao_any(rif_ctx* c, const JaoArgs& a) {
  if constexpr (kPieces<P> > 0)
    if (a.Bj.p) return step_jaop<P>(c, a);
  return step_jao<P>(c, a);
}
RIF_GEMM_STEP(kao, KaoArgs, "kao", 2, a.nb, a.na, a.nw)
RIF_GEMM_STEP(fock, FockArgs, "fock", 4, a.nb, a.nw, a.nmo, a.nsplit)
// The direct contraction has few q (n_omega) and many nu (n_bf) columns: its
// first variant for the FP64/FP32 engines is a 256x128 16-wave tile, so one
// tile spans all q of a split (b_half read once) and the b_mo coefficients are
// re-read only once per 256 nu.
template <int P>
struct YdVars {
  using VS = Vars<EngineOf<P>::type::BK>;
  using V0 = typename std::conditional<EngineOf<P>::type::BK == 16, TileCfg<256, 128, 16, 64, 32>,
                                       typename VS::V0>::type;
  using V1 = typename VS::V1;
  using V2 = typename VS::V2;
  using V3 = typename VS::V3;
};
template <int P>
static rif_status step_yd(rif_ctx* c, const YdArgs& a) {
  auto with = [&](int v, auto&& f) {
    using YV = YdVars<P>;
    switch (v) {
      case 0: return f(typename YV::V0());
      case 1: return f(typename YV::V1());
      case 2: return f(typename YV::V2());
      default: return f(typename YV::V3());
    }
  };
  auto run = [&](int v) {
    return with(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_yd<P, Cfg>), dim3((unsigned)yd_tiles<P, Cfg>(a)), dim3(Cfg::NT), 0, c->stream, a);
      return check_launch(c, "direct_gradient");
    });
  };
  const int hv = best_of(4, [&](int v) {
    return with(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      return est_cost(yd_tiles<P, Cfg>(a), wg_per_cu<P, Cfg>(), Cfg::BM * Cfg::BN, useful_yd<Cfg>(a));
    });
  });
  const int v = pick_variant(c, "direct_gradient", {P, a.nb, a.na, a.nw, a.nsplit}, 4, hv, run);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "direct_gradient");
  return run(v);
}

// Fixed-shape steps (64x64 FP64 GEMM tiles, 256-thread element-wise tiles).
using CfgSmall = TileCfg<64, 64, 16, 32, 32>;
#define RIF_FIXED_STEP(NAME, ARGS, LABEL, PP, CFG)                                              \
  static rif_status step1_##NAME(rif_ctx* c, const ARGS& a) {                                  \
    ProfScope ps(c, LABEL);                                                                     \
    hipLaunchKernelGGL((k_##NAME<PP, CFG>), dim3((unsigned)NAME##_tiles<PP, CFG>(a)), dim3(CFG::NT), 0, \
                       c->stream, a);                                                           \
    return check_launch(c, LABEL);                                                             \
  }
RIF_FIXED_STEP(gemm, GemmArgs, "small_gemm", kF64, CfgSmall)
RIF_FIXED_STEP(coef, CoefArgs, "coef", kF64, Cfg256)
RIF_FIXED_STEP(energy, EnergyArgs, "energy", kF64, CfgEnergy)
RIF_FIXED_STEP(fred, FockRedArgs, "fock_reduce", kF64, Cfg256)
RIF_FIXED_STEP(grad, GradArgs, "grad", kF64, Cfg256)
template <int P>
static rif_status step_ydz(rif_ctx* c, const YdzArgs& a) {
  ProfScope ps(c, "direct_coef");
  hipLaunchKernelGGL((k_ydz<P, Cfg256>), dim3((unsigned)ydz_tiles<P, Cfg256>(a)), dim3(256), 0, c->stream, a);
  return check_launch(c, "direct_coef");
}

rif_status op_gemm_kn(rif_ctx* c, int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                      double* out, long ldo) {
  return step1_gemm(c, GemmArgs{M, N, K, A, lda, B, ldb, out, ldo, 1, K, 0});
}
template <int P>
static rif_status step_psplit(rif_ctx* c, const PSplitArgs& a) {
  if constexpr (kPieces<P> == 0) {
    return RIF_OK;
  } else {
    ProfScope ps(c, "presplit");
    hipLaunchKernelGGL((k_psplit<P, Cfg256>), dim3((unsigned)psplit_tiles<P, Cfg256>(a)), dim3(256), 0, c->stream, a);
    return check_launch(c, "presplit");
  }
}
template <int P>
static rif_status step1_jk(rif_ctx* c, const JkArgs& a) {
  rif_status st;
  {
    ProfScope ps(c, "jk_mo_partial");
    hipLaunchKernelGGL((k_jkp<P, Cfg256>), dim3((unsigned)jkp_tiles<P, Cfg256>(a)), dim3(256), 0, c->stream, a);
    if ((st = check_launch(c, "jk_mo_partial"))) return st;
  }
  ProfScope ps(c, "jk_mo_reduce");
  hipLaunchKernelGGL((k_jkr<P, Cfg256>), dim3((unsigned)jkr_tiles<P, Cfg256>(a)), dim3(256), 0, c->stream, a);
  return check_launch(c, "jk_mo_reduce");
}

// ---- workspace plan of one molecule (shared by the single and batched paths)
struct Plan {
  int nb, na, nw, nmo, npairs, ncwo;
  int jk_nsplit, fock_nsplit, nparts, lam_split, small_kc, yd_nsplit;
  long yd_kc;
  size_t o_part, o_hc, o_a, o_b, o_yp, o_y, o_ep, o_lp, o_cs, o_ds, bytes;
  size_t o_ydp, o_zt, o_bt, bytes_direct;   // the gradient without per-MO AO matrices
  Plan(int nb_, int na_, int npairs_, int ncwo_, int nmo_) {
    nb = nb_; na = na_; npairs = npairs_; ncwo = ncwo_; nmo = nmo_;
    nw = npairs * (1 + ncwo);
    const long w2 = (long)nw * nw;
    const long nx = cdiv(w2, 256);
    jk_nsplit = (int)std::max(1L, std::min((long)na, (1024L + nx - 1) / nx));
    // fock split-K over the stacked slabs' slices, sized so the 128x128-tile
    // launch fills the 512 slots of two workgroups per CU in one round (the
    // 64x64 one then fills four per CU in about two); at most one split per
    // 32-deep slice
    const long t128 = (long)cdiv(nb, 128) * cdiv(nw, 128);
    const long smax = 2L * nw * cdiv(nb, 32);
    fock_nsplit = (int)std::max(1L, std::min(smax, 512L / t128));
    nparts = (int)nx;
    // lambda = C^T Y (n_mo x n_omega, k = n_bf) sits on the main chain: k split
    // so its launch has about 256 tiles of 64x64, at least two 16-deep slices
    // each.  H C_Omega runs on the side stream, in the shadow of the half
    // transform, and writes HC in one piece (no partials to add up later).
    {
      const long tiles = cdiv(nb, 64) * cdiv(nw, 64);
      const int slices = cdiv(nb, 16);
      const int want = (int)std::max(1L, std::min((long)std::max(1, slices / 2), (long)cdiv(256, tiles)));
      small_kc = 16 * cdiv(slices, want);
      lam_split = cdiv(nb, small_kc);
    }
    Carve cv;
    o_part = cv.take<double>(2L * jk_nsplit * w2);
    o_hc = cv.take<double>((size_t)nb * nw);
    o_a = cv.take<double>((size_t)w2);
    o_b = cv.take<double>((size_t)w2);
    o_yp = cv.take<double>((size_t)fock_nsplit * nb * nw);
    o_y = cv.take<double>((size_t)nb * nw);
    o_ep = cv.take<double>((size_t)nparts);
    o_lp = cv.take<double>((size_t)lam_split * nmo * nw);
    o_cs = cv.take<unsigned short>((size_t)3 * nw * round32(nb));   // C_Omega^T pieces (split modes)
    o_ds = cv.take<unsigned short>((size_t)3 * nw * round32(na));   // d^T pieces (split modes)
    bytes = cv.off;
    // direct gradient: split-K over (r, l), sized so a 64x64-tile launch has
    // at most 2048 tiles (two full rounds of four per CU; rounding up instead
    // would spill a few tiles into a third round); each split a multiple of
    // 32 deep
    {
      const long K = (long)na * nw, t64 = cdiv(nb, 64) * cdiv(nw, 64);
      const long slices = cdiv(K, 32L);
      const long ns = std::max(1L, std::min(slices, 2048L / t64));
      yd_kc = 32L * cdiv(slices, ns);
      yd_nsplit = (int)cdiv(K, yd_kc);
    }
    o_ydp = cv.take<double>((size_t)yd_nsplit * nb * nw);
    o_zt = cv.take<double>((size_t)na * nw);
    o_bt = cv.take<double>((size_t)w2);
    bytes_direct = cv.off;
  }
};

// All argument blocks of one build of one molecule, workspace at `ws`.
struct BuildArgs {
  PSplitArgs psc, psd;
  HalfArgs half; MoArgs mo; JkArgs jk; JaoArgs jao; KaoArgs kao;
  GemmArgs hc; CoefArgs coef; EnergyArgs energy; FockArgs fock; FockRedArgs fred; GemmArgs lam; GradArgs grad;
  YdzArgs ydz; YdArgs yd; FockRedArgs ydred;
};
static BuildArgs make_build_args(const Plan& pl, const rif_instance& in, int prec, int functional, char* ws,
                                 int* flag) {
  BuildArgs A;
  const int nb = pl.nb, na = pl.na, nw = pl.nw, nmo = pl.nmo;
  double* part = (double*)(ws + pl.o_part);
  double* HC = (double*)(ws + pl.o_hc);
  double* Ac = (double*)(ws + pl.o_a);
  double* Bc = (double*)(ws + pl.o_b);
  double* Yp = (double*)(ws + pl.o_yp);
  double* Y = (double*)(ws + pl.o_y);
  double* Ep = (double*)(ws + pl.o_ep);
  double* Lp = (double*)(ws + pl.o_lp);
  unsigned short* Cs = (unsigned short*)(ws + pl.o_cs);
  unsigned short* Ds = (unsigned short*)(ws + pl.o_ds);
  const int lc = round32(nb), ldd = round32(na);
  A.psc = PSplitArgs{in.C, (long)nmo, nw, nb, lc, Cs, (long)nw * lc};
  A.psd = PSplitArgs{in.d, (long)nw, nw, na, ldd, Ds, (long)nw * ldd};
  const Planes cs{Cs, (long)nw * lc, lc}, ds{Ds, (long)nw * ldd, ldd};
  A.half = HalfArgs{nb, nw, nmo, (long)na * nb, in.b, in.C, in.b_half, cs, Planes{nullptr, 0, 0}, nullptr,
                    half_dma_ok(nb, nmo, nw, in.b, in.C)};
  if (in.b_split && (prec == RIF_BF16X3 || prec == RIF_BF16X6 || prec == RIF_FP16X3)) {
    const int lb = round32(nb);
    A.half.Bs = Planes{(const unsigned short*)in.b_split, (long)na * nb * lb, lb};
  } else if (in.b_split && prec == RIF_FP32) {
    A.half.bf = (const float*)in.b_split;
  }
  A.mo = MoArgs{nb, na, nw, nmo, in.b_half, in.C, in.b_mo, in.d, cs,
                nb % 2 == 0 && nmo % 2 == 0 && ((uintptr_t)in.b_half | (uintptr_t)in.C) % 16 == 0};
  A.jk = JkArgs{na, nw, pl.jk_nsplit, in.b_mo, in.d, part, in.J, in.K};
  A.jao = JaoArgs{nb, na, nw, in.b, in.d, in.Jn, ds, Planes{nullptr, 0, 0},
                  nb % 2 == 0 && nw % 2 == 0 && ((uintptr_t)in.b | (uintptr_t)in.d) % 16 == 0};
  if (in.b_split && (prec == RIF_BF16X3 || prec == RIF_BF16X6 || prec == RIF_FP16X3)) {
    const long npc = prec == RIF_BF16X6 ? 3 : 2;
    const int lj = round32(na);
    const unsigned short* j0 = (const unsigned short*)in.b_split + npc * (long)na * nb * round32(nb);
    A.jao.Bj = Planes{j0, (long)nb * nb * lj, lj};
  }
  A.kao = KaoArgs{nb, na, nw, in.b_half, in.Kn, nb % 2 == 0 && (uintptr_t)in.b_half % 16 == 0};
  A.hc = GemmArgs{nb, nw, nb, in.H, (long)nb, in.C, (long)nmo, HC, (long)nw, 1, nb, (long)nb * nw};
  A.coef = CoefArgs{functional, nw, pl.npairs, pl.ncwo, in.pair_of, in.occ, in.J, in.K, Ac, Bc, Ep};
  A.energy = EnergyArgs{nw, pl.npairs, pl.ncwo, nb, nmo, pl.nparts, in.pair_of, in.occ, in.C, HC, Ep, in.energy,
                        flag};
  A.fock = FockArgs{nb, nw, nmo, pl.fock_nsplit, in.Jn, in.Kn, Ac, Bc, in.C, Yp,
                    nb % 2 == 0 && nw % 2 == 0 && nmo % 2 == 0 &&
                        ((uintptr_t)in.Jn | (uintptr_t)in.Kn | (uintptr_t)in.C) % 16 == 0};
  A.fred = FockRedArgs{nb, nw, pl.fock_nsplit, Yp, in.occ, HC, Y};
  A.lam = GemmArgs{nmo, nw, nb, in.C, (long)nmo, Y, (long)nw, Lp, (long)nw, pl.lam_split, pl.small_kc,
                   (long)nmo * nw};
  A.grad = GradArgs{nmo, nw, pl.lam_split, Lp, in.lambda, in.grad, flag};
  void* Zt = ws + pl.o_zt;
  void* Bt = ws + pl.o_bt;
  double* Ydp = (double*)(ws + pl.o_ydp);
  A.ydz = YdzArgs{na, nw, Ac, Bc, in.d, Zt, Bt};
  A.yd = YdArgs{nb, na, nw, pl.yd_nsplit, pl.yd_kc, in.b_half, in.b_mo, Zt, Bt, Ydp};
  A.ydred = FockRedArgs{nb, nw, pl.yd_nsplit, Ydp, in.occ, HC, Y};
  return A;
}

template <int P>
static rif_status run_transform(rif_ctx* c, const PSplitArgs& ps, const HalfArgs& h, const MoArgs& m) {
  rif_status st = step_psplit<P>(c, ps);
  if (st || (st = step_half_any<P>(c, h))) return st;
  return step_mo<P>(c, m);
}
template <int P>
static rif_status run_jk_ao(rif_ctx* c, const PSplitArgs& ps, const JaoArgs& j, const KaoArgs& k) {
  rif_status st = kPlanesHalfJao<P> ? step_psplit<P>(c, ps) : RIF_OK;
  if (st || (st = step_jao<P>(c, j))) return st;
  return step_kao<P>(c, k);
}
template <int P>
static rif_status run_energy_grad(rif_ctx* c, const BuildArgs& A) {
  rif_status st;
  if ((st = step1_gemm(c, A.hc))) return st;
  if ((st = step1_coef(c, A.coef))) return st;
  if ((st = step1_energy(c, A.energy))) return st;
  if ((st = step_fock<P>(c, A.fock))) return st;
  if ((st = step1_fred(c, A.fred))) return st;
  if ((st = step1_gemm(c, A.lam))) return st;
  return step1_grad(c, A.grad);
}

// ---- mode dispatch (the single-molecule entry points the ABI layer calls) ----
#define RIF_PREC_SWITCH(prec, call)                                              \
  switch (prec) {                                                                \
    case kF64: { constexpr int P = kF64; return call; }                          \
    case kF32: { constexpr int P = kF32; return call; }                          \
    case kBF16x3: { constexpr int P = kBF16x3; return call; }                    \
    case kBF16x6: { constexpr int P = kBF16x6; return call; }                    \
    case kF16x3: { constexpr int P = kF16x3; return call; }                      \
    default: return fail(c, RIF_ENOTSUP, "precision mode not available");       \
  }

static bool prec_ok(int prec) { return prec >= kF64 && prec <= kF16x3; }

rif_status op_transform(rif_ctx* c, int prec, int nb, int na, int nw, int nmo, const double* b, const double* C,
                        void* bh, void* bmo, double* d) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  const int lc = round32(nb);
  Carve cv;
  const size_t o_cs = cv.take<unsigned short>((size_t)3 * nw * lc);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  unsigned short* Cs = (unsigned short*)((char*)c->ws + o_cs);
  const Planes cs{Cs, (long)nw * lc, lc};
  const PSplitArgs ps{C, (long)nmo, nw, nb, lc, Cs, (long)nw * lc};
  const HalfArgs h{nb, nw, nmo, (long)na * nb, b, C, bh, cs, Planes{}, nullptr, half_dma_ok(nb, nmo, nw, b, C)};
  const MoArgs m{nb, na, nw, nmo, bh, C, bmo, d, cs,
                 nb % 2 == 0 && nmo % 2 == 0 && ((uintptr_t)bh | (uintptr_t)C) % 16 == 0};
  RIF_PREC_SWITCH(prec, run_transform<P>(c, ps, h, m))
}

rif_status op_half_slabs_f64(rif_ctx* c, int nb, long nslab, int nw, int nmo, const double* slabs, const double* C,
                             double* out) {
  const HalfArgs h{nb, nw, nmo, nslab * nb, slabs, C, out, Planes{}, Planes{}, nullptr,
                   half_dma_ok(nb, nmo, nw, slabs, C)};
  return step_half<kF64>(c, h);
}

rif_status op_jk_mo(rif_ctx* c, int prec, int na, int nw, const void* bmo, const double* d, double* J, double* K) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  const long w2 = (long)nw * nw;
  const long nx = cdiv(w2, 256);
  const int nsplit = (int)std::max(1L, std::min((long)na, (1024L + nx - 1) / nx));
  Carve cv;
  const size_t o_part = cv.take<double>(2L * nsplit * w2);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  const JkArgs a{na, nw, nsplit, bmo, d, (double*)((char*)c->ws + o_part), J, K};
  RIF_PREC_SWITCH(prec, step1_jk<P>(c, a))
}

// ---- MO J/K without allocation (rif_jk_mo_noalloc) --------------------------
// The per-slice partials live in this file-scope device array instead of the
// context's arena.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, so host
// code uses only the device address that hipGetSymbolAddress returns for it
// (resolved once per context, at rif_create, with the context's device current).
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

rif_status op_static_scratch_init(rif_ctx* c) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    return fail(c, RIF_EHIP, std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
  }
  c->scratch = p;
  c->scratch_bytes = kStaticScratchBytes;
  return RIF_OK;
}

rif_status op_jk_mo_noalloc(rif_ctx* c, int prec, int na, int nw, const void* bmo, const double* d, double* J,
                            double* K) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  if (!c->scratch) return fail(c, RIF_EHIP, "rif_jk_mo_noalloc: the static scratch could not be resolved");
  const long w2 = (long)nw * nw;
  const long nx = cdiv(w2, 256);
  const int nsplit = (int)std::max(1L, std::min((long)na, (1024L + nx - 1) / nx));
  const size_t need = sizeof(double) * 2 * (size_t)nsplit * (size_t)w2;
  if (need > c->scratch_bytes)
    return fail(c, RIF_ENOMEM, "rif_jk_mo_noalloc: needs " + std::to_string(need) + " bytes of scratch, more than its " +
                                   std::to_string(c->scratch_bytes) + " (n_omega above 1024)");
  // the same kernels and split as rif_jk_mo, on the static partials; no event
  // pairs either (profiling is suspended for the call)
  const JkArgs a{na, nw, nsplit, bmo, d, (double*)c->scratch, J, K};
  const bool prof = c->prof;
  c->prof = false;
  rif_status st;
  switch (prec) {
    case kF64: st = step1_jk<kF64>(c, a); break;
    case kF32: st = step1_jk<kF32>(c, a); break;
    case kBF16x3: st = step1_jk<kBF16x3>(c, a); break;
    case kBF16x6: st = step1_jk<kBF16x6>(c, a); break;
    default: st = step1_jk<kF16x3>(c, a); break;
  }
  c->prof = prof;
  return st;
}

rif_status op_jk_ao(rif_ctx* c, int prec, int nb, int na, int nw, const double* b, const void* bh,
                    const double* d, void* Jn, void* Kn) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  const int ldd = round32(na);
  Carve cv;
  const size_t o_ds = cv.take<unsigned short>((size_t)3 * nw * ldd);
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  unsigned short* Ds = (unsigned short*)((char*)c->ws + o_ds);
  const PSplitArgs ps{d, (long)nw, nw, na, ldd, Ds, (long)nw * ldd};
  const JaoArgs j{nb, na, nw, b, d, Jn, Planes{Ds, (long)nw * ldd, ldd}, Planes{nullptr, 0, 0},
                  nb % 2 == 0 && nw % 2 == 0 && ((uintptr_t)b | (uintptr_t)d) % 16 == 0};
  const KaoArgs k{nb, na, nw, bh, Kn, nb % 2 == 0 && (uintptr_t)bh % 16 == 0};
  RIF_PREC_SWITCH(prec, run_jk_ao<P>(c, ps, j, k))
}

rif_status op_energy_grad(rif_ctx* c, int prec, int functional, int nb, int nmo, int npairs, int ncwo,
                          const int* pair_of, const double* H, const double* C, const double* occ,
                          const double* J, const double* K, const void* Jn, const void* Kn, double* energy,
                          double* lambda, double* grad) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  const Plan pl(nb, 1, npairs, ncwo, nmo);
  rif_status st = ws_reserve(c, pl.bytes);
  if (st) return st;
  rif_instance in{};
  in.n_bf = nb; in.n_aux = 1; in.n_pairs = npairs; in.n_cwo = ncwo; in.n_mo = nmo;
  in.H = H; in.C = C; in.occ = occ; in.pair_of = pair_of; in.J = (double*)J; in.K = (double*)K;
  in.Jn = (void*)Jn; in.Kn = (void*)Kn; in.energy = energy; in.lambda = lambda; in.grad = grad;
  const BuildArgs A = make_build_args(pl, in, prec, functional, (char*)c->ws, c->dflag);
  RIF_PREC_SWITCH(prec, run_energy_grad<P>(c, A))
}

// ---- one whole build (rif_build) ------------------------------------------
// The main stream runs the chain that carries the time (half, mo, J^q, K^q,
// coefficients, Fock, lambda, G).  H C_Omega, the J/K-MO reduction and the
// energy feed neither of their neighbours, so they run on the side stream:
//   main: fork | half  mo  [e_mo] J^q  K^q  (wait e_side) coef [e_coef]  fock fred lambda grad  (wait e_energy)
//   side:      | H C_Omega  (wait e_mo) jk_mo [e_side]  (wait e_coef) energy [e_energy]
// Every kernel and reduction order is the same as in the one-stream order.
struct OnStream {  // launches of the enclosed steps go to `s`
  rif_ctx* c;
  hipStream_t saved;
  OnStream(rif_ctx* c_, hipStream_t s) : c(c_), saved(c_->stream) { c->stream = s; }
  ~OnStream() { c->stream = saved; }
};

template <int P>
static rif_status run_build(rif_ctx* c, const BuildArgs& A) {
  hipStream_t main = c->stream, side = c->side;
  hipEvent_t e_fork = c->ev[0], e_mo = c->ev[1], e_side = c->ev[2], e_coef = c->ev[3], e_energy = c->ev[4];
  rif_status st;
  auto hip = [&](hipError_t e) { return e == hipSuccess ? RIF_OK : fail(c, RIF_EHIP, "stream fork/join failed"); };
  if ((st = hip(hipEventRecord(e_fork, main))) || (st = hip(hipStreamWaitEvent(side, e_fork, 0)))) return st;
  {
    OnStream on(c, side);
    if ((st = step1_gemm(c, A.hc))) return st;
  }
  if ((st = step_psplit<P>(c, A.psc)) || (st = step_half_any<P>(c, A.half)) || (st = step_mo<P>(c, A.mo))) return st;
  if ((st = hip(hipEventRecord(e_mo, main)))) return st;
  {
    OnStream on(c, side);
    if ((st = hip(hipStreamWaitEvent(side, e_mo, 0))) || (st = step1_jk<P>(c, A.jk)) ||
        (st = hip(hipEventRecord(e_side, side))))
      return st;
  }
  if (((kPlanesHalfJao<P> || (kPieces<P> > 0 && A.jao.Bj.p)) && (st = step_psplit<P>(c, A.psd))) ||
      (st = step_jao_any<P>(c, A.jao)) || (st = step_kao<P>(c, A.kao)))
    return st;
  if ((st = hip(hipStreamWaitEvent(main, e_side, 0))) || (st = step1_coef(c, A.coef)) ||
      (st = hip(hipEventRecord(e_coef, main))))
    return st;
  {
    OnStream on(c, side);
    if ((st = hip(hipStreamWaitEvent(side, e_coef, 0))) || (st = step1_energy(c, A.energy)) ||
        (st = hip(hipEventRecord(e_energy, side))))
      return st;
  }
  if ((st = step_fock<P>(c, A.fock)) || (st = step1_fred(c, A.fred)) || (st = step1_gemm(c, A.lam)) ||
      (st = step1_grad(c, A.grad)))
    return st;
  return hip(hipStreamWaitEvent(main, e_energy, 0));
}

// The same energy, lambda and G without J^q/K^q: after the transforms, the
// coefficients (side stream: H C_Omega, J/K, energy as in run_build), then
// Zt/Bt, the contraction over (r, l), the fixed-order sum with n_q H c_q,
// lambda = C^T Y and G.
template <int P>
static rif_status run_build_direct(rif_ctx* c, const BuildArgs& A) {
  hipStream_t main = c->stream, side = c->side;
  hipEvent_t e_fork = c->ev[0], e_mo = c->ev[1], e_side = c->ev[2], e_coef = c->ev[3], e_energy = c->ev[4];
  rif_status st;
  auto hip = [&](hipError_t e) { return e == hipSuccess ? RIF_OK : fail(c, RIF_EHIP, "stream fork/join failed"); };
  if ((st = hip(hipEventRecord(e_fork, main))) || (st = hip(hipStreamWaitEvent(side, e_fork, 0)))) return st;
  {
    OnStream on(c, side);
    if ((st = step1_gemm(c, A.hc))) return st;
  }
  if ((st = step_psplit<P>(c, A.psc)) || (st = step_half_any<P>(c, A.half)) || (st = step_mo<P>(c, A.mo))) return st;
  if ((st = hip(hipEventRecord(e_mo, main)))) return st;
  {
    OnStream on(c, side);
    if ((st = hip(hipStreamWaitEvent(side, e_mo, 0))) || (st = step1_jk<P>(c, A.jk)) ||
        (st = hip(hipEventRecord(e_side, side))))
      return st;
  }
  if ((st = hip(hipStreamWaitEvent(main, e_side, 0))) || (st = step1_coef(c, A.coef)) ||
      (st = hip(hipEventRecord(e_coef, main))))
    return st;
  {
    OnStream on(c, side);
    if ((st = hip(hipStreamWaitEvent(side, e_coef, 0))) || (st = step1_energy(c, A.energy)) ||
        (st = hip(hipEventRecord(e_energy, side))))
      return st;
  }
  if ((st = step_ydz<P>(c, A.ydz)) || (st = step_yd<P>(c, A.yd)) || (st = step1_fred(c, A.ydred)) ||
      (st = step1_gemm(c, A.lam)) || (st = step1_grad(c, A.grad)))
    return st;
  return hip(hipStreamWaitEvent(main, e_energy, 0));
}

static rif_status ensure_side(rif_ctx* c) {
  if (c->side) return RIF_OK;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess)
    return fail(c, RIF_EHIP, "side stream creation failed");
  for (auto& e : c->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail(c, RIF_EHIP, "event creation failed");
  return RIF_OK;
}

rif_status op_build(rif_ctx* c, int prec, int functional, const rif_instance& in) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  rif_status st = ensure_side(c);
  if (st) return st;
  const Plan pl(in.n_bf, in.n_aux, in.n_pairs, in.n_cwo, in.n_mo);
  if ((st = ws_reserve(c, pl.bytes))) return st;
  const BuildArgs A = make_build_args(pl, in, prec, functional, (char*)c->ws, c->dflag);
  RIF_PREC_SWITCH(prec, run_build<P>(c, A))
}

unsigned long long presplit_b_bytes(int nb, int na, int prec) {
  const unsigned long long nr = (unsigned long long)na * nb;
  if (prec == RIF_FP32) return nr * nb * 4ull;
  if (prec == RIF_BF16X3 || prec == RIF_BF16X6 || prec == RIF_FP16X3) {
    const unsigned long long npc = prec == RIF_BF16X6 ? 3ull : 2ull;
    return npc * nr * (unsigned long long)round32(nb) * 2ull +                        // half transform
           npc * (unsigned long long)nb * nb * (unsigned long long)round32(na) * 2ull;  // J^q
  }
  return 0;
}

rif_status op_presplit_b(rif_ctx* c, int prec, int nb, int na, const double* b, void* out) {
  const int ld = round32(nb);
  const BSplitArgs a{b, (long)na * nb, nb, ld, out, (long)na * nb * ld};
  ProfScope ps(c, "presplit_b");
  switch (prec) {
    case RIF_FP32:
      hipLaunchKernelGGL((k_bsplit<kF32, Cfg256>), dim3((unsigned)bsplit_tiles<kF32, Cfg256>(a)), dim3(256), 0,
                         c->stream, a);
      break;
    case RIF_BF16X3:
      hipLaunchKernelGGL((k_bsplit<kBF16x3, Cfg256>), dim3((unsigned)bsplit_tiles<kBF16x3, Cfg256>(a)), dim3(256),
                         0, c->stream, a);
      break;
    case RIF_BF16X6:
      hipLaunchKernelGGL((k_bsplit<kBF16x6, Cfg256>), dim3((unsigned)bsplit_tiles<kBF16x6, Cfg256>(a)), dim3(256),
                         0, c->stream, a);
      break;
    case RIF_FP16X3:
      hipLaunchKernelGGL((k_bsplit<kF16x3, Cfg256>), dim3((unsigned)bsplit_tiles<kF16x3, Cfg256>(a)), dim3(256),
                         0, c->stream, a);
      break;
    default:
      return fail(c, RIF_ENOTSUP, "rif_presplit_b: FP32, BF16x3, BF16x6 or FP16x3 only");
  }
  rif_status st = check_launch(c, "presplit_b");
  if (st || prec == RIF_FP32) return st;
  // the second region: b in J^q's operand order
  const long npc = prec == RIF_BF16X6 ? 3 : 2;
  const int lj = round32(na);
  const BSplitJArgs aj{b, (long)nb * nb, na, lj, (unsigned short*)out + npc * (long)na * nb * ld, (long)nb * nb * lj};
  const dim3 grid((unsigned)cdiv((long)nb * nb, 64), (unsigned)cdiv(lj, 64));
  switch (prec) {
    case RIF_BF16X3: hipLaunchKernelGGL((k_bsplitj<kBF16x3>), grid, dim3(256), 0, c->stream, aj); break;
    case RIF_BF16X6: hipLaunchKernelGGL((k_bsplitj<kBF16x6>), grid, dim3(256), 0, c->stream, aj); break;
    default: hipLaunchKernelGGL((k_bsplitj<kF16x3>), grid, dim3(256), 0, c->stream, aj); break;
  }
  return check_launch(c, "presplit_b");
}

rif_status op_build_direct(rif_ctx* c, int prec, int functional, const rif_instance& in) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  rif_status st = ensure_side(c);
  if (st) return st;
  const Plan pl(in.n_bf, in.n_aux, in.n_pairs, in.n_cwo, in.n_mo);
  if ((st = ws_reserve(c, pl.bytes_direct))) return st;
  const BuildArgs A = make_build_args(pl, in, prec, functional, (char*)c->ws, c->dflag);
  RIF_PREC_SWITCH(prec, run_build_direct<P>(c, A))
}

// ---------------------------------------------------------------------------
// Batched builds of many molecules.  Every step is one persistent grouped
// launch over a work-list spanning all molecules (largest molecules first, so
// the small ones fill the tail), each step's tile variant chosen for the
// batch as a whole.  The launch sequence can be captured in a hipGraph once
// and replayed; nothing in it allocates or sets memory.

struct GroupStep {
  std::string name;
  int nvar = 1;              // tile variants available (1 for fixed steps)
  int variant = 0;
  void* args_d = nullptr;    // device array of per-molecule argument blocks
  long* off_d = nullptr;     // device [nvar][n+1] tile offsets
  std::vector<long> total;   // per variant
  std::vector<int> grid;     // per variant
};

struct BatchImpl {
  rif_ctx* c = nullptr;
  int prec = 0, n = 0;
  std::vector<int> order;    // molecule indices, largest first
  void* ws = nullptr;        // workspace of all molecules
  std::vector<void*> dev;    // device allocations to free
  GroupStep psc, psd, half, halfp, mo, jkp, jkr, jao, kao, hc, coef, energy, fock, fred, lam, grad;
  bool bpre = false;         // every molecule's b pre-split (grouped halfp in place of half)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

template <int P, class Cfg, class Args, class TilesFn>
static void group_offsets(const std::vector<Args>& a, TilesFn tiles, std::vector<long>& off) {
  off.assign(a.size() + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) off[i + 1] = off[i] + tiles(a[i]);
}

#define RIF_GROUP_SETUP(NAME, ARGS, LABEL, NVAR)                                                           \
  template <int P>                                                                                         \
  static rif_status setup_##NAME(BatchImpl* B, const std::vector<ARGS>& a) {                              \
    GroupStep& g = B->NAME;                                                                                \
    g.name = LABEL;                                                                                        \
    g.nvar = NVAR;                                                                                         \
    const int n = (int)a.size();                                                                           \
    std::vector<long> offs((size_t)NVAR * (n + 1));                                                        \
    g.total.assign(NVAR, 0);                                                                               \
    g.grid.assign(NVAR, 0);                                                                                \
    for (int v = 0; v < NVAR; ++v) {                                                                       \
      dispatch<P>(v, [&](auto cfg) {                                                                       \
        using Cfg = decltype(cfg);                                                                         \
        long acc = 0;                                                                                      \
        for (int i = 0; i < n; ++i) {                                                                      \
          offs[(size_t)v * (n + 1) + i] = acc;                                                             \
          acc += NAME##_tiles<P, Cfg>(a[i]);                                                               \
        }                                                                                                  \
        offs[(size_t)v * (n + 1) + n] = acc;                                                               \
        g.total[v] = acc;                                                                                  \
        g.grid[v] = (int)std::min(acc, 256L * wg_per_cu<P, Cfg>());                                        \
        return 0;                                                                                          \
      });                                                                                                  \
    }                                                                                                      \
    if (hipMalloc(&g.args_d, sizeof(ARGS) * n) != hipSuccess ||                                           \
        hipMalloc((void**)&g.off_d, sizeof(long) * offs.size()) != hipSuccess)                            \
      return fail(B->c, RIF_ENOMEM, "batch: device allocation failed");                                    \
    B->dev.push_back(g.args_d);                                                                            \
    B->dev.push_back(g.off_d);                                                                             \
    if (hipMemcpy(g.args_d, a.data(), sizeof(ARGS) * n, hipMemcpyHostToDevice) != hipSuccess ||           \
        hipMemcpy(g.off_d, offs.data(), sizeof(long) * offs.size(), hipMemcpyHostToDevice) != hipSuccess) \
      return fail(B->c, RIF_EHIP, "batch: upload failed");                                                 \
    return RIF_OK;                                                                                         \
  }                                                                                                        \
  template <int P>                                                                                         \
  static rif_status launch_##NAME(BatchImpl* B, int v) {                                                   \
    GroupStep& g = B->NAME;                                                                                \
    const int n = B->n;                                                                                    \
    return dispatch<P>(v, [&](auto cfg) {                                                                  \
      using Cfg = decltype(cfg);                                                                           \
      if constexpr (NVAR == 2 && Cfg::BM != Cfg::BN) {                                                     \
        return fail(B->c, RIF_ENOTSUP, LABEL ": non-square tile variant");                                 \
      } else {                                                                                             \
        if (g.total[v] == 0) return RIF_OK;                                                                \
        hipLaunchKernelGGL((k_##NAME##_g<P, Cfg>), dim3(g.grid[v]), dim3(Cfg::NT), 0, B->c->stream,        \
                           (const ARGS*)g.args_d, g.off_d + (size_t)v * (n + 1), n, g.total[v]);           \
        return check_launch(B->c, LABEL);                                                                  \
      }                                                                                                    \
    });                                                                                                    \
  }

// element-wise steps are not tile variants; dispatch<> is only used for the count
#define RIF_GROUP_FIXED(NAME, TILE, ARGS, LABEL, PP, CFG)                                                  \
  static rif_status setup_##NAME(BatchImpl* B, const std::vector<ARGS>& a) {                              \
    GroupStep& g = B->NAME;                                                                                \
    g.name = LABEL;                                                                                        \
    g.nvar = 1;                                                                                            \
    const int n = (int)a.size();                                                                           \
    std::vector<long> offs(n + 1, 0);                                                                      \
    for (int i = 0; i < n; ++i) offs[i + 1] = offs[i] + TILE##_tiles<PP, CFG>(a[i]);                      \
    g.total.assign(1, offs[n]);                                                                            \
    g.grid.assign(1, (int)std::min(offs[n], 256L * 8));                                                    \
    if (hipMalloc(&g.args_d, sizeof(ARGS) * n) != hipSuccess ||                                           \
        hipMalloc((void**)&g.off_d, sizeof(long) * (n + 1)) != hipSuccess)                                \
      return fail(B->c, RIF_ENOMEM, "batch: device allocation failed");                                    \
    B->dev.push_back(g.args_d);                                                                            \
    B->dev.push_back(g.off_d);                                                                             \
    if (hipMemcpy(g.args_d, a.data(), sizeof(ARGS) * n, hipMemcpyHostToDevice) != hipSuccess ||           \
        hipMemcpy(g.off_d, offs.data(), sizeof(long) * (n + 1), hipMemcpyHostToDevice) != hipSuccess)     \
      return fail(B->c, RIF_EHIP, "batch: upload failed");                                                 \
    return RIF_OK;                                                                                         \
  }                                                                                                        \
  static rif_status launch_##NAME(BatchImpl* B, int) {                                                     \
    GroupStep& g = B->NAME;                                                                                \
    if (g.total[0] == 0) return RIF_OK;                                                                    \
    hipLaunchKernelGGL((k_##TILE##_g<PP, CFG>), dim3(g.grid[0]), dim3(CFG::NT), 0, B->c->stream,           \
                       (const ARGS*)g.args_d, g.off_d, B->n, g.total[0]);                                  \
    return check_launch(B->c, LABEL);                                                                      \
  }

RIF_GROUP_SETUP(half, HalfArgs, "g_half_transform", 4)
RIF_GROUP_SETUP(halfp, HalfArgs, "g_half_transform_presplit", 4)
RIF_GROUP_SETUP(mo, MoArgs, "g_mo_transform", 4)
RIF_GROUP_SETUP(jao, JaoArgs, "g_jao", 4)
RIF_GROUP_SETUP(kao, KaoArgs, "g_kao", 2)
RIF_GROUP_SETUP(fock, FockArgs, "g_fock", 4)
#define RIF_GROUP_FIXED_P(NAME, ARGS, LABEL)                                                               \
  template <int P>                                                                                         \
  static rif_status setup_##NAME(BatchImpl* B, const std::vector<ARGS>& a) {                              \
    GroupStep& g = B->NAME;                                                                                \
    g.name = LABEL;                                                                                        \
    g.nvar = 1;                                                                                            \
    const int n = (int)a.size();                                                                           \
    std::vector<long> offs(n + 1, 0);                                                                      \
    for (int i = 0; i < n; ++i) offs[i + 1] = offs[i] + NAME##_tiles<P, Cfg256>(a[i]);                    \
    g.total.assign(1, offs[n]);                                                                            \
    g.grid.assign(1, (int)std::min(offs[n], 256L * 8));                                                    \
    if (hipMalloc(&g.args_d, sizeof(ARGS) * n) != hipSuccess ||                                           \
        hipMalloc((void**)&g.off_d, sizeof(long) * (n + 1)) != hipSuccess)                                \
      return fail(B->c, RIF_ENOMEM, "batch: device allocation failed");                                    \
    B->dev.push_back(g.args_d);                                                                            \
    B->dev.push_back(g.off_d);                                                                             \
    if (hipMemcpy(g.args_d, a.data(), sizeof(ARGS) * n, hipMemcpyHostToDevice) != hipSuccess ||           \
        hipMemcpy(g.off_d, offs.data(), sizeof(long) * (n + 1), hipMemcpyHostToDevice) != hipSuccess)     \
      return fail(B->c, RIF_EHIP, "batch: upload failed");                                                 \
    return RIF_OK;                                                                                         \
  }                                                                                                        \
  template <int P>                                                                                         \
  static rif_status launch_##NAME(BatchImpl* B, int) {                                                     \
    GroupStep& g = B->NAME;                                                                                \
    if (g.total[0] == 0) return RIF_OK;                                                                    \
    hipLaunchKernelGGL((k_##NAME##_g<P, Cfg256>), dim3(g.grid[0]), dim3(256), 0, B->c->stream,             \
                       (const ARGS*)g.args_d, g.off_d, B->n, g.total[0]);                                  \
    return check_launch(B->c, LABEL);                                                                      \
  }
// pre-split steps: same tile function (psplit) for C_Omega and d
#define RIF_GROUP_PSPLIT(NAME, LABEL)                                                                      \
  template <int P>                                                                                         \
  static rif_status setup_##NAME(BatchImpl* B, const std::vector<PSplitArgs>& a) {                        \
    GroupStep& g = B->NAME;                                                                                \
    g.name = LABEL;                                                                                        \
    g.nvar = 1;                                                                                            \
    const int n = (int)a.size();                                                                           \
    std::vector<long> offs(n + 1, 0);                                                                      \
    for (int i = 0; i < n; ++i) offs[i + 1] = offs[i] + psplit_tiles<P, Cfg256>(a[i]);                    \
    g.total.assign(1, offs[n]);                                                                            \
    g.grid.assign(1, (int)std::min(offs[n], 256L * 8));                                                    \
    if (hipMalloc(&g.args_d, sizeof(PSplitArgs) * n) != hipSuccess ||                                     \
        hipMalloc((void**)&g.off_d, sizeof(long) * (n + 1)) != hipSuccess)                                \
      return fail(B->c, RIF_ENOMEM, "batch: device allocation failed");                                    \
    B->dev.push_back(g.args_d);                                                                            \
    B->dev.push_back(g.off_d);                                                                             \
    if (hipMemcpy(g.args_d, a.data(), sizeof(PSplitArgs) * n, hipMemcpyHostToDevice) != hipSuccess ||     \
        hipMemcpy(g.off_d, offs.data(), sizeof(long) * (n + 1), hipMemcpyHostToDevice) != hipSuccess)     \
      return fail(B->c, RIF_EHIP, "batch: upload failed");                                                 \
    return RIF_OK;                                                                                         \
  }                                                                                                        \
  template <int P>                                                                                         \
  static rif_status launch_##NAME(BatchImpl* B, int) {                                                     \
    GroupStep& g = B->NAME;                                                                                \
    if constexpr (kPieces<P> == 0) {                                                                       \
      return RIF_OK;                                                                                       \
    } else {                                                                                               \
      if (g.total[0] == 0) return RIF_OK;                                                                  \
      hipLaunchKernelGGL((k_psplit_g<P, Cfg256>), dim3(g.grid[0]), dim3(256), 0, B->c->stream,             \
                         (const PSplitArgs*)g.args_d, g.off_d, B->n, g.total[0]);                          \
      return check_launch(B->c, LABEL);                                                                    \
    }                                                                                                      \
  }
RIF_GROUP_PSPLIT(psc, "g_presplit_C")
RIF_GROUP_PSPLIT(psd, "g_presplit_d")
RIF_GROUP_FIXED_P(jkp, JkArgs, "g_jk_mo_partial")
RIF_GROUP_FIXED_P(jkr, JkArgs, "g_jk_mo_reduce")
RIF_GROUP_FIXED(hc, gemm, GemmArgs, "g_hc_gemm", kF64, CfgSmall)
RIF_GROUP_FIXED(lam, gemm, GemmArgs, "g_lambda_gemm", kF64, CfgSmall)
RIF_GROUP_FIXED(coef, coef, CoefArgs, "g_coef", kF64, Cfg256)
RIF_GROUP_FIXED(energy, energy, EnergyArgs, "g_energy", kF64, CfgEnergy)
RIF_GROUP_FIXED(fred, fred, FockRedArgs, "g_fock_reduce", kF64, Cfg256)
RIF_GROUP_FIXED(grad, grad, GradArgs, "g_grad", kF64, Cfg256)

template <int P>
static rif_status batch_setup(BatchImpl* B, const std::vector<BuildArgs>& A) {
  std::vector<PSplitArgs> psc, psd;
  std::vector<HalfArgs> half; std::vector<MoArgs> mo; std::vector<JkArgs> jk; std::vector<JaoArgs> jao;
  std::vector<KaoArgs> kao; std::vector<GemmArgs> hc, lam; std::vector<CoefArgs> coef;
  std::vector<EnergyArgs> en; std::vector<FockArgs> fock; std::vector<FockRedArgs> fred; std::vector<GradArgs> grad;
  for (auto& x : A) {
    psc.push_back(x.psc); psd.push_back(x.psd);
    half.push_back(x.half); mo.push_back(x.mo); jk.push_back(x.jk); jao.push_back(x.jao); kao.push_back(x.kao);
    hc.push_back(x.hc); lam.push_back(x.lam); coef.push_back(x.coef); en.push_back(x.energy);
    fock.push_back(x.fock); fred.push_back(x.fred); grad.push_back(x.grad);
  }
  rif_status st;
  int npre = 0;
  for (auto& h : half) npre += b_presplit<P>(h) ? 1 : 0;
  if (npre != 0 && npre != (int)half.size())
    return fail(B->c, RIF_EINVAL, "batch: give b_split for every molecule or for none");
  B->bpre = npre > 0;
  if constexpr (P != kF64) {
    if (B->bpre && (st = setup_halfp<P>(B, half))) return st;
  }
  if ((st = setup_psc<P>(B, psc)) || (st = setup_psd<P>(B, psd)) ||
      (!B->bpre && (st = setup_half<P>(B, half))) || (st = setup_mo<P>(B, mo)) || (st = setup_jkp<P>(B, jk)) ||
      (st = setup_jkr<P>(B, jk)) || (st = setup_jao<P>(B, jao)) || (st = setup_kao<P>(B, kao)) ||
      (st = setup_hc(B, hc)) || (st = setup_coef(B, coef)) || (st = setup_energy(B, en)) ||
      (st = setup_fock<P>(B, fock)) || (st = setup_fred(B, fred)) || (st = setup_lam(B, lam)) ||
      (st = setup_grad(B, grad)))
    return st;
  // tile variants for the grouped GEMM steps: measured if autotuning, else the
  // variant with the fewest tile-area rounds
  auto choose = [&](GroupStep& g, const std::function<rif_status(int)>& run) {
    long key = 0;
    for (long t : g.total) key = key * 1000003 + t;
    int hv = 0;
    double best = 1e300;
    for (int v = 0; v < g.nvar; ++v) {
      const double e = (double)dispatch<P>(v, [&](auto cfg) {
        using Cfg = decltype(cfg);
        const long slots = (long)g.grid[v];
        return (double)((g.total[v] + slots - 1) / std::max(1L, slots)) * Cfg::BM * Cfg::BN * wg_per_cu<P, Cfg>();
      });
      if (e < best) { best = e; hv = v; }
    }
    g.variant = pick_variant(B->c, g.name.c_str(), {P, B->n, key}, g.nvar, hv, run);
    return g.variant < 0 ? RIF_EHIP : RIF_OK;
  };
  if constexpr (P != kF64) {
    if (B->bpre && (st = choose(B->halfp, [&](int v) { return launch_halfp<P>(B, v); }))) return st;
  }
  if (!B->bpre && (st = choose(B->half, [&](int v) { return launch_half<P>(B, v); }))) return st;
  if ((st = choose(B->mo, [&](int v) { return launch_mo<P>(B, v); }))) return st;
  if ((st = choose(B->jao, [&](int v) { return launch_jao<P>(B, v); }))) return st;
  if ((st = choose(B->kao, [&](int v) { return launch_kao<P>(B, v); }))) return st;
  if ((st = choose(B->fock, [&](int v) { return launch_fock<P>(B, v); }))) return st;
  return RIF_OK;
}

template <int P>
static rif_status batch_enqueue(BatchImpl* B) {
  rif_ctx* c = B->c;
  rif_status st;
#define RIF_G(STEP, ...)                                         \
  {                                                              \
    ProfScope ps(c, B->STEP.name.c_str());                       \
    if ((st = launch_##STEP __VA_ARGS__(B, B->STEP.variant))) return st; \
  }
  RIF_G(psc, <P>)
  if constexpr (P != kF64) {
    if (B->bpre) RIF_G(halfp, <P>)
  }
  if (!B->bpre) RIF_G(half, <P>)
  RIF_G(mo, <P>)
  RIF_G(jkp, <P>)
  RIF_G(jkr, <P>)
  if (kPlanesHalfJao<P>) RIF_G(psd, <P>)
  RIF_G(jao, <P>)
  RIF_G(kao, <P>)
  RIF_G(hc)
  RIF_G(coef)
  RIF_G(energy)
  RIF_G(fock, <P>)
  RIF_G(fred)
  RIF_G(lam)
  RIF_G(grad)
#undef RIF_G
  return RIF_OK;
}

rif_status op_batch_create(rif_ctx* c, int prec, int functional, int n, const rif_instance* inst, void** out) {
  if (!prec_ok(prec)) return fail(c, RIF_ENOTSUP, "precision mode not available");
  BatchImpl* B = new BatchImpl();
  B->c = c;
  B->prec = prec;
  B->n = n;
  // largest molecules first
  B->order.resize(n);
  for (int i = 0; i < n; ++i) B->order[i] = i;
  auto cost = [&](int i) { return (double)inst[i].n_aux * inst[i].n_bf * inst[i].n_bf * inst[i].n_pairs * (1 + inst[i].n_cwo); };
  std::stable_sort(B->order.begin(), B->order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<Plan> plans;
  std::vector<size_t> base;
  size_t total = 0;
  for (int k = 0; k < n; ++k) {
    const rif_instance& in = inst[B->order[k]];
    plans.emplace_back(in.n_bf, in.n_aux, in.n_pairs, in.n_cwo, in.n_mo);
    base.push_back(total);
    total += (plans.back().bytes + 255) & ~size_t(255);
  }
  if (hipMalloc(&B->ws, std::max(total, (size_t)256)) != hipSuccess) {
    (void)hipGetLastError();
    delete B;
    return fail(c, RIF_ENOMEM, "batch: workspace allocation failed");
  }
  std::vector<BuildArgs> A;
  for (int k = 0; k < n; ++k)
    A.push_back(make_build_args(plans[k], inst[B->order[k]], prec, functional, (char*)B->ws + base[k], c->dflag));
  rif_status st;
  auto setup = [&]() -> rif_status { RIF_PREC_SWITCH(prec, batch_setup<P>(B, A)) };
  if ((st = setup())) {
    op_batch_destroy(B);
    return st;
  }
  *out = B;
  return RIF_OK;
}

rif_status op_batch_run(void* handle, int use_graph) {
  BatchImpl* B = (BatchImpl*)handle;
  rif_ctx* c = B->c;
  auto enqueue = [&]() -> rif_status { RIF_PREC_SWITCH(B->prec, batch_enqueue<P>(B)) };
  if (!use_graph) return enqueue();
  if (!B->exec) {
    const bool prof = c->prof;
    c->prof = false;  // no event pairs inside the captured sequence
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      c->prof = prof;
      return fail(c, RIF_EHIP, "hipStreamBeginCapture failed");
    }
    rif_status st = enqueue();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->prof = prof;
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess || !g) return fail(c, RIF_EHIP, "hipStreamEndCapture failed");
    B->graph = g;
    if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      B->exec = nullptr;
      return fail(c, RIF_EHIP, "hipGraphInstantiate failed");
    }
  }
  ProfScope ps(c, "batch_graph");
  if (hipGraphLaunch(B->exec, c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipGraphLaunch failed");
  return RIF_OK;
}

void op_batch_destroy(void* handle) {
  BatchImpl* B = (BatchImpl*)handle;
  if (!B) return;
  (void)hipStreamSynchronize(B->c->stream);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (void* p : B->dev) (void)hipFree(p);
  if (B->ws) (void)hipFree(B->ws);
  delete B;
}

}  // namespace rif
