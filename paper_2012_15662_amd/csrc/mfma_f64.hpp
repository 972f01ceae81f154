// FP64 MFMA tile engine for gfx950 (v_mfma_f64_16x16x4_f64).
//
// A workgroup owns a BM x BN output tile and walks the reduction index in
// BK-deep slices.  Each slice of both operands is staged global -> registers
// -> LDS (double-buffered, one barrier per slice); waves are laid out
// (BM/WM) x (BN/WN) and each wave accumulates WM x WN with 16x16 MFMA blocks.
//
// LDS holds each operand slice k-major ([k][x], x contiguous), which is what
// the MFMA fragment layout reads: lane l takes row x = l%16, k = l/16.
// Operand loaders are small structs (see the *Loader templates) so that each
// kernel can describe its own memory layout while sharing this engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rif {

typedef double d4 __attribute__((ext_vector_type(4)));
// LDS pointer type: keeps ds_read/ds_write (a generic pointer would compile to
// flat accesses, whose waits also drain the in-flight global prefetch).
typedef __attribute__((address_space(3))) double lds_f64;

constexpr int kPadF64 = 16;   // 128 B row padding: the 4 k-rows of a fragment land in distinct banks

// x-contiguous operand: element (x, k) at base[k*ld + xoff(x)].
// Thread t owns column x = t % BX of the slice and rows k = t/BX + j*(NT/BX).
template <int BX, int BK, int NT>
struct XCLoader {
  static_assert(NT % BX == 0, "NT must be a multiple of BX");
  static constexpr int KSTEP = NT / BX;
  static_assert(BK % KSTEP == 0, "BK must be a multiple of NT/BX");
  static constexpr int R = BK / KSTEP;
  static constexpr int RR = R;  // registers staged per thread and slice
  const double* base;
  long ld;
  long xoff;
  int kmax;
  int kx, x;
  bool ok;
  // off(x, o) sets o = offset of column x and returns whether column x exists.
  template <class OffFn>
  __device__ void init(const double* base_, long ld_, int K, OffFn off) {
    base = base_; ld = ld_; kmax = K;
    x = threadIdx.x % BX; kx = threadIdx.x / BX;
    long o = 0;
    ok = off(x, o);
    xoff = ok ? o : 0;  // absent columns read a valid element and mask it
  }
  // kt = slice index; this slice covers k in [kt*BK, kt*BK + BK).
  __device__ void fetch(int kt, double (&r)[R]) const {
    const int k0 = kt * BK;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int k = k0 + kx + j * KSTEP;
      const int kc = k < kmax ? k : kmax - 1;
      r[j] = base[(long)kc * ld + xoff];
    }
  }
  // Masks out-of-range elements while writing to LDS (after the MFMAs of the
  // current slice), so the prefetch is not waited for any earlier.
  __device__ void stash(lds_f64* S, const double (&r)[R], int kt) const {
    const int k0 = kt * BK;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int k = k0 + kx + j * KSTEP;
      S[(kx + j * KSTEP) * (BX + kPadF64) + x] = (ok && k < kmax) ? r[j] : 0.0;
    }
  }
};

// k-contiguous operand: element (x, k) at row(x)[k].
// Threads take pairs of consecutive k; BK/2 threads cover one row slice.
template <int BX, int BK, int NT>
struct KCLoader {
  static constexpr int TPR = BK / 2;
  static constexpr int RSTEP = NT / TPR;
  static_assert(NT % TPR == 0 && BX % RSTEP == 0, "bad KC tiling");
  static constexpr int NP = BX / RSTEP;
  static constexpr int R = 2 * NP;
  static constexpr int RR = R;
  const double* rp[NP];
  unsigned valid;
  int kk, xr, kmax;
  // rowptr(x) returns the row base pointer or nullptr if row x is outside the
  // operand; `fallback` is any valid row, read in its place and masked.
  template <class RowPtr>
  __device__ void init(RowPtr rowptr, const double* fallback, int K) {
    kk = 2 * (threadIdx.x % TPR);
    xr = threadIdx.x / TPR;
    kmax = K;
    valid = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double* q = rowptr(xr + p * RSTEP);
      valid |= (q != nullptr) << p;
      rp[p] = q ? q : fallback;
    }
  }
  __device__ void fetch(int kt, double (&r)[R]) const {
    const int k0 = kt * BK;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int k = k0 + kk + v;
        const int kc = k < kmax ? k : kmax - 1;
        r[2 * p + v] = rp[p][kc];
      }
    }
  }
  __device__ void stash(lds_f64* S, const double (&r)[R], int kt) const {
    const int k0 = kt * BK;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int k = k0 + kk + v;
        S[(kk + v) * (BX + kPadF64) + xr + p * RSTEP] = ((valid >> p & 1) && k < kmax) ? r[2 * p + v] : 0.0;
      }
    }
  }
};

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = 64 * NWAVES;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int LDA = BM + kPadF64, LDB = BN + kPadF64;
  static constexpr int SMEM_DOUBLES = 2 * BK * (LDA + LDB);
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0 && BK % 4 == 0, "tile");
};

// Accumulator of one wave.
template <class Cfg>
struct Acc {
  d4 v[Cfg::TM][Cfg::TN];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j) v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }
  // Calls f(m_local, n_local, value) for every element this lane holds, with
  // m_local/n_local relative to the workgroup tile origin.  For the f64
  // 16x16x4 MFMA, register r of lane l holds row l/16 + 4r, column l%16 of
  // the 16x16 block (operands: lane l supplies A[l%16][l/16] and B[l/16][l%16]).
  template <class F>
  __device__ void for_each(F&& f) const {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave / Cfg::WAVES_N) * Cfg::WM, wn0 = (wave % Cfg::WAVES_N) * Cfg::WN;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          f(wm0 + i * 16 + (lane >> 4) + 4 * r, wn0 + j * 16 + (lane & 15), v[i][j][r]);
  }
};

// One BK-deep slice of MFMA work from LDS buffers As[BK][LDA], Bs[BK][LDB].
template <class Cfg>
__device__ __forceinline__ void mma_slice(const lds_f64* __restrict__ As, const lds_f64* __restrict__ Bs,
                                          Acc<Cfg>& acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / Cfg::WAVES_N) * Cfg::WM, wn0 = (wave % Cfg::WAVES_N) * Cfg::WN;
  const int kr = lane >> 4, xc = lane & 15;
#pragma unroll
  for (int kk = 0; kk < Cfg::BK; kk += 4) {
    double a[Cfg::TM], b[Cfg::TN];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i) a[i] = As[(kk + kr) * Cfg::LDA + wm0 + i * 16 + xc];
#pragma unroll
    for (int j = 0; j < Cfg::TN; ++j) b[j] = Bs[(kk + kr) * Cfg::LDB + wn0 + j * 16 + xc];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.v[i][j], 0, 0, 0);
  }
}

// Main loop: nk slices; la.fetch/lb.fetch take the slice index and handle
// their own k offsets.  smem must hold Cfg::SMEM_DOUBLES doubles.
template <class Cfg, class LA, class LB>
__device__ __forceinline__ void gemm_mainloop(LA& la, LB& lb, int nk, Acc<Cfg>& acc, double* smem) {
  lds_f64* L = (lds_f64*)smem;
  lds_f64* As[2] = {L, L + Cfg::BK * Cfg::LDA};
  lds_f64* Bs[2] = {L + 2 * Cfg::BK * Cfg::LDA, L + 2 * Cfg::BK * Cfg::LDA + Cfg::BK * Cfg::LDB};
  double ra[LA::RR], rb[LB::RR];
  acc.zero();
  if (nk <= 0) return;
  la.fetch(0, ra);
  lb.fetch(0, rb);
  la.stash(As[0], ra, 0);
  lb.stash(Bs[0], rb, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      la.fetch(kt + 1, ra);
      lb.fetch(kt + 1, rb);
    }
    mma_slice<Cfg>(As[cur], Bs[cur], acc);
    if (more) {
      la.stash(As[cur ^ 1], ra, kt + 1);
      lb.stash(Bs[cur ^ 1], rb, kt + 1);
    }
    __syncthreads();
  }
}

}  // namespace rif
