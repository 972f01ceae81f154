// MFMA tile engines for gfx950, one per arithmetic mode, behind one interface.
//
// A workgroup owns a BM x BN output tile and walks the reduction index in
// BK-deep slices.  Operand slices go global -> registers -> LDS (double
// buffered, one barrier per slice).  Waves are laid out (BM/WM) x (BN/WN); each
// accumulates WM x WN with 16x16 MFMA blocks.  Kernels describe their operand
// layouts with source loaders (XCSrc / KCSrc or their own) and read results
// through Acc::for_each, which always yields FP64 values.
//
// Modes
//   kF64    v_mfma_f64_16x16x4_f64, FP64 operands and accumulation.
//   kF32    v_mfma_f32_16x16x4_f32 on operands rounded to FP32; FP32 partial
//           sums are folded into FP64 accumulators every 128 k.
//   kBF16x3 v_mfma_f32_16x16x32_bf16 on pieces split from each FP64 (or FP32)
//           operand x = hi + lo (+ lo2) with hi = bf16(x), lo = bf16(x - hi),
//           lo2 = bf16(x - hi - lo).  x3: hi.hi + (hi.lo + lo.hi);
//   kBF16x6 x6 adds hi.lo2 + lo.lo + lo2.hi.  The hi.hi products and the cross
//           products accumulate in separate FP32 registers, folded into FP64
//           every 128 k.
//   kF16x3  v_mfma_f32_16x16x32_f16 on x = hi + lo 2^-11 with hi = fp16(x),
//           lo = fp16((x - hi) 2^11): hi.hi + 2^-11 (hi.lo + lo.hi), the cross
//           products accumulated apart and scaled by 2^-11 when folded.  The
//           low piece is stored scaled so it keeps fp16's 11 bits wherever hi
//           is normal; |x| must stay below fp16's largest value (65504), or
//           the results are not finite.
//
// LDS layouts: FP64/FP32 slices are k-major ([k][x], x contiguous), which is
// what the 16x16x4 fragments read (lane l takes x = l%16, k = l/16).  BF16
// pieces are x-major with k contiguous ([x][k], 16-byte chunks swizzled per
// row), since a 16x16x32 fragment is 8 consecutive k of one row per lane
// (x = l%16, k = 8*(l/16) .. +7).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rif {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
// LDS pointer types: keep ds_read/ds_write (generic pointers would compile to
// flat accesses, whose waits also drain the in-flight global prefetch).
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) u16x8 lds_u16x8;
typedef __attribute__((address_space(3))) u32x2 lds_u32x2;
typedef __attribute__((address_space(3))) char lds_char;

enum Prec : int { kF64 = 0, kF32 = 1, kBF16x3 = 2, kBF16x6 = 3, kF16x3 = 4 };

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = 64 * NWAVES;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "tile");
};

// ---------------------------------------------------------------------------
// Source loaders.  A thread holds RR registers per slice: NP groups of KV
// consecutive k of one column x.  xl(p) / kl(p) give the local coordinates of
// group p, valid(p, i, kt) whether element i of group p exists, val() the
// value to stage.  Loads clamp their address into the operand so they never
// branch; out-of-range elements are zeroed at staging time (after the MFMAs
// of the current slice), which keeps the prefetch in flight.

// x-contiguous operand: element (x, k) at base[k*ld + off(x)].
template <class T, int BX, int BK, int NT, int KV>
struct XCSrc {
  static constexpr int TPX = NT / BX;   // threads per column
  static constexpr int NG = BK / KV;    // k-groups per column
  static_assert(NT % BX == 0 && NG % TPX == 0, "bad XC tiling");
  static constexpr int NP = NG / TPX;
  static constexpr int R = NP * KV, RR = R;
  using type = T;
  const T* base;
  long ld, xoff;
  int kmax, x, kg;
  bool ok;
  // off(x, o) sets o = offset of column x and returns whether column x exists.
  template <class OffFn>
  __device__ void init(const T* base_, long ld_, int K, OffFn off) {
    base = base_; ld = ld_; kmax = K;
    x = threadIdx.x % BX; kg = threadIdx.x / BX;
    long o = 0;
    ok = off(x, o);
    xoff = ok ? o : 0;
  }
  __device__ int xl(int) const { return x; }
  __device__ int kl(int p) const { return (kg + p * TPX) * KV; }
  __device__ bool valid(int p, int i, int kt) const { return ok && kt * BK + kl(p) + i < kmax; }
  __device__ void fetch(int kt, T (&r)[RR]) const {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        const int k = kt * BK + kl(p) + i;
        r[p * KV + i] = base[(long)(k < kmax ? k : kmax - 1) * ld + xoff];
      }
  }
  __device__ double val(const T (&r)[RR], int p, int i) const { return (double)r[p * KV + i]; }
};

// k-contiguous operand: element (x, k) at row(x)[k].
//   KV == 1 (k-major LDS): lanes run along x sixteen at a time, so one wave's
//     LDS writes cover 16 consecutive x of 4 k rows (no bank conflicts) while
//     its global loads read 4 consecutive k of 16 rows.  Thread t holds one k
//     (kq) of NP rows x = xl0 + 16*(xh0 + p*XSTEP16).
//   KV > 1 (x-major LDS): a thread holds KV consecutive k of NP rows.
template <class T, int BX, int BK, int NT, int KV>
struct KCSrc {
  static constexpr bool XFAST = (KV == 1);
  static constexpr int TPR = BK / KV;                         // k-groups per row
  static constexpr int RSTEP = XFAST ? 16 * (NT / (16 * BK)) : NT / TPR;   // rows per pass
  static_assert(XFAST ? (NT % (16 * BK) == 0 && BX % 16 == 0) : (NT % TPR == 0), "bad KC tiling");
  static_assert(BX % RSTEP == 0, "bad KC tiling");
  static constexpr int NP = BX / RSTEP;
  static constexpr int R = NP * KV, RR = R;
  using type = T;
  const T* rp[NP];
  unsigned vmask;
  int kg, xr, kmax;
  // rowptr(x) returns row x's base or nullptr if absent; `fallback` is any
  // valid row, read in its place and masked.
  template <class RowPtr>
  __device__ void init(RowPtr rowptr, const T* fallback, int K) {
    if constexpr (XFAST) {
      kg = (threadIdx.x / 16) % BK;
      xr = threadIdx.x % 16 + 16 * (threadIdx.x / (16 * BK));
    } else {
      kg = threadIdx.x % TPR;
      xr = threadIdx.x / TPR;
    }
    kmax = K;
    vmask = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const T* q = rowptr(xr + p * RSTEP);
      vmask |= (unsigned)(q != nullptr) << p;
      rp[p] = q ? q : fallback;
    }
  }
  __device__ int xl(int p) const { return xr + p * RSTEP; }
  __device__ int kl(int) const { return kg * KV; }
  __device__ bool valid(int p, int i, int kt) const { return (vmask >> p & 1) && kt * BK + kg * KV + i < kmax; }
  __device__ void fetch(int kt, T (&r)[RR]) const {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        const int k = kt * BK + kg * KV + i;
        r[p * KV + i] = rp[p][k < kmax ? k : kmax - 1];
      }
  }
  __device__ double val(const T (&r)[RR], int p, int i) const { return (double)r[p * KV + i]; }
};

__device__ __forceinline__ void wave_origin(int WAVES_N, int WM, int WN, int& wm0, int& wn0) {
  const int wave = threadIdx.x >> 6;
  wm0 = (wave / WAVES_N) * WM;
  wn0 = (wave % WAVES_N) * WN;
}

// Wave plan: which TM x TN block of 16x16 fragments a wave computes (origin
// wm0, wn0 inside the tile) and how many of its fragment rows (ni <= TM, a
// prefix) hold needed outputs.  The regular plan is the fixed layout with all
// rows.  For tiles where some fragments are not needed (blocks on the diagonal
// of a symmetric result, ragged edges), make_wave_plan() trims each region to
// its live rows and hands the regions out so that each SIMD gets a heavy
// region with a light one: regions are ranked by work and wave w takes rank
// kRankOfWave[w], which pairs ranks (0,6) (7,1) (2,4) (5,3) for waves
// {w, w+4} and (0,7) (2,5) (6,1) (4,3) for waves {2k, 2k+1}, whichever way
// the waves of a workgroup are spread over the SIMDs.
struct WavePlan {
  int wm0, wn0, ni;
};
template <class Cfg>
__device__ __forceinline__ WavePlan regular_plan() {
  WavePlan w;
  wave_origin(Cfg::WAVES_N, Cfg::WM, Cfg::WN, w.wm0, w.wn0);
  w.ni = Cfg::TM;
  return w;
}
// live(I, J): whether tile-local fragment (I, J) is needed.
template <class Cfg, class Live>
__device__ __forceinline__ WavePlan make_wave_plan(Live live) {
  constexpr int NW = Cfg::NWAVES;
  int rows[NW];
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const int m0 = (r / Cfg::WAVES_N) * Cfg::TM, n0 = (r % Cfg::WAVES_N) * Cfg::TN;
    int n = 0;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        if (live(m0 + i, n0 + j)) n = i + 1;
    rows[r] = n;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int rank = wave;
  if constexpr (NW == 8) {
    constexpr int kRankOfWave[8] = {0, 7, 2, 5, 6, 1, 4, 3};
    rank = kRankOfWave[wave];
  }
  // region of the given rank: most rows first, ties by region index
  WavePlan w{0, 0, 0};
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    int above = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) above += rows[q] > rows[r] || (rows[q] == rows[r] && q < r);
    if (above == rank) {
      w.wm0 = (r / Cfg::WAVES_N) * Cfg::WM;
      w.wn0 = (r % Cfg::WAVES_N) * Cfg::WN;
      w.ni = rows[r];
    }
  }
  return w;
}
// Calls f(std::integral_constant<int, n>) for n = ni in 0..TM, so each row
// count gets its own straight-line code (callers put this outside their slice
// loop, which keeps one variant's registers live at a time).
template <int TM, class F>
__device__ __forceinline__ void with_rows(int ni, F&& f) {
  if (ni >= TM) {
    f(std::integral_constant<int, TM>());
  } else if constexpr (TM > 0) {
    with_rows<TM - 1>(ni, f);
  }
}

// ---------------------------------------------------------------------------
// FP64 engine (BK_ = slice depth)
// PAD_: doubles of padding per LDS row (0 only for direct-staged 64-column
// operands, whose fragment reads touch one row per 16 lanes).
template <int BK_ = 16, int PAD_ = 16>
struct EngF64T {
  static constexpr int BK = BK_, KV = 1, PAD = PAD_, CHUNK = 1 << 30;
  template <int BX>
  static constexpr int stage_bytes() { return BK * (BX + PAD) * 8; }
  template <class Cfg>
  struct Acc {
    d4 v[Cfg::TM][Cfg::TN];
    __device__ void zero() {
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
    __device__ void flush() {}
    // f64 16x16x4: register r of lane l holds row l/16 + 4r, column l%16.
    template <class F>
    __device__ void for_each(F&& f) const { for_each(regular_plan<Cfg>(), f); }
    template <class F>
    __device__ void for_each(const WavePlan& w, F&& f) const {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j)
          if (i < w.ni) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              f(w.wm0 + i * 16 + (lane >> 4) + 4 * r, w.wn0 + j * 16 + (lane & 15), v[i][j][r]);
          }
    }
  };
  template <int BX, class L>
  __device__ static void stash(lds_char* S, const L& ld, const typename L::type (&r)[L::RR], int kt) {
    lds_f64* s = (lds_f64*)S;
#pragma unroll
    for (int p = 0; p < L::NP; ++p)
      s[ld.kl(p) * (BX + PAD) + ld.xl(p)] = ld.valid(p, 0, kt) ? ld.val(r, p, 0) : 0.0;
  }
  // Rows 0..NI-1 of the wave's fragment block (NI = TM for the regular layout).
  template <class Cfg, int NI>
  __device__ static void mma_rows(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    const lds_f64* As = (const lds_f64*)SA;
    const lds_f64* Bs = (const lds_f64*)SB;
    const int lane = threadIdx.x & 63;
    const int kr = lane >> 4, xc = lane & 15;
    if constexpr (NI > 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[NI], b[Cfg::TN];
#pragma unroll
        for (int i = 0; i < NI; ++i) a[i] = As[(kk + kr) * (Cfg::BM + PAD) + w.wm0 + i * 16 + xc];
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) b[j] = Bs[(kk + kr) * (Cfg::BN + PAD) + w.wn0 + j * 16 + xc];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::TN; ++j)
            acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.v[i][j], 0, 0, 0);
      }
    }
  }
  template <class Cfg>
  __device__ static void mma(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    mma_rows<Cfg, Cfg::TM>(SA, SB, acc, w);
  }
};

// ---------------------------------------------------------------------------
// FP32 engine (FP64 recombination every CHUNK slices = 128 k)
struct EngF32 {
  static constexpr int BK = 16, KV = 1, PAD = 16, CHUNK = 8;
  template <int BX>
  static constexpr int stage_bytes() { return BK * (BX + PAD) * 4; }
  template <class Cfg>
  struct Acc {
    f4 s[Cfg::TM][Cfg::TN];
    d4 v[Cfg::TM][Cfg::TN];
    __device__ void zero() {
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
          s[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }
    }
    __device__ void flush() {
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[i][j][r] += (double)s[i][j][r];
          s[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // f32 MFMA layout: register r of lane l holds row 4*(l/16) + r, column l%16.
    template <class F>
    __device__ void for_each(F&& f) const { for_each(regular_plan<Cfg>(), f); }
    template <class F>
    __device__ void for_each(const WavePlan& w, F&& f) const {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j)
          if (i < w.ni) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              f(w.wm0 + i * 16 + 4 * (lane >> 4) + r, w.wn0 + j * 16 + (lane & 15), v[i][j][r]);
          }
    }
  };
  template <int BX, class L>
  __device__ static void stash(lds_char* S, const L& ld, const typename L::type (&r)[L::RR], int kt) {
    lds_f32* s = (lds_f32*)S;
#pragma unroll
    for (int p = 0; p < L::NP; ++p)
      s[ld.kl(p) * (BX + PAD) + ld.xl(p)] = ld.valid(p, 0, kt) ? (float)ld.val(r, p, 0) : 0.f;
  }
  // Rows 0..NI-1 of the wave's fragment block (NI = TM for the regular layout).
  template <class Cfg, int NI>
  __device__ static void mma_rows(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    const lds_f32* As = (const lds_f32*)SA;
    const lds_f32* Bs = (const lds_f32*)SB;
    const int lane = threadIdx.x & 63;
    const int kr = lane >> 4, xc = lane & 15;
    if constexpr (NI > 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[NI], b[Cfg::TN];
#pragma unroll
        for (int i = 0; i < NI; ++i) a[i] = As[(kk + kr) * (Cfg::BM + PAD) + w.wm0 + i * 16 + xc];
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) b[j] = Bs[(kk + kr) * (Cfg::BN + PAD) + w.wn0 + j * 16 + xc];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::TN; ++j)
            acc.s[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc.s[i][j], 0, 0, 0);
      }
    }
  }
  template <class Cfg>
  __device__ static void mma(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    mma_rows<Cfg, Cfg::TM>(SA, SB, acc, w);
  }
};

// ---------------------------------------------------------------------------
// Split-BF16 engines.  NPC = pieces per operand (2 for x3, 3 for x6).
// Split of two operand values into NPC bf16 pieces each, packed two to a
// 32-bit word per piece (element 0 in the low half).  Shared by the staging
// path and the pre-split kernel.  Pieces come from the packed round-to-
// nearest-even conversion of FP32 values: hi = bf16(f) with f = fp32(x), then
// the first residual x - hi = (x - f) + (f - hi) (both parts exact) rounded
// once to FP32 (about 2^-33 relative to x), whose further residuals are exact
// in FP32.  x6 (three pieces): hi + lo + lo2 holds x to about 2^-32; x3 (two):
// hi + lo to 2^-17.  FP32 operands are their own FP32 value, so every residual
// is exact in FP32.
template <int NPC>
__device__ __forceinline__ void split_tail(float x0, float x1, unsigned (&pc)[NPC]) {
#pragma unroll
  for (int s = 1; s < NPC; ++s) {
    const bf16x2 g = {(__bf16)x0, (__bf16)x1};
    pc[s] = __builtin_bit_cast(unsigned, g);
    if (s + 1 < NPC) {
      x0 -= (float)g[0];
      x1 -= (float)g[1];
    }
  }
}
template <int NPC>
__device__ __forceinline__ void split_pair(double d0, double d1, unsigned (&pc)[NPC]) {
  float f0 = (float)d0, f1 = (float)d1;
  // keep the FP32 rounding visible: otherwise the two conversions fold into
  // one emulated FP64 -> bf16 rounding (no instruction is emitted here)
  asm("" : "+v"(f0), "+v"(f1));
  const bf16x2 h = {(__bf16)f0, (__bf16)f1};
  pc[0] = __builtin_bit_cast(unsigned, h);
  split_tail<NPC>((float)(d0 - (double)f0) + (f0 - (float)h[0]), (float)(d1 - (double)f1) + (f1 - (float)h[1]),
                  pc);
}
template <int NPC>
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned (&pc)[NPC]) {
  const bf16x2 h = {(__bf16)x0, (__bf16)x1};
  pc[0] = __builtin_bit_cast(unsigned, h);
  split_tail<NPC>(x0 - (float)h[0], x1 - (float)h[1], pc);
}

// FP16x3 split: hi = fp16(f) with f = fp32(x) (round to nearest even), then the
// residual (x - f) + (f - hi), exact in its two parts, times 2^11 rounded once
// to fp16.  hi + lo 2^-11 holds x to about 2^-22 relative while hi is normal.
constexpr float kF16LoScale = 2048.f;
__device__ __forceinline__ void split_pair_f16(double d0, double d1, unsigned (&pc)[2]) {
  float f0 = (float)d0, f1 = (float)d1;
  asm("" : "+v"(f0), "+v"(f1));
  const f16x2 h = {(_Float16)f0, (_Float16)f1};
  pc[0] = __builtin_bit_cast(unsigned, h);
  const float r0 = ((float)(d0 - (double)f0) + (f0 - (float)h[0])) * kF16LoScale;
  const float r1 = ((float)(d1 - (double)f1) + (f1 - (float)h[1])) * kF16LoScale;
  const f16x2 g = {(_Float16)r0, (_Float16)r1};
  pc[1] = __builtin_bit_cast(unsigned, g);
}
__device__ __forceinline__ void split_pair_f16(float x0, float x1, unsigned (&pc)[2]) {
  const f16x2 h = {(_Float16)x0, (_Float16)x1};
  pc[0] = __builtin_bit_cast(unsigned, h);
  const f16x2 g = {(_Float16)((x0 - (float)h[0]) * kF16LoScale), (_Float16)((x1 - (float)h[1]) * kF16LoScale)};
  pc[1] = __builtin_bit_cast(unsigned, g);
}
__device__ __forceinline__ f4 mfma_piece(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_piece(f16x8 a, f16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Operand already split into NPC bf16 piece planes (split_pair arithmetic):
// element (x, k) of piece s at planes[s * pstride + row(x) * ld + k], k
// contiguous, every row zero-filled from its length up to ld (a multiple of
// 32), so no k is ever out of range.  A thread loads KV = 4 consecutive k of
// one row per piece (8 bytes); rows beyond the operand read row 0 and are
// zeroed when staged.
template <int NPC_, int BX, int BK, int NT>
struct PieceSrc {
  static constexpr int NPC = NPC_, KV = 4, TPR = BK / KV, RSTEP = NT / TPR;
  static_assert(NT % TPR == 0 && BX % RSTEP == 0, "bad piece tiling");
  static constexpr int NP = BX / RSTEP;
  static constexpr int RR = NP * NPC;
  static constexpr bool kPresplit = true;
  using type = u32x2;
  const unsigned short* rp[NP];
  long pstride;
  unsigned vmask;
  int kg, xr;
  // row(x, o) sets o = the plane row of operand column x and returns whether it exists
  template <class Row>
  __device__ void init(const unsigned short* planes, long pstride_, long ld, Row row) {
    kg = threadIdx.x % TPR;
    xr = threadIdx.x / TPR;
    pstride = pstride_;
    vmask = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      long o = 0;
      const bool ok = row(xr + p * RSTEP, o);
      vmask |= (unsigned)ok << p;
      rp[p] = planes + (ok ? o : 0) * ld + kg * KV;
    }
  }
  __device__ int xl(int p) const { return xr + p * RSTEP; }
  __device__ int kl(int) const { return kg * KV; }
  __device__ bool row_ok(int p) const { return vmask >> p & 1; }
  __device__ void fetch(int kt, u32x2 (&r)[RR]) const {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int s = 0; s < NPC; ++s) r[p * NPC + s] = *(const u32x2*)(rp[p] + s * pstride + kt * BK);
  }
};
// Operand already split into NPC piece planes (layout as for PieceSrc),
// staged by direct global -> LDS loads (global_load_lds_dwordx4): a lane moves
// one 16-byte chunk (8 k of one row of one plane) to LDS at its wave's base
// address + 16 * lane, so staging takes no registers.  The units of a stage
// (NPC * BX rows * 4 chunks) are numbered in LDS order; thread u moves units
// u, u + NT, ..., and unit (plane s, row x, slot c') holds chunk
// c' ^ ((x / 2) % 4) of the row (the split engines' swizzle).  Rows beyond the
// operand read row 0 instead; their products reach only output rows or
// columns that are never stored, so they need no zeroing.
template <int NPC_, int BX, int NT>
struct PieceDma {
  static constexpr int NPC = NPC_;
  static constexpr int UNITS = NPC * BX * 4;
  static constexpr int NU = (UNITS + NT - 1) / NT;
  static_assert(UNITS % 64 == 0 && NT % 64 == 0, "whole waves");
  const unsigned short* src[NU];
  // row(x, o) sets o = the plane row of operand column x and returns whether it exists
  template <class Row>
  __device__ void init(const unsigned short* planes, long pstride, long ld, Row row) {
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      const int u = (int)threadIdx.x + i * NT;
      const int uc = u < UNITS ? u : UNITS - 1;
      const int sp = uc / (BX * 4), v = uc % (BX * 4), x = v / 4, c = (v % 4) ^ ((x >> 1) & 3);
      long o = 0;
      const bool ok = row(x, o);
      src[i] = planes + sp * pstride + (ok ? o : 0) * ld + c * 8;
    }
  }
  // loads this wave issues per slice (the same in every slice)
  __device__ int count() const {
    const int w0 = (int)(threadIdx.x & ~63u);
    int n = 0;
#pragma unroll
    for (int i = 0; i < NU; ++i) n += w0 + i * NT < UNITS;
    return n;
  }
  // slice kt (32 k) into the stage at S
  __device__ void issue(int kt, lds_char* S) const {
    const int w0 = (int)(threadIdx.x & ~63u);
#pragma unroll
    for (int i = 0; i < NU; ++i)
      if (w0 + i * NT < UNITS)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[i] + kt * 32),
                                         (__attribute__((address_space(3))) void*)(S + (w0 + i * NT) * 16), 16, 0, 0);
  }
};

// Zeros read by the direct-staging loader below for k rows past the end.
static __device__ __attribute__((aligned(16))) double kDmaZeros[128];

// FP64 x-contiguous operand staged by direct global -> LDS loads (16 bytes,
// two doubles of one k-row per lane).  With 128 columns one wave's load fills
// one k-row of the stage; with 64 columns each half-wave fills one row (the
// load's LDS address is the wave's base plus 16 bytes per lane index): one
// wave load for the row pair when the rows are unpadded (and so adjacent),
// else two half-wave loads.  count() is the number of loads a wave issues
// per slice, which the main loop's waits rely on.
// The rows' padding stays untouched.  Rows at or past K read zeros; a column
// pair that does not exist reads column 0 (its outputs are never stored).
// Needs 16-byte aligned rows and even column offsets.
template <int NT, int BK, int PAD, int BX = 128>
struct XcDma64 {
  static_assert(BX == 128 || BX == 64, "one row per wave or half-wave");
  static constexpr int NW = NT / 64, RPI = 128 / BX;   // k-rows per wave instruction pair
  static constexpr int UPW = BK / (NW * RPI);          // row groups per wave per slice
  static_assert(BK % (NW * RPI) == 0, "k rows per wave");
  static constexpr int STRIDE = (BX + PAD) * 8;        // bytes per LDS row
  const double* col;   // this lane's column pair in k row 0
  long ld;
  int K;
  template <class OffFn>
  __device__ void init(const double* base, long ld_, int K_, OffFn off) {
    ld = ld_;
    K = K_;
    long o = 0;
    const bool ok = off(2 * (int)(threadIdx.x & (BX / 2 - 1)), o);
    col = base + (ok ? o : 0);
  }
  // unpadded 64-column rows: the two rows of a pair are one contiguous 1 KB
  // destination, filled by one wave load
  static constexpr bool kPair = BX == 64 && STRIDE == 512;
  __device__ int count() const { return kPair ? UPW : UPW * RPI; }
  __device__ void issue(int kt, lds_char* S) const {
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
      const int g = w + j * NW;   // row group
      if constexpr (kPair) {
        const int k = kt * BK + 2 * g + (lane >> 5);
        const double* src = k < K ? col + (long)k * ld : kDmaZeros + 2 * (lane & 31);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(S + 2 * g * STRIDE), 16, 0, 0);
      } else if constexpr (BX == 128) {
        const int k = kt * BK + g;
        const double* src = k < K ? col + (long)k * ld : kDmaZeros + 2 * lane;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(S + g * STRIDE), 16, 0, 0);
      } else {
        // rows 2g (lanes 0-31) and 2g+1 (lanes 32-63) from one wave-uniform
        // LDS base; the upper half's shift to its row goes into the immediate
        // offset (applied to both addresses, so its global address is set back
        // by as much), which also keeps the two loads from being merged into
        // one with a lane-varying base
        constexpr int kUp = STRIDE - 512;
        const int h = lane >> 5, kl = 2 * g + h, k = kt * BK + kl;
        const double* src = k < K ? col + (long)k * ld : kDmaZeros + 2 * (lane & 31);
        lds_char* dst = S + 2 * g * STRIDE;
        if (h == 0)
          __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                           (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        else
          __builtin_amdgcn_global_load_lds(
              (const __attribute__((address_space(1))) void*)((const char*)src - kUp),
              (__attribute__((address_space(3))) void*)dst, 16, kUp, 0);
      }
    }
  }
};

template <class L, class = void>
struct is_presplit : std::false_type {};
template <class L>
struct is_presplit<L, std::void_t<decltype(L::kPresplit)>> : std::true_type {};

// Split engines: NPC pieces per operand, bf16 pieces (kHalf = false) or the
// fp16 pair with its scaled low piece (kHalf = true, NPC = 2 only).
template <int NPC, bool kHalf = false>
struct EngSplit {
  static_assert(!kHalf || NPC == 2, "fp16 split has two pieces");
  static constexpr int BK = 32, KV = 4, CHUNK = 4;
  using PV = typename std::conditional<kHalf, f16x8, bf16x8>::type;
  // weight of the cross-product accumulator when folded into FP64
  static constexpr double kCross = kHalf ? 1.0 / kF16LoScale : 1.0;
  // One piece plane of BX rows of 64 B (32 k); a stage holds NPC planes.  The
  // four 16-byte chunks (8 k each) of row x sit at chunk c ^ ((x / 2) % 4).  A
  // fragment read (ds_read_b128: sixteen rows at one chunk) is served eight
  // lanes at a time; with this swizzle every eight consecutive rows at one
  // chunk fill all eight 16-byte bank groups.  Measured with an LDS probe:
  // 200 B/clk per CU against 112 with c ^ ((x / 4) % 4), which put rows x and
  // x + 2 on the same banks (four conflict cycles per read).
  template <int BX>
  static constexpr int piece_bytes() { return BX * BK * 2; }
  __device__ static int chunk_off(int x, int c) { return x * (BK * 2) + ((c ^ ((x >> 1) & 3)) << 4); }
  template <int BX>
  static constexpr int stage_bytes() { return NPC * piece_bytes<BX>(); }
  template <class Cfg>
  struct Acc {
    f4 hh[Cfg::TM][Cfg::TN];
    f4 xx[Cfg::TM][Cfg::TN];
    d4 v[Cfg::TM][Cfg::TN];
    __device__ void zero() {
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
          hh[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          xx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }
    }
    __device__ void flush() {
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[i][j][r] += (double)hh[i][j][r] + kCross * (double)xx[i][j][r];
          hh[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          xx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    template <class F>
    __device__ void for_each(F&& f) const { for_each(regular_plan<Cfg>(), f); }
    template <class F>
    __device__ void for_each(const WavePlan& w, F&& f) const {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j)
          if (i < w.ni) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              f(w.wm0 + i * 16 + 4 * (lane >> 4) + r, w.wn0 + j * 16 + (lane & 15), v[i][j][r]);
          }
    }
  };
  // Writes each group of KV = 4 consecutive k as NPC bf16 pieces, one 8-byte
  // vector per piece: split here (split_pair) or loaded already split.
  template <int BX, class L>
  __device__ static void stash(lds_char* S, const L& ld, const typename L::type (&r)[L::RR], int kt) {
    if constexpr (is_presplit<L>::value) {
      // planes made by the same mode's split (the kernels pair them by mode)
      static_assert(L::NPC == NPC && L::KV == KV, "piece planes of another split");
#pragma unroll
      for (int p = 0; p < L::NP; ++p) {
        const int k = ld.kl(p);
        const int off = chunk_off(ld.xl(p), k / 8) + (k % 8) * 2;
        const bool ok = ld.row_ok(p);
#pragma unroll
        for (int s = 0; s < NPC; ++s) {
          const u32x2 v = ok ? r[p * NPC + s] : u32x2{0u, 0u};
          *(lds_u32x2*)(S + s * piece_bytes<BX>() + off) = v;
        }
      }
    } else {
      static_assert(L::NP * KV <= L::RR, "groups of KV");
#pragma unroll
      for (int p = 0; p < L::NP; ++p) {
        unsigned pc[KV / 2][NPC];
#pragma unroll
        for (int i = 0; i < KV; i += 2) {
          if constexpr (std::is_same<typename L::type, float>::value) {
            const float x0 = ld.valid(p, i, kt) ? (float)ld.val(r, p, i) : 0.f;
            const float x1 = ld.valid(p, i + 1, kt) ? (float)ld.val(r, p, i + 1) : 0.f;
            if constexpr (kHalf) split_pair_f16(x0, x1, pc[i / 2]);
            else split_pair<NPC>(x0, x1, pc[i / 2]);
          } else {
            const double x0 = ld.valid(p, i, kt) ? ld.val(r, p, i) : 0.0;
            const double x1 = ld.valid(p, i + 1, kt) ? ld.val(r, p, i + 1) : 0.0;
            if constexpr (kHalf) split_pair_f16(x0, x1, pc[i / 2]);
            else split_pair<NPC>(x0, x1, pc[i / 2]);
          }
        }
        const int k = ld.kl(p);
        const int off = chunk_off(ld.xl(p), k / 8) + (k % 8) * 2;
#pragma unroll
        for (int s = 0; s < NPC; ++s) {
          const u32x2 v = {pc[0][s], pc[1][s]};
          *(lds_u32x2*)(S + s * piece_bytes<BX>() + off) = v;
        }
      }
    }
  }
  // Rows 0..NI-1 of the wave's fragment block (NI = TM for the regular layout).
  // The B pieces of the wave's TN columns stay in registers; the A pieces are
  // loaded one fragment row at a time (keeps the 16-wave tiles within 128 VGPRs).
  template <class Cfg, int NI>
  __device__ static void mma_rows(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    const int lane = threadIdx.x & 63;
    const int xc = lane & 15, kc = lane >> 4;
    if constexpr (NI > 0) {
      PV b[NPC][Cfg::TN];
#pragma unroll
      for (int s = 0; s < NPC; ++s)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j)
          b[s][j] = __builtin_bit_cast(PV, *(const lds_u16x8*)(SB + s * piece_bytes<Cfg::BN>() +
                                                                chunk_off(w.wn0 + j * 16 + xc, kc)));
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        PV a[NPC];
#pragma unroll
        for (int s = 0; s < NPC; ++s)
          a[s] = __builtin_bit_cast(PV, *(const lds_u16x8*)(SA + s * piece_bytes<Cfg::BM>() +
                                                             chunk_off(w.wm0 + i * 16 + xc, kc)));
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
          f4 x = acc.xx[i][j];
          if constexpr (NPC == 3) {
            x = mfma_piece(a[0], b[2][j], x);
            x = mfma_piece(a[1], b[1][j], x);
            x = mfma_piece(a[2], b[0][j], x);
          }
          x = mfma_piece(a[0], b[1][j], x);
          x = mfma_piece(a[1], b[0][j], x);
          acc.xx[i][j] = x;
          acc.hh[i][j] = mfma_piece(a[0], b[0][j], acc.hh[i][j]);
        }
      }
    }
  }
  template <class Cfg>
  __device__ static void mma(const lds_char* SA, const lds_char* SB, Acc<Cfg>& acc, const WavePlan& w) {
    mma_rows<Cfg, Cfg::TM>(SA, SB, acc, w);
  }
};

template <class E, class Cfg>
constexpr int smem_bytes() { return 2 * (E::template stage_bytes<Cfg::BM>() + E::template stage_bytes<Cfg::BN>()); }

template <int P> struct EngineOf;
using EngF64 = EngF64T<16>;
template <> struct EngineOf<kF64> { using type = EngF64; };
template <> struct EngineOf<kF32> { using type = EngF32; };
template <> struct EngineOf<kBF16x3> { using type = EngSplit<2>; };
template <> struct EngineOf<kBF16x6> { using type = EngSplit<3>; };
template <> struct EngineOf<kF16x3> { using type = EngSplit<2, true>; };

// Main loop over nk slices.  smem: smem_bytes<E, Cfg>() bytes of LDS, laid
// out [A stage 0][A stage 1][B stage 0][B stage 1].  mma(SA, SB, acc)
// consumes one staged slice.  With b_is_a (square tiles whose two operands
// are the same panel) only A is loaded and staged, and mma reads it twice.
// DEPTH slices of global loads are in flight: with DEPTH = 2 the registers
// alternate between two sets, so the loads of slice kt+2 are issued while
// slice kt+1 is still being staged (a split engine's slice holds a few
// hundred cycles of MFMA work, shorter than a load's latency from HBM).  It
// costs the registers of one more set.
template <class E, class Cfg, int DEPTH = 1, class LA, class LB, class MMA>
__device__ __forceinline__ void gemm_mainloop_with(LA& la, LB& lb, int nk, typename E::template Acc<Cfg>& acc,
                                                   char* smem_generic, bool b_is_a, MMA&& mma) {
  constexpr int SA = E::template stage_bytes<Cfg::BM>();
  constexpr int SB = E::template stage_bytes<Cfg::BN>();
  lds_char* smem = (lds_char*)smem_generic;
  lds_char* As[2] = {smem, smem + SA};
  lds_char* Bs[2] = {smem + 2 * SA, smem + 2 * SA + SB};
  if (b_is_a) {
    Bs[0] = As[0];
    Bs[1] = As[1];
  }
  typename LA::type ra[LA::RR];
  typename LB::type rb[LB::RR];
  acc.zero();
  if (nk <= 0) return;
  la.fetch(0, ra);
  if (!b_is_a) lb.fetch(0, rb);
  static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
  if constexpr (DEPTH == 2) {
    // Every step issues its loads and staging writes on every path (past the
    // end they re-read slice nk-1 and stage unused data into the idle buffer),
    // and the loop runs an even number of steps (a last step past nk skips only
    // its MFMAs).  The in-order load counter then lets each wait cover exactly
    // the older set.
    typename LA::type ra2[LA::RR];
    typename LB::type rb2[LB::RR];
    la.fetch(nk > 1 ? 1 : 0, ra2);
    if (!b_is_a) lb.fetch(nk > 1 ? 1 : 0, rb2);
    E::template stash<Cfg::BM>(As[0], la, ra, 0);
    if (!b_is_a) E::template stash<Cfg::BN>(Bs[0], lb, rb, 0);
    __syncthreads();
    // slice kt: loads of slice kt+2 into the set that held slice kt (staged
    // already), MFMAs on stage kt&1, then slice kt+1 staged from the other set
    auto step = [&](int kt, typename LA::type (&fa)[LA::RR], typename LB::type (&fb)[LB::RR],
                    const typename LA::type (&sa)[LA::RR], const typename LB::type (&sb)[LB::RR]) {
      const int cur = kt & 1;
      const int kf = kt + 2 < nk ? kt + 2 : nk - 1;
      __builtin_amdgcn_s_setprio(1);
      la.fetch(kf, fa);
      if (!b_is_a) lb.fetch(kf, fb);
      __builtin_amdgcn_s_setprio(0);
      if (kt < nk) mma(As[cur], Bs[cur], acc);
      if ((kt + 1) % E::CHUNK == 0) acc.flush();
      E::template stash<Cfg::BM>(As[cur ^ 1], la, sa, kt + 1);
      if (!b_is_a) E::template stash<Cfg::BN>(Bs[cur ^ 1], lb, sb, kt + 1);
      __syncthreads();
    };
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, ra, rb, ra2, rb2);
      step(kt + 1, ra2, rb2, ra, rb);
    }
  } else {
    E::template stash<Cfg::BM>(As[0], la, ra, 0);
    if (!b_is_a) E::template stash<Cfg::BN>(Bs[0], lb, rb, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        // issue the next slice's global loads ahead of other waves' MFMAs, so
        // they are in flight for the whole slice
        __builtin_amdgcn_s_setprio(1);
        la.fetch(kt + 1, ra);
        if (!b_is_a) lb.fetch(kt + 1, rb);
        __builtin_amdgcn_s_setprio(0);
      }
      mma(As[cur], Bs[cur], acc);
      if ((kt + 1) % E::CHUNK == 0) acc.flush();
      if (more) {
        E::template stash<Cfg::BM>(As[cur ^ 1], la, ra, kt + 1);
        if (!b_is_a) E::template stash<Cfg::BN>(Bs[cur ^ 1], lb, rb, kt + 1);
      }
      __syncthreads();
    }
  }
  acc.flush();
}

template <class E, class Cfg, int DEPTH = 1, class LA, class LB>
__device__ __forceinline__ void gemm_mainloop(LA& la, LB& lb, int nk, typename E::template Acc<Cfg>& acc,
                                              char* smem_generic) {
  gemm_mainloop_with<E, Cfg, DEPTH>(la, lb, nk, acc, smem_generic, false,
                                    [&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
                                      E::template mma<Cfg>(SA, SB, c, regular_plan<Cfg>());
                                    });
}

// s_waitcnt vmcnt(n) for a wave-uniform n (0..31; larger n waits for 31),
// other counters untouched.  vmcnt's six bits sit at [3:0] and [15:14].
__device__ __forceinline__ void wait_vmcnt(int n) {
#define RIF_VMCNT(k) __builtin_amdgcn_s_waitcnt(((k) & 15) | (7 << 4) | (15 << 8) | (((k) >> 4) << 14))
#define RIF_VMCNT_CASE(k) case k: RIF_VMCNT(k); break;
  switch (n) {
    RIF_VMCNT_CASE(0) RIF_VMCNT_CASE(1) RIF_VMCNT_CASE(2) RIF_VMCNT_CASE(3) RIF_VMCNT_CASE(4)
    RIF_VMCNT_CASE(5) RIF_VMCNT_CASE(6) RIF_VMCNT_CASE(7) RIF_VMCNT_CASE(8) RIF_VMCNT_CASE(9)
    RIF_VMCNT_CASE(10) RIF_VMCNT_CASE(11) RIF_VMCNT_CASE(12) RIF_VMCNT_CASE(13) RIF_VMCNT_CASE(14)
    RIF_VMCNT_CASE(15) RIF_VMCNT_CASE(16) RIF_VMCNT_CASE(17) RIF_VMCNT_CASE(18) RIF_VMCNT_CASE(19)
    RIF_VMCNT_CASE(20) RIF_VMCNT_CASE(21) RIF_VMCNT_CASE(22) RIF_VMCNT_CASE(23) RIF_VMCNT_CASE(24)
    RIF_VMCNT_CASE(25) RIF_VMCNT_CASE(26) RIF_VMCNT_CASE(27) RIF_VMCNT_CASE(28) RIF_VMCNT_CASE(29)
    RIF_VMCNT_CASE(30)
    default: RIF_VMCNT(31); break;
  }
#undef RIF_VMCNT_CASE
#undef RIF_VMCNT
}

// Stages that fit in LDS for the direct-load main loop (at most 4).
template <class E, class Cfg>
constexpr int dma_stages() {
  constexpr int st = E::template stage_bytes<Cfg::BM>() + E::template stage_bytes<Cfg::BN>();
  return 163840 / st >= 4 ? 4 : 163840 / st;
}
template <class E, class Cfg>
constexpr int smem_bytes_dma() {
  return dma_stages<E, Cfg>() * (E::template stage_bytes<Cfg::BM>() + E::template stage_bytes<Cfg::BN>());
}

// Main loop for two direct-staged operands (PieceDma, XcDma64): S = S_ (or
// dma_stages()) LDS stages, S-1 slices of loads in flight; with b_is_a one
// panel is staged and read as both operands.  mma(SA, SB, acc) does a slice.  Per slice kt: wait for this wave's loads of
// slice kt (the loads of the S-2 later slices stay in flight), a plain
// s_barrier (so every wave's loads of slice kt have landed and every wave is
// done reading the stage about to be refilled), the loads of slice kt+S-1
// into that stage, then the MFMAs of slice kt.  The barrier carries no
// memory fence: a fence would wait for every load in flight.  Past the last
// slice the loads re-read slice nk-1 into a stage nobody reads, which keeps
// the count of loads per slice fixed for the waits.
template <class E, class Cfg, int S_ = 0, class LA, class LB, class MMA>
__device__ __forceinline__ void gemm_mainloop_dma_with(const LA& la, const LB& lb, int nk,
                                                       typename E::template Acc<Cfg>& acc, char* smem_generic,
                                                       bool b_is_a, MMA&& mma) {
  constexpr int S = S_ > 0 ? S_ : dma_stages<E, Cfg>();
  static_assert(S >= 2, "two stages at least");
  constexpr int SA = E::template stage_bytes<Cfg::BM>();
  constexpr int ST = SA + E::template stage_bytes<Cfg::BN>();
  lds_char* smem = (lds_char*)smem_generic;
  acc.zero();
  if (nk <= 0) return;
  // b_is_a: one panel staged (stage's A part) and read as both operands
  const int per_slice = la.count() + (b_is_a ? 0 : lb.count());
#pragma unroll
  for (int j = 0; j < S - 1; ++j) {
    const int k = j < nk ? j : nk - 1;
    la.issue(k, smem + j * ST);
    if (!b_is_a) lb.issue(k, smem + j * ST + SA);
  }
  for (int kt = 0; kt < nk; ++kt) {
    wait_vmcnt((S - 2) * per_slice);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const int kf = kt + S - 1 < nk ? kt + S - 1 : nk - 1;
    lds_char* sf = smem + ((kt + S - 1) % S) * ST;
    la.issue(kf, sf);
    if (!b_is_a) lb.issue(kf, sf + SA);
    const lds_char* sc = smem + (kt % S) * ST;
    mma(sc, b_is_a ? sc : sc + SA, acc);
    if ((kt + 1) % E::CHUNK == 0) acc.flush();
  }
  acc.flush();
  // no load may still write LDS when the workgroup moves on
  wait_vmcnt(0);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
}

// FP64 k-contiguous operand (element (x, k) at row(x)[k]) staged by direct
// global -> LDS loads into a [x][k] layout of BX rows of BK doubles (128 bytes
// per row at BK = 16, no padding) whose 16-byte chunks, two k each, are
// swizzled per row: chunk c of row x sits in slot c ^ (x % 8).  One wave
// instruction fills eight rows (1 KB); each lane loads the chunk that the
// swizzle puts in its slot, so eight lanes read one row's 128 contiguous bytes.
// Chunks at or past K read zeros (K even, so a chunk is all in or all out);
// a row that does not exist reads row `fallback` (its outputs are never
// stored).  Needs 16-byte aligned rows.  mma_xk_f64 reads this layout.
template <int NT, int BK, int BX>
struct KcDma64 {
  static_assert(BK == 16, "eight chunks per row");
  static constexpr int NW = NT / 64, ROWS = 8;            // rows per wave instruction
  static constexpr int NI = BX / (NW * ROWS);              // instructions per wave per slice
  static_assert(BX % (NW * ROWS) == 0, "whole row groups per wave");
  const double* src[NI];   // this lane's row base plus its chunk's first k
  int kc[NI];              // the chunk's first k within a slice
  int K;
  template <class RowPtr>
  __device__ void init(RowPtr rowptr, const double* fallback, int K_) {
    K = K_;
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int x = (w + j * NW) * ROWS + lane / 8, slot = lane % 8, c = slot ^ (x & 7);
      const double* r = rowptr(x);
      src[j] = (r ? r : fallback) + 2 * c;
      kc[j] = 2 * c;
    }
  }
  __device__ int count() const { return NI; }
  __device__ void issue(int kt, lds_char* S) const {
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const double* g = kt * BK + kc[j] < K ? src[j] + kt * BK : kDmaZeros + 2 * (lane & 7);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                       (__attribute__((address_space(3))) void*)(S + (w + j * NW) * ROWS * BK * 8),
                                       16, 0, 0);
    }
  }
};

// Persistent form of the direct-staged main loop: one workgroup computes the
// tiles t = first, first + step, ... below n.  make(t, la, lb) points the
// loaders at tile t and epi(t, acc) stores its result.  The loads keep running
// S-1 slices ahead across tile boundaries, so the next tile's first slices are
// in flight while this tile's epilogue stores, and no tile starts from empty
// stages.  The first slice of each later tile waits for all memory operations
// (the epilogue's stores are counted with the loads and need not retire in
// order with them); within a tile the waits are those of the single-tile loop.
template <class E, class Cfg, int S_, class LA, class LB, class Make, class Epi>
__device__ __forceinline__ void gemm_persistent_dma(long first, long step, long n, int nk, char* smem_generic,
                                                    Make&& make, Epi&& epi) {
  constexpr int S = S_ > 0 ? S_ : dma_stages<E, Cfg>();
  static_assert(S >= 2, "two stages at least");
  constexpr int SA = E::template stage_bytes<Cfg::BM>();
  constexpr int ST = SA + E::template stage_bytes<Cfg::BN>();
  lds_char* smem = (lds_char*)smem_generic;
  if (first >= n) return;
  typename E::template Acc<Cfg> acc;
  if (nk <= 0) {
    for (long t = first; t < n; t += step) {
      acc.zero();
      epi(t, acc);
    }
    return;
  }
  LA la;
  LB lb;
  long it = first;   // tile and slice of the next loads
  int ik = 0;
  make(it, la, lb);
  const int per_slice = la.count() + lb.count();
  // loads of the next slice in order; past the last tile they re-read the
  // last slice into a stage nobody reads, keeping the count per slice fixed
  auto issue_next = [&](lds_char* st) {
    if (it < n) {
      la.issue(ik, st);
      lb.issue(ik, st + SA);
      if (++ik == nk) {
        ik = 0;
        it += step;
        if (it < n) make(it, la, lb);
      }
    } else {
      la.issue(nk - 1, st);
      lb.issue(nk - 1, st + SA);
    }
  };
#pragma unroll
  for (int j = 0; j < S - 1; ++j) issue_next(smem + j * ST);
  long g = 0;   // slices computed so far (the stage ring position)
  for (long t = first; t < n; t += step) {
    acc.zero();
    for (int kt = 0; kt < nk; ++kt, ++g) {
      if (kt == 0 && t != first)
        wait_vmcnt(0);
      else
        wait_vmcnt((S - 2) * per_slice);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      issue_next(smem + (int)((g + S - 1) % S) * ST);
      const lds_char* sc = smem + (int)(g % S) * ST;
      E::template mma<Cfg>(sc, sc + SA, acc, regular_plan<Cfg>());
      if ((kt + 1) % E::CHUNK == 0) acc.flush();
    }
    acc.flush();
    epi(t, acc);
  }
  // no load may still write LDS when the workgroup ends
  wait_vmcnt(0);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
}

template <class E, class Cfg, int S_ = 0, class LA, class LB>
__device__ __forceinline__ void gemm_mainloop_dma(const LA& la, const LB& lb, int nk,
                                                  typename E::template Acc<Cfg>& acc, char* smem_generic) {
  gemm_mainloop_dma_with<E, Cfg, S_>(la, lb, nk, acc, smem_generic, false,
                                     [&](const lds_char* SA, const lds_char* SB, typename E::template Acc<Cfg>& c) {
                                       E::template mma<Cfg>(SA, SB, c, regular_plan<Cfg>());
                                     });
}

}  // namespace rif
