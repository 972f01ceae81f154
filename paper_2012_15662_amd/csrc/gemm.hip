// FP64 GEMM out[m][n] = sum_k A[k][m] B[k][n] (both operands k-major, row
// strides lda, ldb, ldo) with the tile shape chosen per problem.  It serves the
// large one-off product outside the build, the solve of the b preparation
// (n_aux x n_bf(n_bf+1)/2 x n_aux), where the build's fixed 64x64 small-GEMM
// tile leaves MFMA time unused.  With lower_a, A is zero past its first
// superdiagonal (A[k][m] = 0 for k > m + 1) and each row tile stops its k range
// there, so only exact zeros are skipped.  Same engine,
// loader and main loop as the build's GEMM steps (mfma_engine.hpp); tiles run
// m-fastest, so consecutive workgroups share the panel of B.
#include <algorithm>

#include "mfma_engine.hpp"
#include "rif_internal.hpp"

namespace rif {

namespace {
struct BigGemm {
  int M, N, K;
  const double* A;
  long lda;
  const double* B;
  long ldb;
  double* out;
  long ldo;
  int lower;   // A[k][m] = 0 for k > m + 1: a row tile m0 stops at k = m0 + BM + 1
};

using E64 = EngineOf<kF64>::type;
// 0: 128x128, 1: 64x64, 2: 128x64, 3: 64x128 (8 waves), 4: 64x64 (4 waves)
using G0 = TileCfg<128, 128, 16, 64, 32>;
using G1 = TileCfg<64, 64, 16, 16, 32>;
using G2 = TileCfg<128, 64, 16, 32, 32>;
using G3 = TileCfg<64, 128, 16, 32, 32>;
using G4 = TileCfg<64, 64, 16, 32, 32>;
constexpr int kBigVariants = 5;

template <class Cfg>
long big_tiles(const BigGemm& a) {
  return (long)((a.M + Cfg::BM - 1) / Cfg::BM) * ((a.N + Cfg::BN - 1) / Cfg::BN);
}

template <class Cfg>
__global__ __launch_bounds__(Cfg::NT) __attribute__((amdgpu_waves_per_eu(Cfg::NT == 512 ? 4 : 1))) void
k_gemm_big(BigGemm a) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<E64, Cfg>()];
  const long t = blockIdx.x;
  const int nmt = (a.M + Cfg::BM - 1) / Cfg::BM;
  const int m0 = (int)(t % nmt) * Cfg::BM, n0 = (int)(t / nmt) * Cfg::BN;
  const int M = a.M, N = a.N;
  const int K = a.lower ? min(a.K, m0 + Cfg::BM + 1) : a.K;   // only exact zeros are skipped
  XCSrc<double, Cfg::BM, E64::BK, Cfg::NT, E64::KV> la;
  la.init(a.A, a.lda, K, [&](int x, long& o) { o = m0 + x; return m0 + x < M; });
  XCSrc<double, Cfg::BN, E64::BK, Cfg::NT, E64::KV> lb;
  lb.init(a.B, a.ldb, K, [&](int x, long& o) { o = n0 + x; return n0 + x < N; });
  typename E64::template Acc<Cfg> acc;
  gemm_mainloop<E64, Cfg>(la, lb, (K + E64::BK - 1) / E64::BK, acc, smem);
  acc.for_each([&](int m, int n, double v) {
    if (m0 + m < M && n0 + n < N) a.out[(long)(m0 + m) * a.ldo + n0 + n] = v;
  });
}

template <class F>
decltype(auto) with_big(int v, F&& f) {
  switch (v) {
    case 0: return f(G0());
    case 1: return f(G1());
    case 2: return f(G2());
    case 3: return f(G3());
    default: return f(G4());
  }
}

// Rounds of resident workgroups times the tile area per useful output: the
// same wave-quantisation model as the build's steps.
template <class Cfg>
double big_cost(const BigGemm& a) {
  const int by_lds = 163840 / smem_bytes<E64, Cfg>(), by_waves = 32 / Cfg::NWAVES;
  const int per_cu = std::max(1, std::min(std::min(by_lds, by_waves), 4));
  const long tiles = big_tiles<Cfg>(a), slots = 256L * per_cu;
  const double useful = (double)a.M * a.N / ((double)tiles * Cfg::BM * Cfg::BN);
  return (double)((tiles + slots - 1) / slots) * Cfg::BM * Cfg::BN * per_cu / useful;
}
}  // namespace

rif_status op_gemm_big(rif_ctx* c, int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                       double* out, long ldo, bool lower_a) {
  const BigGemm a{M, N, K, A, lda, B, ldb, out, ldo, lower_a ? 1 : 0};
  auto run = [&](int v) -> rif_status {
    return with_big(v, [&](auto cfg) {
      using Cfg = decltype(cfg);
      hipLaunchKernelGGL((k_gemm_big<Cfg>), dim3((unsigned)big_tiles<Cfg>(a)), dim3(Cfg::NT), 0, c->stream, a);
      return check_launch(c, "gemm");
    });
  };
  int hv = 0;
  double best = 1e300;
  for (int v = 0; v < kBigVariants; ++v) {
    const double e = with_big(v, [&](auto cfg) { return big_cost<decltype(cfg)>(a); });
    if (e < best) { best = e; hv = v; }
  }
  const int v = pick_variant(c, "gemm", {M, N, K, lower_a ? 1 : 0}, kBigVariants, hv, run);
  if (v < 0) return RIF_EHIP;
  ProfScope ps(c, "gemm");
  return run(v);
}

}  // namespace rif
