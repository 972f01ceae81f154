// Preparation of the three-index factors b from the three-centre integrals
// T[k][mu][nu] = (mu nu|k) and the metric G_kl = (k|l) (Sec. II, RI): the
// metric is factorised as G = P L D L^T P^T (L unit lower triangular, D block
// diagonal with 1x1 and 2x2 blocks, Bunch-Kaufman partial pivoting), each D
// block's eigenvalues below delta are raised to delta (D~), and
//   b^T = D~^(-1/2) L^-1 P^T T,
// i.e. the solution of P L D~^(1/2) b^T = T.  Done once per molecule.
//
//   k_rowsum     ||G||_inf (max row sum of |G|), for the default delta
//   k_bk_init    working copy of G, L = I, perm, step state
//   k_bk_pivot   one workgroup: the pivot decision at the current column, the
//                symmetric interchange, the D block and the L column(s)
//   k_bk_update  trailing update A -= L_k D_k L_k^T (all workgroups)
//   k_bk_correct D~^(-1/2) per block (2x2 blocks in closed form)
//   k_linv_rows  X = L^-1, one wave per column (forward substitution), one
//                launch; k_linv (one column step at a time, rank-1 updates)
//                above 2048 auxiliary functions
//   k_compose    M'^T[i][k] = sum_r D~^(-1/2)[k][r] X[r][i]  (M' = D~^(-1/2) L^-1,
//                zero right of its first superdiagonal)
//   then b^T = M T on the FP64 MFMA GEMM (tile chosen per shape), over the packed upper triangles of
//   the slabs (k_pack_upper before, k_unpack_sym after).
//
// Pivot rule (alpha = (1 + sqrt 17)/8) at column k, with colmax/imax the
// largest |A_ik| below the diagonal (lowest index on ties) and rowmax the
// largest off-diagonal |A_{imax,j}| of the trailing row imax: 1x1 at k if
// |A_kk| >= alpha colmax or |A_kk| rowmax >= alpha colmax^2; else 1x1 at imax
// if |A_{imax,imax}| >= alpha rowmax; else 2x2 on (k, imax).  Interchanges
// also swap the rows of the L columns already computed (P L form).
#include <algorithm>
#include <cmath>
#include <string>

#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

namespace {
constexpr double kAlpha = 0.6403882032022076;   // (1 + sqrt(17)) / 8
constexpr int kPivThreads = 1024;
struct BkState { int k, kstep, next; };
}  // namespace

__global__ __launch_bounds__(256) void k_rowsum(int n, const double* __restrict__ G, double* __restrict__ rs) {
  // row sum i of |G| per wave, the lanes reading along the row
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  const double* g = G + (long)i * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += fabs(g[j]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) rs[i] = s;
}

__global__ __launch_bounds__(256) void k_delta(int nblk, const double* __restrict__ part, double* __restrict__ del) {
  // delta = sqrt(2^-52) * max row sum = 2^-26 * ||G||_inf
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) m = fmax(m, part[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) del[0] = red[0] * 0x1p-26;
}

__global__ __launch_bounds__(256) void k_bk_init(int n, const double* __restrict__ G, double* __restrict__ A,
                                                 double* __restrict__ L, double* __restrict__ D,
                                                 int* __restrict__ perm, int* __restrict__ bsz, BkState* st) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const long nn = (long)n * n;
  if (i < nn) {
    const int r = (int)(i / n), c = (int)(i - (long)r * n);
    A[i] = G[i];
    L[i] = r == c ? 1.0 : 0.0;
    D[i] = 0.0;
  }
  if (i < n) { perm[i] = (int)i; bsz[i] = 0; }
  if (i == 0) { st->k = 0; st->kstep = 0; st->next = 0; }
}

// Max of |v| with its index (lowest index on ties) over a workgroup.
__device__ void block_argmax(double& v, int& idx, double* sv, int* si) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = idx;
  __syncthreads();
  for (int h = kPivThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double a = sv[t], b = sv[t + h];
      const int ia = si[t], ib = si[t + h];
      if (b > a || (b == a && ib < ia)) { sv[t] = b; si[t] = ib; }
    }
    __syncthreads();
  }
  v = sv[0];
  idx = si[0];
  __syncthreads();
}

__global__ __launch_bounds__(kPivThreads) void k_bk_pivot(int n, double* __restrict__ A, double* __restrict__ L,
                                                          double* __restrict__ D, int* __restrict__ perm,
                                                          int* __restrict__ bsz, BkState* st) {
  __shared__ double sv[kPivThreads];
  __shared__ int si[kPivThreads];
  const int t = threadIdx.x;
  const int k = st->next;
  if (k >= n) {   // factorisation finished: the update launched after this does nothing
    if (t == 0) st->kstep = 0;
    return;
  }
  auto a = [&](int i, int j) -> double& { return A[(long)i * n + j]; };
  // column search below the diagonal
  double cm = 0.0;
  int im = n;
  for (int i = k + 1 + t; i < n; i += kPivThreads) {
    const double v = fabs(a(i, k));
    if (v > cm || (v == cm && i < im)) { cm = v; im = i; }
  }
  block_argmax(cm, im, sv, si);
  const double absakk = fabs(a(k, k));
  int kstep = 1, kp = k;
  if (k + 1 < n && fmax(absakk, cm) != 0.0 && absakk < kAlpha * cm) {
    // rowmax: row imax left of the diagonal (columns k..imax-1), column imax
    // below it (the trailing matrix is symmetric only to rounding)
    double rm = 0.0;
    int dummy = 0;
    for (int j = k + t; j < n; j += kPivThreads)
      if (j != im) rm = fmax(rm, fabs(j < im ? a(im, j) : a(j, im)));
    block_argmax(rm, dummy, sv, si);
    if (absakk * rm >= kAlpha * cm * cm) {
      kstep = 1; kp = k;
    } else if (fabs(a(im, im)) >= kAlpha * rm) {
      kstep = 1; kp = im;
    } else {
      kstep = 2; kp = im;
    }
  }
  const int kk = k + kstep - 1;
  if (kp != kk) {
    // symmetric interchange: rows kk <-> kp (all columns), then columns
    for (int j = t; j < n; j += kPivThreads) {
      const double x = a(kk, j);
      a(kk, j) = a(kp, j);
      a(kp, j) = x;
    }
    __syncthreads();
    for (int i = t; i < n; i += kPivThreads) {
      const double x = a(i, kk);
      a(i, kk) = a(i, kp);
      a(i, kp) = x;
    }
    for (int j = t; j < k; j += kPivThreads) {   // rows of the L columns already final
      const double x = L[(long)kk * n + j];
      L[(long)kk * n + j] = L[(long)kp * n + j];
      L[(long)kp * n + j] = x;
    }
    if (t == 0) {
      const int x = perm[kk];
      perm[kk] = perm[kp];
      perm[kp] = x;
    }
    __syncthreads();
  }
  if (kstep == 1) {
    const double d = a(k, k);
    if (t == 0) { D[(long)k * n + k] = d; bsz[k] = 1; }
    if (d != 0.0)
      for (int i = k + 1 + t; i < n; i += kPivThreads) L[(long)i * n + k] = a(i, k) / d;
  } else {
    const double e00 = a(k, k), e10 = a(k + 1, k), e11 = a(k + 1, k + 1);
    const double det = e00 * e11 - e10 * e10;
    const double i00 = e11 / det, i01 = -e10 / det, i11 = e00 / det;
    if (t == 0) {
      D[(long)k * n + k] = e00;
      D[(long)k * n + k + 1] = e10;
      D[(long)(k + 1) * n + k] = e10;
      D[(long)(k + 1) * n + k + 1] = e11;
      bsz[k] = 2;
      bsz[k + 1] = 0;
    }
    for (int i = k + 2 + t; i < n; i += kPivThreads) {
      const double x0 = a(i, k), x1 = a(i, k + 1);
      L[(long)i * n + k] = x0 * i00 + x1 * i01;
      L[(long)i * n + k + 1] = x0 * i01 + x1 * i11;
    }
  }
  if (t == 0) {
    st->k = k;
    st->kstep = kstep;
    st->next = k + kstep;
  }
}

// Trailing update of the step just decided: for i, j >= k + kstep,
//   1x1: A_ij -= L_ik A_jk;  2x2: A_ij -= L_ik A_jk + L_i,k+1 A_j,k+1.
__global__ __launch_bounds__(256) void k_bk_update(int n, double* __restrict__ A, const double* __restrict__ L,
                                                   const BkState* st) {
  const int k = st->k, s = st->kstep;
  const int k0 = k + s;
  if (s == 0 || k0 >= n) return;
  const long m = n - k0, mm = m * m;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < mm; e += (long)gridDim.x * 256) {
    const int i = k0 + (int)(e / m), j = k0 + (int)(e - (e / m) * m);
    double v = A[(long)i * n + j] - L[(long)i * n + k] * A[(long)j * n + k];
    if (s == 2) v -= L[(long)i * n + k + 1] * A[(long)j * n + k + 1];
    A[(long)i * n + j] = v;
  }
}

// D~^(-1/2) per block into Dih (dense, zero outside the blocks); counts the
// raised eigenvalues.
__global__ __launch_bounds__(256) void k_bk_correct(int n, const double* __restrict__ D,
                                                    const int* __restrict__ bsz, const double* __restrict__ delta_p,
                                                    double delta_in, double* __restrict__ Dih,
                                                    int* __restrict__ nraised) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const double delta = delta_in > 0.0 ? delta_in : delta_p[0];
  const int s = bsz[k];
  if (s == 1) {
    const double w = D[(long)k * n + k];
    const double wt = w < delta ? delta : w;
    if (w < delta) atomicAdd(nraised, 1);
    Dih[(long)k * n + k] = 1.0 / sqrt(wt);
  } else if (s == 2) {
    const double a = D[(long)k * n + k], b = D[(long)(k + 1) * n + k], c = D[(long)(k + 1) * n + k + 1];
    // eigenvalues and the unit eigenvector (cs, sn) of the larger one
    const double h = 0.5 * (a - c), r = sqrt(h * h + b * b);
    const double w1 = 0.5 * (a + c) + r, w2 = 0.5 * (a + c) - r;
    double cs, sn;
    if (h >= 0.0) {
      const double x = h + r;
      const double nrm = sqrt(x * x + b * b);
      cs = nrm > 0.0 ? x / nrm : 1.0;
      sn = nrm > 0.0 ? b / nrm : 0.0;
    } else {
      const double y = r - h;
      const double nrm = sqrt(b * b + y * y);
      cs = nrm > 0.0 ? b / nrm : 1.0;
      sn = nrm > 0.0 ? y / nrm : 0.0;
    }
    const double t1 = w1 < delta ? delta : w1, t2 = w2 < delta ? delta : w2;
    if (w1 < delta) atomicAdd(nraised, 1);
    if (w2 < delta) atomicAdd(nraised, 1);
    const double f1 = 1.0 / sqrt(t1), f2 = 1.0 / sqrt(t2);
    // Q = [[cs, -sn], [sn, cs]], Dih = Q diag(f1, f2) Q^T
    Dih[(long)k * n + k] = cs * cs * f1 + sn * sn * f2;
    Dih[(long)k * n + k + 1] = cs * sn * (f1 - f2);
    Dih[(long)(k + 1) * n + k] = cs * sn * (f1 - f2);
    Dih[(long)(k + 1) * n + k + 1] = sn * sn * f1 + cs * cs * f2;
  }
}

__global__ __launch_bounds__(256) void k_fill_eye(long nn, int n, double* __restrict__ X, double* __restrict__ Dih) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= nn) return;
  const int r = (int)(i / n), c = (int)(i - (long)r * n);
  X[i] = r == c ? 1.0 : 0.0;
  Dih[i] = 0.0;
}

// Column step k of X = L^-1: X[i][j] -= L[i][k] X[k][j] for i > k, j <= k.
__global__ __launch_bounds__(256) void k_linv(int n, int k, const double* __restrict__ L, double* __restrict__ X) {
  const long m = n - k - 1, w = k + 1, mm = m * w;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < mm; e += (long)gridDim.x * 256) {
    const int i = k + 1 + (int)(e / w), j = (int)(e - (e / w) * w);
    X[(long)i * n + j] -= L[(long)i * n + k] * X[(long)k * n + j];
  }
}

// M^T[perm[i]][k] = sum_r Dih[k][r] X[r][i] (Dih block diagonal: r in k's block).
__global__ __launch_bounds__(256) void k_compose(int n, const double* __restrict__ Dih, const int* __restrict__ bsz,
                                                 const double* __restrict__ X, double* __restrict__ Mt) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n * n) return;
  const int k = (int)(e / n), i = (int)(e - (long)k * n);
  double v = Dih[(long)k * n + k] * X[(long)k * n + i];
  if (k + 1 < n && bsz[k] == 2) v += Dih[(long)k * n + k + 1] * X[(long)(k + 1) * n + i];
  if (k > 0 && bsz[k] == 0) v += Dih[(long)k * n + k - 1] * X[(long)(k - 1) * n + i];
  Mt[(long)i * n + k] = v;
}

// ---- the factorisation in one cooperative launch -----------------------------
// Row i of A lives in the LDS of workgroup i mod G for the whole factorisation;
// its entries left of the current column, no longer needed as A, hold row i of
// L.  Workgroups exchange data through single-write slots: each slot is filled
// beforehand with a signalling-NaN pattern that no arithmetic result takes
// (arithmetic on NaNs yields quiet NaNs), written once with an agent-scope
// atomic store, and read by polling it with agent-scope atomic loads until it
// no longer holds that pattern.  Every wait is bounded; past the limit, or once
// another workgroup has flagged a timeout, a workgroup flags it and returns.
// Per step at column k:
//   1. every workgroup reads column k (C1; each workgroup published its rows'
//      entries of it at the end of the previous step, before the rest of its
//      update) and forms colmax, imax and |A_kk| itself (the same data and
//      order-free reductions, so the same decision everywhere);
//   2. where the first pivot test fails: its rows' entries of column imax
//      (CI) and, from the owners of rows imax, k and k+1, those whole rows (RI,
//      RK, RK1: the only rows an interchange can move); every workgroup forms
//      rowmax and takes the decision;
//   3. every workgroup forms the pivot column(s) after the interchange from
//      column k and column imax, swaps the interchanged columns in its rows,
//      takes over a moved row (from RK, RK1 or RI), writes its L entries and
//      updates its rows with the arithmetic of k_bk_pivot and k_bk_update.
// Workgroup 0 keeps perm, the block sizes and D.
constexpr unsigned long long kBkEmpty = 0x7FF4C0FFEE5E7F11ull;   // signalling NaN
constexpr size_t kBkLds = 150 * 1024;

struct BkcArgs {
  int n, G;
  const double* Gm;              // [n][n] the metric
  double *L, *D;                 // [n][n] out
  int *perm, *bsz;               // [n] out (bsz zero-filled beforehand)
  double *C1, *CI;               // [n][n] slots: C1[k][i] = A_ik, CI[k][i] = A_i,imax
  double *RK, *RK1, *RI;         // [n][n] slots: whole rows k, k+1, imax at step k
  int* err;
  long long spin;                // polls of one value before giving up; < 0: give up at once
};

__device__ __forceinline__ void bk_put(double* p, double v) {
  __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long bk_peek(const double* p) {
  return __hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// dst[j] = slot src[j] for j in [j0, j1), strided over the workgroup
__device__ bool bk_take_range(const double* src, double* dst, int j0, int j1, const int* err, long long spin) {
  if (spin < 0) return false;
  for (int j = j0 + (int)threadIdx.x; j < j1; j += 256) {
    unsigned long long u = bk_peek(src + j);
    for (long long s = 0; u == kBkEmpty; ++s) {
      if (s >= spin || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
      __builtin_amdgcn_s_sleep(1);
      u = bk_peek(src + j);
    }
    dst[j] = __longlong_as_double((long long)u);
  }
  return true;
}

__global__ __launch_bounds__(256) void k_bk_coop(BkcArgs a) {
  extern __shared__ double sm[];
  const int n = a.n, G = a.G, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int R = g < n ? (n - g + G - 1) / G : 0;   // rows i = g + G t, t < R
  double* rows = sm;                                // [R][n]
  double* c1 = rows + (long)R * n;                  // column k
  double* ci = c1 + n;                              // column imax
  double* ri = ci + n;                              // row imax
  double* ck = ri + n;                              // column k after the interchange
  double* cq = ck + n;                              // column k+1 after the interchange (2x2)
  for (long x = tid; x < (long)R * n; x += 256) {
    const int t = (int)(x / n), j = (int)(x - (long)t * n);
    rows[x] = a.Gm[(long)(g + G * t) * n + j];
  }
  if (g == 0)
    for (int i = tid; i < n; i += 256) a.perm[i] = i;
  __syncthreads();
  auto fail = [&]() { atomicExch(a.err, 1); };
  int k = 0;
  while (k < n) {
    const int t0 = k > g ? (k - g + G - 1) / G : 0;   // first row held here at or past k
    // 1. column k
    {
      double* C1k = a.C1 + (long)k * n;
      if (k == 0)
        for (int t = wv; t < R; t += 4)
          if (lane == 0) bk_put(C1k + g + G * t, rows[(long)t * n]);
      const bool ok = bk_take_range(C1k, c1, k, n, a.err, a.spin);
      if (!ok) fail();
      if (__syncthreads_or(!ok)) return;
    }
    // colmax / imax below the diagonal (lowest index on ties; NaNs never
    // chosen; 0 and k+1 when the column is zero), the same in every wave
    double cm = 0.0;
    int im = n;
    for (int i = k + 1 + lane; i < n; i += 64) {
      const double v = fabs(c1[i]);
      if (v > cm || (v == cm && i < im)) { cm = v; im = i; }
    }
    {
      const double top = wave_max_dpp(cm);
      im = wave_min_int_dpp(cm == top ? im : n);
      cm = top;
    }
    const double absakk = fabs(c1[k]);
    int kstep = 1, kp = k;
    if (k + 1 < n && fmax(absakk, cm) != 0.0 && absakk < kAlpha * cm) {
      // 2. column imax and row imax; rowmax over row imax left of the diagonal
      //    (columns k..imax-1) and column imax below it
      double* CIk = a.CI + (long)k * n;
      double* RIk = a.RI + (long)k * n;
      for (int t = t0 + wv; t < R; t += 4)
        if (lane == 0) bk_put(CIk + g + G * t, rows[(long)t * n + im]);
      if (im % G == g)
        for (int j = tid; j < n; j += 256) bk_put(RIk + j, rows[(long)(im / G) * n + j]);
      if (k % G == g)
        for (int j = tid; j < n; j += 256) bk_put(a.RK + (long)k * n + j, rows[(long)(k / G) * n + j]);
      if ((k + 1) % G == g)
        for (int j = tid; j < n; j += 256) bk_put(a.RK1 + (long)k * n + j, rows[(long)((k + 1) / G) * n + j]);
      bool ok = bk_take_range(CIk, ci, k, n, a.err, a.spin);
      ok = ok && bk_take_range(RIk, ri, k, n, a.err, a.spin);
      if (!ok) fail();
      if (__syncthreads_or(!ok)) return;
      double rm = 0.0;
      for (int j = k + lane; j < n; j += 64)
        if (j != im) rm = fmax(rm, fabs(j < im ? ri[j] : ci[j]));
      rm = wave_max_dpp(rm);
      if (absakk * rm >= kAlpha * cm * cm) {
        kstep = 1; kp = k;
      } else if (fabs(ri[im]) >= kAlpha * rm) {
        kstep = 1; kp = im;
      } else {
        kstep = 2; kp = im;
      }
    }
    const int kk = k + kstep - 1;
    auto pi = [&](int j) { return j == kk ? kp : (j == kp ? kk : j); };
    // 3. pivot column(s) after the interchange (kk kp)
    for (int j = k + tid; j < n; j += 256) {
      if (kstep == 1) {
        ck[j] = kp == k ? c1[j] : ci[pi(j)];
      } else {
        ck[j] = c1[pi(j)];
        cq[j] = ci[pi(j)];
      }
    }
    if (kp != kk) {
      // the row moving into a position held here (its whole row, L part included)
      const double* from = nullptr;
      int tdst = -1;
      if (kk % G == g) { from = a.RI + (long)k * n; tdst = kk / G; }                          // old row kp
      else if (kp % G == g) { from = (kstep == 1 ? a.RK : a.RK1) + (long)k * n; tdst = kp / G; }   // old row kk
      if (kk % G == g && kp % G == g) {   // both positions held here: swap in place
        from = nullptr;
        for (int j = tid; j < n; j += 256) {
          const double x = rows[(long)(kk / G) * n + j];
          rows[(long)(kk / G) * n + j] = rows[(long)(kp / G) * n + j];
          rows[(long)(kp / G) * n + j] = x;
        }
      }
      if (from) {
        const bool ok = bk_take_range(from, rows + (long)tdst * n, 0, n, a.err, a.spin);
        if (!ok) fail();
        if (__syncthreads_or(!ok)) return;
      }
      __syncthreads();
      // columns kk <-> kp in the rows still active
      for (int t = t0 + wv; t < R; t += 4)
        if (lane == 0) {
          double* r = rows + (long)t * n;
          const double x = r[kk];
          r[kk] = r[kp];
          r[kp] = x;
        }
      if (g == 0 && tid == 0) {
        const int x = a.perm[kk];
        a.perm[kk] = a.perm[kp];
        a.perm[kp] = x;
      }
    }
    __syncthreads();
    // D block, L entries and the trailing update on the rows held here; each
    // row's entry of the next pivot column k0 is published before the rest
    const int k0 = k + kstep;
    double* C1n = a.C1 + (long)(k0 < n ? k0 : 0) * n;
    if (kstep == 1) {
      const double d = ck[k];
      if (g == 0 && tid == 0) { a.D[(long)k * n + k] = d; a.bsz[k] = 1; }
      for (int t = (k0 > g ? (k0 - g + G - 1) / G : 0) + wv; t < R; t += 4) {
        double* r = rows + (long)t * n;
        const int i = g + G * t;
        const double l = d != 0.0 ? ck[i] / d : 0.0;
        if (lane == 0) bk_put(C1n + i, r[k0] - l * ck[k0]);   // next pivot column first
        for (int j = k0 + lane; j < n; j += 64) r[j] = r[j] - l * ck[j];
        if (lane == 0) r[k] = l;
      }
    } else {
      const double e00 = ck[k], e10 = ck[k + 1], e11 = cq[k + 1];
      const double det = e00 * e11 - e10 * e10;
      const double i00 = e11 / det, i01 = -e10 / det, i11 = e00 / det;
      if (g == 0 && tid == 0) {
        a.D[(long)k * n + k] = e00;
        a.D[(long)k * n + k + 1] = e10;
        a.D[(long)(k + 1) * n + k] = e10;
        a.D[(long)(k + 1) * n + k + 1] = e11;
        a.bsz[k] = 2;
        a.bsz[k + 1] = 0;
      }
      if ((k + 1) % G == g && tid == 0) rows[(long)((k + 1) / G) * n + k] = 0.0;   // L is I on the block
      for (int t = (k0 > g ? (k0 - g + G - 1) / G : 0) + wv; t < R; t += 4) {
        double* r = rows + (long)t * n;
        const int i = g + G * t;
        const double x0 = ck[i], x1 = cq[i];
        const double l0 = x0 * i00 + x1 * i01, l1 = x0 * i01 + x1 * i11;
        if (lane == 0) {   // next pivot column first
          double v = r[k0] - l0 * ck[k0];
          v -= l1 * cq[k0];
          bk_put(C1n + i, v);
        }
        for (int j = k0 + lane; j < n; j += 64) {
          double v = r[j] - l0 * ck[j];
          v -= l1 * cq[j];
          r[j] = v;
        }
        if (lane == 0) { r[k] = l0; r[k + 1] = l1; }
      }
    }
    __syncthreads();
    k = k0;
  }
  // L: the left parts of the rows, unit diagonal, zero above
  for (long x = tid; x < (long)R * n; x += 256) {
    const int t = (int)(x / n), j = (int)(x - (long)t * n), i = g + G * t;
    a.L[(long)i * n + j] = j < i ? rows[x] : (j == i ? 1.0 : 0.0);
  }
}

__global__ void k_bk_coop_reset(unsigned long long* slots, long count, int* err) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) slots[i] = kBkEmpty;
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}
// a timed-out factorisation leaves 1x1 blocks of NaN on the diagonal of D, so
// every slab of b comes out NaN, never silently wrong
__global__ void k_bk_coop_check(int n, const int* err, double* D, int* bsz) {
  if (*err == 0) return;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    D[(long)i * n + i] = __longlong_as_double(0x7FF8000000000000ll);
    bsz[i] = 1;
  }
}

size_t bk_coop_lds(int n, int G) { return (size_t)(((n + G - 1) / G) + 5L) * n * sizeof(double); }

// X = L^-1 by columns, one wave per column j: x_j = 1 and, for i > j in order,
// x_i = -sum_{j <= k < i} L[i][k] x_k (forward substitution on L x = e_j).
// The four waves of a workgroup take four adjacent columns and share each row
// of L through a double-buffered LDS row: the next row's loads are issued
// before the current row's dot products and stored after them.  Needs
// n <= kLinvMaxN (eight row elements per thread).
constexpr int kLinvMaxN = 2048;
__global__ __launch_bounds__(256) void k_linv_rows(int n, const double* __restrict__ L, double* __restrict__ X) {
  extern __shared__ double sh[];
  double* rowbuf = sh;         // [2][n]
  double* xs = sh + 2L * n;    // [4][n]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j0 = blockIdx.x * 4, j = j0 + w;
  double* x = xs + (long)w * n;
  for (int k = lane; k < n; k += 64) x[k] = k == j ? 1.0 : 0.0;
  const int i0 = j0 + 1;
  if (i0 < n)
    for (int k = threadIdx.x; k < i0; k += 256) rowbuf[k] = L[(long)i0 * n + k];
  __syncthreads();
  for (int i = i0; i < n; ++i) {
    const double* cur = rowbuf + (long)((i - i0) & 1) * n;
    double* nxt = rowbuf + (long)((i - i0 + 1) & 1) * n;
    const int in = i + 1;
    double pre[kLinvMaxN / 256];
#pragma unroll
    for (int u = 0; u < kLinvMaxN / 256; ++u) {
      const int k = threadIdx.x + 256 * u;
      pre[u] = in < n && k < in ? L[(long)in * n + k] : 0.0;
    }
    if (j < n && i > j) {   // whole wave
      double s = 0.0;
      for (int k = j + lane; k < i; k += 64) s += cur[k] * x[k];
      s = wave_sum_dpp(s);
      if (lane == 0) x[i] = -s;
    }
#pragma unroll
    for (int u = 0; u < kLinvMaxN / 256; ++u) {
      const int k = threadIdx.x + 256 * u;
      if (in < n && k < in) nxt[k] = pre[u];
    }
    __syncthreads();
  }
  // columns j0..j0+3 of X, four adjacent doubles per row
  for (int y = threadIdx.x; y < 4 * n; y += 256) {
    const int i = y >> 2, c = y & 3;
    if (j0 + c < n) X[(long)i * n + j0 + c] = xs[(long)c * n + i];
  }
}

// The solve works on the upper triangle of each slab only (T and b are
// symmetric in mu, nu), with the slabs in pivot order: packed by rows,
// Tp[i][o(mu) + nu - mu] = T[perm[i]][mu][nu] for nu >= mu,
// o(mu) = mu nb - mu (mu - 1) / 2, so that b^T = M' Tp with M' = D~^(-1/2) L^-1
// (the (P^T T)[i] = T[perm[i]] of the solve).  One workgroup per (i, mu) row,
// grid-strided; reads and writes both run along nu.
__global__ __launch_bounds__(256) void k_pack_upper(int nb, long rows, const double* __restrict__ T,
                                                    const int* __restrict__ perm, double* __restrict__ Tp) {
  const long npk = (long)nb * (nb + 1) / 2;
  for (long rr = blockIdx.x; rr < rows; rr += gridDim.x) {
    const long k = rr / nb;
    const int mu = (int)(rr - k * nb);
    const double* src = T + ((long)perm[k] * nb + mu) * nb;
    double* dst = Tp + k * npk + (long)mu * nb - (long)mu * (mu - 1) / 2 - mu;
    for (int nu = mu + threadIdx.x; nu < nb; nu += 256) dst[nu] = src[nu];
  }
}
// b[k] from the packed solution, by 64x64 tiles (rb <= cb) of each slab: the
// tile's upper-triangle elements are read once along c into LDS and written
// to (r, c) and, through the LDS transpose, to (c, r), both along rows.
constexpr int kUT = 64;
__global__ __launch_bounds__(256) void k_unpack_sym(int nb, long ntiles, const double* __restrict__ bp,
                                                    double* __restrict__ b) {
  __shared__ double t[kUT][kUT + 1];
  const long npk = (long)nb * (nb + 1) / 2;
  const int nbt = (nb + kUT - 1) / kUT, per = nbt * (nbt + 1) / 2;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (long tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
    const long k = tt / per;
    int rem = (int)(tt - k * per), rb = 0;
    while (rem >= nbt - rb) { rem -= nbt - rb; ++rb; }
    const int cb = rb + rem, r0 = rb * kUT, c0 = cb * kUT;
    const double* src = bp + k * npk;
    double* dst = b + k * (long)nb * nb;
    __syncthreads();
    for (int y = ty; y < kUT; y += 4) {
      const int r = r0 + y, cc = c0 + tx;
      if (r < nb && cc < nb && cc >= r) t[y][tx] = src[(long)r * nb - (long)r * (r - 1) / 2 + (cc - r)];
    }
    __syncthreads();
    for (int y = ty; y < kUT; y += 4) {
      const int r = r0 + y, cc = c0 + tx;   // (r, cc) from the upper triangle: itself or its mirror
      if (r < nb && cc < nb) dst[(long)r * nb + cc] = cc >= r ? t[y][tx] : t[tx][y];
    }
    if (rb != cb) {
      for (int y = ty; y < kUT; y += 4) {
        const int r = c0 + y, cc = r0 + tx;   // lower tile (cb, rb): element (r, cc) = upper (cc, r)
        if (r < nb && cc < nb) dst[(long)r * nb + cc] = t[tx][y];
      }
    }
  }
}

rif_status op_prepare_b(rif_ctx* c, int nb, int na, const double* T, const double* Gm, double delta,
                        double* b, int* perm_out, double* L_out, double* D_out, int* nraised_out) {
  const int n = na;
  const long nn = (long)n * n;
  Carve cv;
  const size_t oA = cv.take<double>(nn), oL = cv.take<double>(nn), oD = cv.take<double>(nn);
  const size_t oX = cv.take<double>(nn), oM = cv.take<double>(nn), oDih = cv.take<double>(nn);
  const size_t oP = cv.take<int>(n), oB = cv.take<int>(n), oS = cv.take<BkState>(1);
  const size_t oPart = cv.take<double>((size_t)n), oDel = cv.take<double>(1);
  const size_t oR = cv.take<int>(1);
  const long npk = (long)nb * (nb + 1) / 2;
  const size_t oBp = cv.take<double>((size_t)n * npk);   // packed solution
  // the one-launch factorisation where the rows fit the LDS of at most one
  // workgroup per CU (n_aux up to about 1600), else a pivot and an update
  // launch per column
  int G = 0;
  {
    int ncu = 0, coop = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device) == hipSuccess && coop) {
      G = std::min({ncu, n, 256});
      if (bk_coop_lds(n, G) > kBkLds) G = 0;
    }
    (void)hipGetLastError();
  }
  const size_t oSlots = G ? cv.take<double>((size_t)5 * nn) : 0, oErr = G ? cv.take<int>(1) : 0;
  rif_status st = ws_reserve(c, cv.off);
  if (st) return st;
  char* w = (char*)c->ws;
  double *A = (double*)(w + oA), *L = (double*)(w + oL), *D = (double*)(w + oD), *X = (double*)(w + oX);
  double *Mt = (double*)(w + oM), *Dih = (double*)(w + oDih), *part = (double*)(w + oPart);
  double* del = (double*)(w + oDel);
  int *perm = (int*)(w + oP), *bsz = (int*)(w + oB), *nr = (int*)(w + oR);
  BkState* sp = (BkState*)(w + oS);
  const unsigned gnn = (unsigned)((nn + 255) / 256);
  {
    ProfScope ps(c, "prep_factorise");
    hipLaunchKernelGGL(k_rowsum, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, c->stream, n, Gm, part);
    // max over the row sums, times sqrt(2^-52), into del
    hipLaunchKernelGGL(k_delta, dim3(1), dim3(256), 0, c->stream, n, part, del);
    hipLaunchKernelGGL(k_bk_init, dim3(gnn), dim3(256), 0, c->stream, n, Gm, A, L, D, perm, bsz, sp);
    if ((st = check_launch(c, "prep_init"))) return st;
    if (G) {
      BkcArgs ba{};
      ba.n = n;
      ba.G = G;
      ba.Gm = Gm;
      ba.L = L;
      ba.D = D;
      ba.perm = perm;
      ba.bsz = bsz;
      double* sl = (double*)(w + oSlots);
      ba.C1 = sl;
      ba.CI = sl + nn;
      ba.RK = sl + 2 * nn;
      ba.RK1 = sl + 3 * nn;
      ba.RI = sl + 4 * nn;
      ba.err = (int*)(w + oErr);
      ba.spin = c->wait_limit;
      const size_t lds = bk_coop_lds(n, G);
      if (lds > 64 * 1024 &&
          hipFuncSetAttribute((const void*)k_bk_coop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
              hipSuccess) {
        (void)hipGetLastError();
        return fail(c, RIF_EHIP, "factorisation: LDS attribute failed");
      }
      hipLaunchKernelGGL(k_bk_coop_reset, dim3((unsigned)std::min(4096L, (5 * nn + 255) / 256)), dim3(256), 0,
                         c->stream, (unsigned long long*)sl, 5 * nn, ba.err);
      if ((st = check_launch(c, "prep_factorise_reset"))) return st;
      void* args[] = {&ba};
      const hipError_t he =
          hipLaunchCooperativeKernel((const void*)k_bk_coop, dim3(G), dim3(256), args, (unsigned)lds, c->stream);
      if (he != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, RIF_EHIP, std::string("cooperative launch of the factorisation failed: ") +
                                     hipGetErrorString(he));
      }
      hipLaunchKernelGGL(k_bk_coop_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n,
                         (const int*)ba.err, D, bsz);
    } else {
      const unsigned gup = (unsigned)std::min(1024L, (nn + 255) / 256);
      for (int it = 0; it < n; ++it) {
        hipLaunchKernelGGL(k_bk_pivot, dim3(1), dim3(kPivThreads), 0, c->stream, n, A, L, D, perm, bsz, sp);
        hipLaunchKernelGGL(k_bk_update, dim3(gup), dim3(256), 0, c->stream, n, A, L, (const BkState*)sp);
      }
    }
    if ((st = check_launch(c, "prep_factorise"))) return st;
  }
  {
    ProfScope ps(c, "prep_correct_invert");
    hipLaunchKernelGGL(k_fill_eye, dim3(gnn), dim3(256), 0, c->stream, nn, n, X, Dih);
    if (hipMemsetAsync(nr, 0, sizeof(int), c->stream) != hipSuccess) return fail(c, RIF_EHIP, "hipMemsetAsync failed");
    hipLaunchKernelGGL(k_bk_correct, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, D, bsz, del,
                       delta, Dih, nr);
    if (n <= kLinvMaxN) {
      const size_t lds = (size_t)6 * n * sizeof(double);
      if (lds > 64 * 1024 &&
          hipFuncSetAttribute((const void*)k_linv_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
              hipSuccess) {
        (void)hipGetLastError();
        return fail(c, RIF_EHIP, "L^-1: LDS attribute failed");
      }
      hipLaunchKernelGGL(k_linv_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), lds, c->stream, n, L, X);
    } else {
      for (int k = 0; k + 1 < n; ++k) {
        const long work = (long)(n - k - 1) * (k + 1);
        const unsigned g = (unsigned)std::max(1L, std::min(1024L, (work + 255) / 256));
        hipLaunchKernelGGL(k_linv, dim3(g), dim3(256), 0, c->stream, n, k, L, X);
      }
    }
    hipLaunchKernelGGL(k_compose, dim3(gnn), dim3(256), 0, c->stream, n, Dih, bsz, X, Mt);
    if ((st = check_launch(c, "prep_correct_invert"))) return st;
  }
  {
    ProfScope ps(c, "prep_solve_gemm");
    // b^T[k][mu nu] = sum_i M'[k][i] T[perm[i]][mu nu] on the packed upper
    // triangles (A operand M'^T, i-major; B the packed T in pivot order,
    // staged in b's own buffer, which is free until the unpacking writes it),
    // then mirrored into b
    double* Tp = b;
    double* bp = (double*)(w + oBp);
    const long rows = (long)n * nb;
    const unsigned g = (unsigned)std::min(rows, 65536L);
    hipLaunchKernelGGL(k_pack_upper, dim3(g), dim3(256), 0, c->stream, nb, rows, T, (const int*)perm, Tp);
    if ((st = check_launch(c, "prep_pack"))) return st;
    // M' is zero right of its first superdiagonal: row tile m0 needs k < m0 + BM + 1 only
    if ((st = op_gemm_big(c, n, (int)npk, n, Mt, n, Tp, npk, bp, npk, true))) return st;
    const int nbt = (nb + kUT - 1) / kUT;
    const long ntiles = (long)n * (nbt * (nbt + 1) / 2);
    hipLaunchKernelGGL(k_unpack_sym, dim3((unsigned)std::min(ntiles, 65536L)), dim3(256), 0, c->stream, nb, ntiles,
                       (const double*)bp, b);
    if ((st = check_launch(c, "prep_unpack"))) return st;
  }
  if (perm_out && hipMemcpyAsync(perm_out, perm, sizeof(int) * n, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, RIF_EHIP, "copying perm failed");
  if (L_out && hipMemcpyAsync(L_out, L, sizeof(double) * nn, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, RIF_EHIP, "copying L failed");
  if (D_out && hipMemcpyAsync(D_out, D, sizeof(double) * nn, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, RIF_EHIP, "copying D failed");
  if (nraised_out && hipMemcpyAsync(nraised_out, nr, sizeof(int), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, RIF_EHIP, "copying the correction count failed");
  return RIF_OK;
}

}  // namespace rif
