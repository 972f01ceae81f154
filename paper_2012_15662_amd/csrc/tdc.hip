// Eigen-decomposition of the symmetric tridiagonal T = Q^T F^lambda Q left by
// the one-launch reduction (the orbital step's diagonalisation, Sec. II and
// Fig. 1), by divide and conquer: Cuppen's tearing, the rank-one secular
// equation, and Gu and Eisenstat's recomputed update vector, which keeps the
// eigenvectors orthogonal to working precision however close the eigenvalues.
//
// Tearing.  T splits at row m into T1 (rows < m) and T2 (rows >= m) joined by
// e = T[m-1][m]: with beta = |e| and sigma = sign(e),
//   T = diag(T1 - beta e_last e_last^T, T2 - beta e_0 e_0^T) + beta w w^T,
//   w = (e_last ; sigma e_0).
// The range [0, n) is halved recursively (block p of level t is
// [floor(p n / 2^t), floor((p+1) n / 2^t))) down to leaves of at most 16 rows,
// so every split point's two diagonal corrections fall on leaf boundaries.
//
// Leaves: implicit symmetric QR steps with the Wilkinson shift, the rotations
// accumulated into the leaf's eigenvector matrix (Golub and Van Loan,
// Sec. 8.3), one wave per leaf.
//
// Merge of two solved halves (T1 = Z1 D1 Z1^T, T2 = Z2 D2 Z2^T):
//   T = Zh (D + rho z z^T) Zh^T,  Zh = diag(Z1, Z2),
//   z = (last row of Z1 ; sigma first row of Z2) / sqrt(2),  rho = 2 beta.
// 1. Sort D (a merge of two sorted lists), carrying z and the source column.
// 2. Deflation, with tol = 8 eps max(max|D|, rho): an entry with
//    rho |z_j| <= tol keeps eigenvalue D_j and its column of Zh.  Of two
//    neighbouring survivors p < j, a plane rotation moves z_p's weight onto
//    z_j; it leaves the off-diagonal (D_p - D_j) z_p z_j / (z_p^2 + z_j^2),
//    and when that is <= tol, p is deflated with the rotated D_p.
// 3. The k survivors (D strictly increasing, z nonzero) have one root of
//    f(lambda) = 1 + rho sum_j z_j^2 / (D_j - lambda) in each gap
//    (D_i, D_{i+1}) and one in (D_k, D_k + rho sum z^2].  Each root is held
//    as lambda_i = D_o + tau_i with the nearer pole o as origin (the sign of f
//    at the gap's midpoint decides), so every difference D_j - lambda_i is
//    (D_j - D_o) - tau_i to high relative accuracy.  tau_i is found by steps
//    of a two-pole rational model of f (a few per root), safeguarded by a
//    bracket and by bisection on the bit pattern of |tau| (the order of
//    positive doubles is the order of their bits), which alone ends within one
//    ulp in at most 64 evaluations of f whatever the scale of tau.
// 4. Gu-Eisenstat: the roots are exact eigenvalues of D + rho zh zh^T with
//      zh_j^2 = (lambda_j - D_j)/rho * prod_{i != j} (lambda_i - D_j)/(D_i - D_j)
//    (sign of z_j), and the eigenvectors are u_i = (zh_j / (D_j - lambda_i))_j
//    normalised; these are orthogonal to working precision.
// 5. Eigenvectors of T: Zh P R U, P the sort, R the deflation rotations, U
//    the u_i with unit columns for the deflated entries, columns in ascending
//    order of eigenvalue.  P and R are folded into the small matrix
//    B = P R U (rows of U permuted and rotated), and the products Zh B of a
//    level are one FP64 MFMA launch.
//
// Eigenvectors are kept as rows: Zt[c][r] = component r of eigenvector c, so
// that the merge product Zt_new = B^T Zt has both operands k-major for the
// engine's GEMM.  The two halves' blocks sit on the diagonal of an n x n
// array whose other entries are zero, which makes that block Zh^T itself.
// Every level runs as seven launches, each covering all of its merges.
#include <algorithm>
#include <string>

#include "mfma_engine.hpp"
#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

namespace {
constexpr int kLeaf = 16;
constexpr int kTdcMaxN = 2048;
constexpr double kEps = 2.220446049250313e-16;   // 2^-52

__host__ __device__ inline int cut(int n, int t, long p) { return (int)((p * (long)n) >> t); }

int tdc_levels(int n) {   // smallest T with ceil(n / 2^T) <= kLeaf
  int T = 0;
  while (((n + (1 << T) - 1) >> T) > kLeaf) ++T;
  return T;
}
int tdc_smax(int n, int t) { return (n + (1 << t) - 1) >> t; }

struct TdcArgs {
  int n;
  double* d;           // [n] in: T's diagonal; out: eigenvalues, ascending
  const double* e;     // [n-1] T's off-diagonal
  double* B;           // [n][n] merge matrices (diagonal blocks)
  // per merge, at the merge's first row lo: counts and rho
  int *kcnt, *nrot;
  double* rho;
  // per merge entry (index lo + i)
  double *dk, *zk;     // survivors: poles and update vector (sorted)
  int* ndrow;          // survivor's source row in B
  double* dvs;         // deflated eigenvalues, ascending
  int* dvrow;          // their source rows in B
  int *rp, *rj;        // deflation rotations: source rows
  double *rc, *rs;     //   and cosine / sine
  int* org;            // root i's origin pole
  double* tau;         // root i = dk[org] + tau
  double* zh;          // recomputed update vector
  double* invn;        // 1 / |u_i|
  int* colsrc;         // output column c: root i (>= 0) or deflated t (-(t+1))
  int* err;            // set by a non-finite T or a leaf that fails to converge
};

__device__ __forceinline__ double wave_prod(double x) {
  // butterfly; IEEE products commute exactly, so every lane gets the same bits
  for (int o = 32; o > 0; o >>= 1) x *= __shfl_xor(x, o, 64);
  return x;
}

// Plane rotation (c, s) with c x - s y = r, s x + c y = 0 for the pair (x, y):
// r = |(x, y)| by one reciprocal square root where x^2 + y^2 is safely in
// range, else by hypot.
__device__ __forceinline__ void givens(double x, double y, double& c, double& sn, double& r) {
  const double t = x * x + y * y;
  if (t > 1e-290 && t < 1e290) {
    const double q = rsqrt(t);
    c = x * q;
    sn = -y * q;
    r = t * q;
  } else if (x == 0.0 && y == 0.0) {
    c = 1.0;
    sn = 0.0;
    r = 0.0;
  } else {
    r = hypot(x, y);
    c = x / r;
    sn = -y / r;
  }
}

// Leaves: one wave each.  Lane i holds d_i and e_i (e_i = T[i][i+1]) in
// registers; the sweep's scalar chain reads them with readlane and runs
// identically in every lane, and each rotation is kept in lane k's registers.
// The rotations are then applied to the leaf's eigenvector matrix in LDS, lane
// r owning row r (Z[r][c] = component r of eigenvector c).
__global__ __launch_bounds__(64) void k_tdc_leaf(TdcArgs a, int T, double* Zt) {
  __shared__ double Z[kLeaf][kLeaf + 1];
  const int n = a.n, lane = threadIdx.x;
  const int lo = cut(n, T, blockIdx.x), hi = cut(n, T, blockIdx.x + 1), s = hi - lo;
  double dv = 0.0, ev = 0.0;
  if (lane < s) {
    dv = a.d[lo + lane];
    if (lane == 0 && lo > 0) dv -= fabs(a.e[lo - 1]);        // tearing corrections
    if (lane == s - 1 && hi < n) dv -= fabs(a.e[hi - 1]);
    ev = lane + 1 < s ? a.e[lo + lane] : 0.0;
    for (int c = 0; c < s; ++c) Z[lane][c] = lane == c ? 1.0 : 0.0;
  }
  __syncthreads();
  double cv = 0.0, sv = 0.0;
  int h = s - 1, iters = 0;
  bool bad = false;
  while (h > 0) {
    // couplings negligible against their diagonal neighbours, below h
    const double dn = __shfl_down(dv, 1, 64);
    const bool small = fabs(ev) <= kEps * (fabs(dv) + fabs(dn));
    const unsigned long long msk = __ballot(small) & ((1ull << h) - 1ull);
    if ((msk >> (h - 1)) & 1ull) {
      if (lane == h - 1) ev = 0.0;
      --h;
      continue;
    }
    if (++iters > 30 * s) {   // also ends a NaN-filled leaf
      bad = true;
      break;
    }
    const int l = msk ? 64 - __clzll(msk) : 0;   // the unreduced block is [l, h]
    // Wilkinson shift: the eigenvalue of the trailing 2x2 nearer d_h
    const double dh = lane_value(dv, h), bh = lane_value(ev, h - 1);
    const double dd = 0.5 * (lane_value(dv, h - 1) - dh);
    const double mu = dh - bh * (bh / (dd + copysign(hypot(dd, bh), dd)));
    double dcur = lane_value(dv, l), ecur = lane_value(ev, l);
    double x = dcur - mu, y = ecur;
    for (int k = l; k < h; ++k) {
      // rotation on (k, k+1): first column along (x, y) at k = l, else chosen
      // to clear the bulge at (k-1, k+1)
      const double c0 = lane_value(dv, k + 1), e1 = k + 1 < h ? lane_value(ev, k + 1) : 0.0;
      double c, sn, r;
      givens(x, y, c, sn, r);
      const double a0 = dcur, b0 = ecur, cs = c * sn;
      const double nk = a0 * c * c - 2.0 * b0 * cs + c0 * sn * sn;
      const double nk1 = a0 * sn * sn + 2.0 * b0 * cs + c0 * c * c;
      const double ne = (a0 - c0) * cs + b0 * (c * c - sn * sn);
      if (lane == k) { dv = nk; cv = c; sv = sn; }
      if (k > l && lane == k - 1) ev = r;
      if (k + 1 < h) {
        y = -sn * e1;            // new bulge at (k, k+2)
        ecur = c * e1;
        x = ne;
        dcur = nk1;
      } else {
        if (lane == k) ev = ne;
        if (lane == k + 1) dv = nk1;
      }
    }
    if (lane < s) {
      double carry = Z[lane][l];
      for (int k = l; k < h; ++k) {
        const double c = lane_value(cv, k), sn = lane_value(sv, k), z1 = Z[lane][k + 1];
        Z[lane][k] = c * carry - sn * z1;
        carry = sn * carry + c * z1;
      }
      Z[lane][h] = carry;
    }
  }
  if (bad && lane == 0) atomicExch(a.err, 1);
  // ascending order: lane i's rank (ties by index)
  int rank = 0;
  for (int j = 0; j < s; ++j) {
    const double dj = lane_value(dv, j);
    rank += (dj < dv || (dj == dv && j < lane)) ? 1 : 0;
  }
  rank = min(rank, s - 1);   // NaN: keep the write in range
  if (lane < s) {
    a.d[lo + rank] = dv;
    for (int c = 0; c < s; ++c) {
      const int rc = __builtin_amdgcn_readlane(rank, c);
      Zt[(long)(lo + rc) * n + lo + lane] = Z[lane][c];
    }
  }
}

// Order-preserving compaction over the workgroup: out[0..count) = the j < s
// with pred(j), ascending; returns count (same in every thread).  Ends with
// a barrier.
template <class Pred>
__device__ int block_compact(int s, Pred pred, int* out, int* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int total = 0;
  for (int base = 0; base < s; base += 256) {
    const int j = base + tid;
    const bool f = j < s && pred(j);
    const unsigned long long b = __ballot(f);
    const int before = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(b);
    __syncthreads();
    int off = total;
    for (int v = 0; v < w; ++v) off += wsum[v];
    if (f) out[off + before] = j;
    total += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  return total;
}

// Merge steps 1-2 for every merge of level t: one workgroup each.
__global__ __launch_bounds__(256) void k_tdc_deflate(TdcArgs a, int t, const double* __restrict__ Zt) {
  extern __shared__ double sm[];
  const int n = a.n, tid = threadIdx.x;
  const long p = blockIdx.x;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), m = cut(n, t + 1, 2 * p + 1);
  const int s = hi - lo, n1 = m - lo;
  double* din = sm;                 // [s] the halves' eigenvalues (left, then right)
  double* sd = din + s;             // [s] sorted poles
  double* sz = sd + s;              // [s] sorted z
  int* src = (int*)(sz + s);        // [s] source row of sorted entry
  int* cand = src + s;              // [s] entries with z above tol (sorted index)
  int* nd = cand + s;               // [s] survivors (sorted index)
  int* df = nd + s;                 // [s] deflated (sorted index)
  __shared__ double red[256];
  __shared__ int wsum[4], cnt[3];
  const double ev = a.e[m - 1];
  const double beta = fabs(ev), sg = ev < 0.0 ? -1.0 : 1.0;
  const double rho = 2.0 * beta, rs2 = 0.70710678118654752440;   // 1/sqrt(2)
  double mx = 0.0;
  for (int i = tid; i < s; i += 256) {
    const double x = a.d[lo + i];
    din[i] = x;
    mx = fmax(mx, fabs(x));
    sd[i] = 0.0;   // every slot valid even if two ranks collided
    sz[i] = 0.0;
    src[i] = i;
  }
  red[tid] = mx;
  __syncthreads();
  // sorted position: left entries before equal right ones
  for (int i = tid; i < s; i += 256) {
    const double x = din[i];
    double z;
    int r;
    if (i < n1) {
      z = Zt[(long)(lo + i) * n + (m - 1)] * rs2;
      int l0 = n1, l1 = s;           // right entries < x
      while (l0 < l1) {
        const int md = (l0 + l1) >> 1;
        if (din[md] < x) l0 = md + 1; else l1 = md;
      }
      r = i + (l0 - n1);
    } else {
      z = sg * Zt[(long)(lo + i) * n + m] * rs2;
      int l0 = 0, l1 = n1;           // left entries <= x
      while (l0 < l1) {
        const int md = (l0 + l1) >> 1;
        if (din[md] <= x) l0 = md + 1; else l1 = md;
      }
      r = (i - n1) + l0;
    }
    r = min(max(r, 0), s - 1);       // NaN input: keep the write in range
    sd[r] = x;
    sz[r] = z;
    src[r] = i;
  }
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double tol = 8.0 * kEps * fmax(red[0], rho);
  // entries whose z is negligible deflate as they are; of the others, a pair
  // of neighbours deflates by a rotation when its coupling is negligible
  const int nc = block_compact(s, [&](int j) { return !(rho * fabs(sz[j]) <= tol); }, cand, wsum);
  bool hit = false;
  for (int i = tid; i + 1 < nc; i += 256) {
    const int pv = cand[i], j = cand[i + 1];
    const double zp = sz[pv], zj = sz[j];
    hit = hit || fabs(zp * zj * (sd[pv] - sd[j])) <= tol * (zp * zp + zj * zj);
  }
  const bool any = __syncthreads_or(hit);
  if (!any) {
    // no rotation: survivors are the candidates, the deflated entries keep
    // their sorted order
    const int nm = block_compact(s, [&](int j) { return rho * fabs(sz[j]) <= tol; }, df, wsum);
    for (int i = tid; i < nc; i += 256) {
      const int j = cand[i];
      a.dk[lo + i] = sd[j];
      a.zk[lo + i] = sz[j];
      a.ndrow[lo + i] = src[j];
    }
    for (int u = tid; u < nm; u += 256) {
      a.dvs[lo + u] = sd[df[u]];
      a.dvrow[lo + u] = src[df[u]];
    }
    if (tid == 0) {
      a.kcnt[lo] = nc;
      a.nrot[lo] = 0;
      a.rho[lo] = rho;
    }
    return;
  }
  if (tid == 0) {   // sequential scan: each rotation changes the next pair's test
    int k = 0, nm = 0, nr = 0, pv = -1;
    for (int j = 0; j < s; ++j) {
      const double zj = sz[j];
      if (rho * fabs(zj) <= tol) { df[nm++] = j; continue; }
      if (pv < 0) { pv = j; continue; }
      const double zp = sz[pv], dp = sd[pv], dj = sd[j];
      const double r2 = zp * zp + zj * zj;
      if (fabs(zp * zj * (dp - dj)) <= tol * r2) {
        const double r = sqrt(r2), c = zj / r, sn = zp / r;
        sd[pv] = c * c * dp + sn * sn * dj;
        sd[j] = sn * sn * dp + c * c * dj;
        sz[pv] = 0.0;
        sz[j] = r;
        a.rp[lo + nr] = src[pv];
        a.rj[lo + nr] = src[j];
        a.rc[lo + nr] = c;
        a.rs[lo + nr] = sn;
        ++nr;
        df[nm++] = pv;
      } else {
        nd[k++] = pv;
      }
      pv = j;
    }
    if (pv >= 0) nd[k++] = pv;
    cnt[0] = k;
    cnt[1] = nm;
    a.kcnt[lo] = k;
    a.nrot[lo] = nr;
    a.rho[lo] = rho;
  }
  __syncthreads();
  const int k = cnt[0], nm = cnt[1];
  for (int i = tid; i < k; i += 256) {
    const int j = nd[i];
    a.dk[lo + i] = sd[j];
    a.zk[lo + i] = sz[j];
    a.ndrow[lo + i] = src[j];
  }
  // deflated values in ascending order (rank sort, ties by scan order)
  double* dv = din;
  for (int u = tid; u < nm; u += 256) dv[u] = sd[df[u]];
  __syncthreads();
  for (int u = tid; u < nm; u += 256) {
    const double x = dv[u];
    int r = 0;
    for (int v = 0; v < nm; ++v) r += (dv[v] < x || (dv[v] == x && v < u)) ? 1 : 0;
    r = min(r, nm - 1);
    a.dvs[lo + r] = x;
    a.dvrow[lo + r] = src[df[u]];
  }
}

// The secular function at tau from origin pole o, split at the gap's left
// pole i: psi over the poles j <= i, phi over j > i, their derivatives, and
// sum |terms| for the rounding bound; every lane gets the same values.
struct Secular {
  double g, psi, phi, dpsi, dphi, sabs;
};
constexpr int kRootRegs = 8;   // up to 512 survivors held in registers
__device__ __forceinline__ void secular_term(double dj, double z2, int j, int i, double dorg, double tau, double& ps,
                                             double& ph, double& dps, double& dph, double& sa) {
  const double dl = (dj - dorg) - tau, r = 1.0 / dl, tt = z2 * r;
  if (j <= i) { ps += tt; dps += tt * r; } else { ph += tt; dph += tt * r; }
  sa += fabs(tt);
}
__device__ __forceinline__ Secular secular_finish(double ps, double ph, double dps, double dph, double sa,
                                                  double rho) {
  Secular f;
  f.psi = rho * wave_sum_dpp(ps);
  f.phi = rho * wave_sum_dpp(ph);
  f.dpsi = rho * wave_sum_dpp(dps);
  f.dphi = rho * wave_sum_dpp(dph);
  f.sabs = rho * wave_sum_dpp(sa);
  f.g = 1.0 + (f.psi + f.phi);
  return f;
}

// Merge step 3: one wave per root; the merge's poles and z in LDS, and in
// registers when there are at most 512.  Each root starts at the end of its
// half-gap bracket and takes steps of the two-pole model of f (the poles
// beside the gap carry the weight that matches f and f' at the current
// point), kept inside a bracket that every evaluation narrows; a step that
// would leave the bracket, and every step after the twelfth, is a bisection
// of the bracket's bit patterns instead.  It stops when |f| is within its
// rounding bound or the bracket is one ulp wide.
__global__ __launch_bounds__(256) void k_tdc_roots(TdcArgs a, int t) {
  extern __shared__ double sm[];
  const int n = a.n, tid = threadIdx.x, lane = tid & 63;
  const long p = blockIdx.y;
  const int lo = cut(n, t, p);
  const int k = a.kcnt[lo];
  if ((int)blockIdx.x * 4 >= k) return;
  double* dk = sm;
  double* zk = sm + k;
  for (int j = tid; j < k; j += 256) {
    dk[j] = a.dk[lo + j];
    zk[j] = a.zk[lo + j];
  }
  __syncthreads();
  const int i = blockIdx.x * 4 + (tid >> 6);
  if (i >= k) return;
  const bool in_regs = k <= 64 * kRootRegs;
  double dq[kRootRegs], zq[kRootRegs];
#pragma unroll
  for (int q = 0; q < kRootRegs; ++q) {
    const int j = lane + 64 * q;
    dq[q] = j < k ? dk[j] : 0.0;
    zq[q] = j < k ? zk[j] * zk[j] : 0.0;
  }
  const double rho = a.rho[lo];
  auto f = [&](int o, double tau) {
    const double dorg = dk[o];
    double ps = 0.0, ph = 0.0, dps = 0.0, dph = 0.0, sa = 0.0;
    if (in_regs) {
#pragma unroll
      for (int q = 0; q < kRootRegs; ++q)
        if (lane + 64 * q < k) secular_term(dq[q], zq[q], lane + 64 * q, i, dorg, tau, ps, ph, dps, dph, sa);
    } else {
      for (int j = lane; j < k; j += 64) secular_term(dk[j], zk[j] * zk[j], j, i, dorg, tau, ps, ph, dps, dph, sa);
    }
    return secular_finish(ps, ph, dps, dph, sa, rho);
  };
  // origin: the pole nearer the root (the sign of f at the gap's midpoint)
  int o = i;
  double sgn = 1.0, thi;
  const bool last = i + 1 == k;
  if (!last) {
    thi = 0.5 * (dk[i + 1] - dk[i]);
    if (!(f(i, thi).g >= 0.0)) {
      o = i + 1;
      sgn = -1.0;
    }
  } else {
    double s2 = 0.0;
    for (int j = lane; j < k; j += 64) s2 += zk[j] * zk[j];
    thi = rho * wave_sum_dpp(s2);
  }
  // tau = sgn t; the root's t lies in (tlo, thi]
  const double dl0 = dk[i] - dk[o], dr0 = last ? 0.0 : dk[i + 1] - dk[o];
  const double tol = kEps * (double)(k + 4);
  double tlo = 0.0, tt = thi;
  bool done = false;
  for (int it = 0; it < 96 && !done; ++it) {
    const double tau = sgn * tt;
    const Secular v = f(o, tau);
    if ((v.g < 0.0) == (sgn > 0.0)) tlo = tt; else thi = tt;
    const long long lb = __double_as_longlong(tlo), hb = __double_as_longlong(thi);
    if (fabs(v.g) <= tol * (1.0 + v.sabs)) { done = true; break; }
    if (hb - lb <= 1) { tt = thi; break; }
    double tn = -1.0;   // the model's step, if it stays inside the bracket
    if (it < 12) {
      const double DL = dl0 - tau;
      const double b1 = DL * DL * v.dpsi, a1 = v.psi - DL * v.dpsi;
      if (!last) {
        const double DR = dr0 - tau;
        const double b2 = DR * DR * v.dphi, a2 = v.phi - DR * v.dphi;
        const double A = 1.0 + (a1 + a2), B = A * (DL + DR) + (b1 + b2), C = DL * DR * v.g;
        const double disc = B * B - 4.0 * A * C;
        if (disc >= 0.0 && A != 0.0) {
          const double q = 0.5 * (B + copysign(sqrt(disc), B));
          const double x1 = q / A, x2 = q != 0.0 ? C / q : x1;
          const double t1 = sgn * (tau + x1), t2 = sgn * (tau + x2);
          if (tlo < t1 && t1 < thi) tn = t1;
          else if (tlo < t2 && t2 < thi) tn = t2;
        }
      } else {
        const double A = 1.0 + a1;
        if (A > 0.0) {
          const double t1 = sgn * (tau + DL + b1 / A);
          if (tlo < t1 && t1 < thi) tn = t1;
        }
      }
    }
    tt = tn > 0.0 ? tn : __longlong_as_double(lb + ((hb - lb) >> 1));
  }
  if (lane == 0) {
    a.org[lo + i] = o;
    a.tau[lo + i] = sgn * tt;
  }
}

// Merge step 4: zh_j by the product formula, one wave per survivor.
__global__ __launch_bounds__(256) void k_tdc_zhat(TdcArgs a, int t) {
  extern __shared__ double sm[];
  const int n = a.n, tid = threadIdx.x, lane = tid & 63;
  const long p = blockIdx.y;
  const int lo = cut(n, t, p);
  const int k = a.kcnt[lo];
  if ((int)blockIdx.x * 4 >= k) return;
  double* dk = sm;
  double* lo_d = sm + k;   // dk[org_i]
  double* tu = sm + 2 * k;
  for (int j = tid; j < k; j += 256) {
    dk[j] = a.dk[lo + j];
    tu[j] = a.tau[lo + j];
  }
  __syncthreads();
  for (int j = tid; j < k; j += 256) lo_d[j] = dk[a.org[lo + j]];
  __syncthreads();
  const int j = blockIdx.x * 4 + (tid >> 6);
  if (j >= k) return;
  const double rho = a.rho[lo], dj = dk[j];
  double pr = 1.0;
  for (int i = lane; i < k; i += 64) {
    const double num = (lo_d[i] - dj) + tu[i];   // lambda_i - d_j
    pr *= i == j ? num / rho : num / (dk[i] - dj);
  }
  pr = wave_prod(pr);
  if (lane == 0) a.zh[lo + j] = copysign(sqrt(fmax(pr, 0.0)), a.zk[lo + j]);
}

// Merge step 5a: norms of the u_i and every eigenvalue's output position,
// one wave per entry (root i < k, then deflated t = w - k).
__global__ __launch_bounds__(256) void k_tdc_place(TdcArgs a, int t) {
  extern __shared__ double sm[];
  const int n = a.n, tid = threadIdx.x, lane = tid & 63;
  const long p = blockIdx.y;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), s = hi - lo;
  if ((int)blockIdx.x * 4 >= s) return;
  const int k = a.kcnt[lo], nm = s - k;
  double* dk = sm;
  double* zh = sm + k;
  double* lam = sm + 2 * k;
  for (int j = tid; j < k; j += 256) {
    dk[j] = a.dk[lo + j];
    zh[j] = a.zh[lo + j];
  }
  __syncthreads();
  for (int j = tid; j < k; j += 256) lam[j] = dk[a.org[lo + j]] + a.tau[lo + j];
  __syncthreads();
  const int w = blockIdx.x * 4 + (tid >> 6);
  if (w >= s) return;
  const double* dvs = a.dvs + lo;
  if (w < k) {
    const int i = w;
    const double dorg = dk[a.org[lo + i]], ti = a.tau[lo + i];
    double s2 = 0.0;
    for (int j = lane; j < k; j += 64) {
      const double u = zh[j] / ((dk[j] - dorg) - ti);
      s2 += u * u;
    }
    const double nrm = sqrt(wave_sum_dpp(s2));
    const double li = lam[i];
    int l0 = 0, l1 = nm;   // deflated values < lambda_i
    while (l0 < l1) {
      const int md = (l0 + l1) >> 1;
      if (dvs[md] < li) l0 = md + 1; else l1 = md;
    }
    const int pos = min(i + l0, s - 1);
    if (lane == 0) {
      a.invn[lo + i] = 1.0 / nrm;
      a.d[lo + pos] = li;
      a.colsrc[lo + pos] = i;
    }
  } else {
    const int u = w - k;
    const double x = dvs[u];
    int l0 = 0, l1 = k;    // roots <= x
    while (l0 < l1) {
      const int md = (l0 + l1) >> 1;
      if (lam[md] <= x) l0 = md + 1; else l1 = md;
    }
    const int pos = min(u + l0, s - 1);
    if (lane == 0) {
      a.d[lo + pos] = x;
      a.colsrc[lo + pos] = -(u + 1);
    }
  }
}

// Merge step 5b: B = P U, one wave per row (survivor j < k, then deflated).
__global__ __launch_bounds__(256) void k_tdc_bmat(TdcArgs a, int t) {
  const int n = a.n, tid = threadIdx.x, lane = tid & 63;
  const long p = blockIdx.y;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), s = hi - lo;
  const int w = blockIdx.x * 4 + (tid >> 6);
  if (w >= s) return;
  const int k = a.kcnt[lo];
  double* B = a.B + (long)lo * n + lo;
  if (w < k) {
    const double zj = a.zh[lo + w], dj = a.dk[lo + w];
    double* row = B + (long)min(max(a.ndrow[lo + w], 0), s - 1) * n;   // (clamp: a source row)
    for (int c = lane; c < s; c += 64) {
      const int i = a.colsrc[lo + c];
      double v = 0.0;
      if (i >= 0 && i < k) v = zj / ((dj - a.dk[lo + a.org[lo + i]]) - a.tau[lo + i]) * a.invn[lo + i];
      row[c] = v;
    }
  } else {
    const int u = w - k;
    double* row = B + (long)min(max(a.dvrow[lo + u], 0), s - 1) * n;
    for (int c = lane; c < s; c += 64) row[c] = a.colsrc[lo + c] == -(u + 1) ? 1.0 : 0.0;
  }
}

// Merge step 5c: the deflation rotations on the rows of B, last first; one
// thread per column.
__global__ __launch_bounds__(256) void k_tdc_rot(TdcArgs a, int t) {
  const int n = a.n;
  const long p = blockIdx.y;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), s = hi - lo;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int nr = a.nrot[lo];
  if (c >= s || nr == 0) return;
  double* B = a.B + (long)lo * n + lo + c;
  for (int r = nr - 1; r >= 0; --r) {
    double* pa = B + (long)a.rp[lo + r] * n;
    double* pb = B + (long)a.rj[lo + r] * n;
    const double cs = a.rc[lo + r], sn = a.rs[lo + r];
    const double xa = *pa, xb = *pb;
    *pa = cs * xa + sn * xb;
    *pb = -sn * xa + cs * xb;
  }
}

// Merge step 5d, every merge of level t in one launch: Zt_new = B^T Zt on
// the merge's diagonal block, 32 x 32 output tiles on the FP64 MFMA engine.
// Rows x < n1 of Zt's block (the left half's eigenvectors) are zero in
// columns >= n1 and the right half's rows in columns < n1, so a tile whose
// columns lie on one side runs over that half's rows only.
using E64 = EngineOf<kF64>::type;
using TdcTile = TileCfg<32, 32, 16, 16, 16>;
__global__ __launch_bounds__(TdcTile::NT) void k_tdc_gemm(int n, int t, const double* __restrict__ B,
                                                          const double* __restrict__ Zt, double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<E64, TdcTile>()];
  const long p = blockIdx.y;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), m = cut(n, t + 1, 2 * p + 1);
  const int s = hi - lo, n1 = m - lo;
  const int nt = (s + TdcTile::BM - 1) / TdcTile::BM;
  if ((int)blockIdx.x >= nt * nt) return;
  const int c0 = ((int)blockIdx.x % nt) * TdcTile::BM, r0 = ((int)blockIdx.x / nt) * TdcTile::BN;
  int k0 = 0, k1 = s;
  if (r0 + TdcTile::BN <= n1) k1 = n1;
  else if (r0 >= n1) k0 = n1;
  const int K = k1 - k0;
  const long base = (long)(lo + k0) * n + lo;
  XCSrc<double, TdcTile::BM, E64::BK, TdcTile::NT, E64::KV> la;
  la.init(B + base, n, K, [&](int x, long& o) { o = c0 + x; return c0 + x < s; });
  XCSrc<double, TdcTile::BN, E64::BK, TdcTile::NT, E64::KV> lb;
  lb.init(Zt + base, n, K, [&](int x, long& o) { o = r0 + x; return r0 + x < s; });
  typename E64::template Acc<TdcTile> acc;
  gemm_mainloop<E64, TdcTile>(la, lb, (K + E64::BK - 1) / E64::BK, acc, smem);
  acc.for_each([&](int mm, int nn, double v) {
    if (c0 + mm < s && r0 + nn < s) out[(long)(lo + c0 + mm) * n + lo + r0 + nn] = v;
  });
}

// Both eigenvector arrays to zero; workgroup 0 also checks T: a non-finite
// entry sets the error flag and T to zero, so that every later step works on
// finite values (the call then reports the failure).
__global__ __launch_bounds__(256) void k_tdc_zero(long count, double* x, double* y, int n, double* d, double* e,
                                                  int* err) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
    x[i] = 0.0;
    y[i] = 0.0;
  }
  if (blockIdx.x != 0) return;
  bool bad = false;
  for (int i = threadIdx.x; i < n; i += 256) {
    bad = bad || !isfinite(d[i]);
    if (i + 1 < n) bad = bad || !isfinite(e[i]);
  }
  bad = __syncthreads_or(bad);
  if (bad)
    for (int i = threadIdx.x; i < n; i += 256) {
      d[i] = 0.0;
      if (i + 1 < n) e[i] = 0.0;
    }
  if (threadIdx.x == 0) *err = bad ? 1 : 0;
}

size_t deflate_lds(int s) { return (size_t)s * (3 * sizeof(double) + 4 * sizeof(int)); }
}  // namespace

size_t tdc_scratch_bytes(int n) {   // B, then 9 double and 8 int arrays of n
  return (size_t)n * n * sizeof(double) + 9 * (size_t)n * sizeof(double) + 8 * (size_t)n * sizeof(int);
}
int tdc_max_n() { return kTdcMaxN; }

rif_status op_tdc(rif_ctx* c, int n, double* d, double* e, double* Z0, double* Z1, void* scratch, int* err) {
  if (n < 2 || n > kTdcMaxN) return fail(c, RIF_ENOTSUP, "tridiagonal divide and conquer: n outside [2, 2048]");
  TdcArgs a{};
  a.n = n;
  a.d = d;
  a.e = e;
  char* s = (char*)scratch;
  auto take = [&](size_t bytes) {
    char* q = s;
    s += bytes;
    return q;
  };
  const size_t dn = (size_t)n * sizeof(double), in_ = (size_t)n * sizeof(int);
  a.B = (double*)take((size_t)n * dn);
  a.rho = (double*)take(dn);
  a.dk = (double*)take(dn);
  a.zk = (double*)take(dn);
  a.dvs = (double*)take(dn);
  a.rc = (double*)take(dn);
  a.rs = (double*)take(dn);
  a.tau = (double*)take(dn);
  a.zh = (double*)take(dn);
  a.invn = (double*)take(dn);
  a.kcnt = (int*)take(in_);
  a.nrot = (int*)take(in_);
  a.ndrow = (int*)take(in_);
  a.dvrow = (int*)take(in_);
  a.rp = (int*)take(in_);
  a.rj = (int*)take(in_);
  a.org = (int*)take(in_);
  a.colsrc = (int*)take(in_);
  a.err = err;
  const int T = tdc_levels(n);
  double* cur = (T % 2 == 0) ? Z0 : Z1;   // the last level writes Z0
  double* nxt = cur == Z0 ? Z1 : Z0;
  rif_status st;
  {
    const long cnt = (long)n * n;
    hipLaunchKernelGGL(k_tdc_zero, dim3((unsigned)std::min(1024L, (cnt + 255) / 256)), dim3(256), 0, c->stream, cnt,
                       Z0, Z1, n, d, e, a.err);
    if ((st = check_launch(c, "tdc_zero"))) return st;
    hipLaunchKernelGGL(k_tdc_leaf, dim3(1u << T), dim3(64), 0, c->stream, a, T, cur);
    if ((st = check_launch(c, "tdc_leaf"))) return st;
  }
  for (int t = T - 1; t >= 0; --t) {
    const int sm = tdc_smax(n, t), nmerge = 1 << t;
    const dim3 gw((unsigned)((sm + 3) / 4), (unsigned)nmerge);
    const size_t lds1 = deflate_lds(sm);
    if (lds1 > 64 * 1024) {
      const hipError_t he =
          hipFuncSetAttribute((const void*)k_tdc_deflate, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
      if (he != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, RIF_EHIP, std::string("divide and conquer: LDS attribute failed: ") + hipGetErrorString(he));
      }
    }
    hipLaunchKernelGGL(k_tdc_deflate, dim3((unsigned)nmerge), dim3(256), lds1, c->stream, a, t, (const double*)cur);
    if ((st = check_launch(c, "tdc_deflate"))) return st;
    hipLaunchKernelGGL(k_tdc_roots, gw, dim3(256), 2 * (size_t)sm * sizeof(double), c->stream, a, t);
    if ((st = check_launch(c, "tdc_roots"))) return st;
    hipLaunchKernelGGL(k_tdc_zhat, gw, dim3(256), 3 * (size_t)sm * sizeof(double), c->stream, a, t);
    if ((st = check_launch(c, "tdc_zhat"))) return st;
    hipLaunchKernelGGL(k_tdc_place, gw, dim3(256), 3 * (size_t)sm * sizeof(double), c->stream, a, t);
    if ((st = check_launch(c, "tdc_place"))) return st;
    hipLaunchKernelGGL(k_tdc_bmat, gw, dim3(256), 0, c->stream, a, t);
    if ((st = check_launch(c, "tdc_bmat"))) return st;
    hipLaunchKernelGGL(k_tdc_rot, dim3((unsigned)((sm + 255) / 256), (unsigned)nmerge), dim3(256), 0, c->stream, a,
                       t);
    if ((st = check_launch(c, "tdc_rot"))) return st;
    {
      const int nt = (sm + TdcTile::BM - 1) / TdcTile::BM;
      hipLaunchKernelGGL(k_tdc_gemm, dim3((unsigned)(nt * nt), (unsigned)nmerge), dim3(TdcTile::NT), 0, c->stream, n,
                         t, (const double*)a.B, (const double*)cur, nxt);
      if ((st = check_launch(c, "tdc_gemm"))) return st;
    }
    std::swap(cur, nxt);
  }
  return RIF_OK;   // cur == Z0
}

}  // namespace rif
