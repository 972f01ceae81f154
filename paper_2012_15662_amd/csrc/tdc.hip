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
// [floor(p n / 2^t), floor((p+1) n / 2^t))) down to leaves of at most 32 rows,
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
//    (D_j - D_o) - tau_i to high relative accuracy.  tau_i is found by
//    bisection on the bit pattern of |tau| (the order of positive doubles is
//    the order of their bits), which ends within one ulp in at most 64
//    evaluations of f whatever the scale of tau.
// 4. Gu-Eisenstat: the roots are exact eigenvalues of D + rho zh zh^T with
//      zh_j^2 = (lambda_j - D_j)/rho * prod_{i != j} (lambda_i - D_j)/(D_i - D_j)
//    (sign of z_j), and the eigenvectors are u_i = (zh_j / (D_j - lambda_i))_j
//    normalised; these are orthogonal to working precision.
// 5. Eigenvectors of T: Zh P R U, P the sort, R the deflation rotations, U
//    the u_i with unit columns for the deflated entries, columns in ascending
//    order of eigenvalue.  P and R are folded into the small matrix
//    B = P R U (rows of U permuted and rotated), and the product Zh B is one
//    FP64 MFMA GEMM per merge.
//
// Eigenvectors are kept as rows: Zt[c][r] = component r of eigenvector c, so
// that the merge product Zt_new = B^T Zt has both operands k-major for the
// engine's GEMM.  The two halves' blocks sit on the diagonal of an n x n
// array whose other entries are zero, which makes that block Zh^T itself.
// Every level runs as six launches covering all of its merges, plus the GEMMs.
#include <algorithm>
#include <string>

#include "rif_internal.hpp"
#include "wave.hpp"

namespace rif {

namespace {
constexpr int kLeaf = 32;
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
  int* err;            // set when a leaf's QR iteration fails to converge
};

__device__ __forceinline__ double wave_prod(double x) {
  // butterfly; IEEE products commute exactly, so every lane gets the same bits
  for (int o = 32; o > 0; o >>= 1) x *= __shfl_xor(x, o, 64);
  return x;
}

// Leaves: one wave each.  The scalar recurrence runs identically in every
// lane (every lane stores the same values), lane r owns row r of the leaf's
// eigenvector matrix Z (Z[r][c] = component r of eigenvector c).
__global__ __launch_bounds__(64) void k_tdc_leaf(TdcArgs a, int T, double* Zt) {
  __shared__ double sd[kLeaf], se[kLeaf], Z[kLeaf][kLeaf + 1];
  const int n = a.n, lane = threadIdx.x;
  const int lo = cut(n, T, blockIdx.x), hi = cut(n, T, blockIdx.x + 1), s = hi - lo;
  if (lane < s) {
    double x = a.d[lo + lane];
    if (lane == 0 && lo > 0) x -= fabs(a.e[lo - 1]);        // tearing corrections
    if (lane == s - 1 && hi < n) x -= fabs(a.e[hi - 1]);
    sd[lane] = x;
    se[lane] = lane + 1 < s ? a.e[lo + lane] : 0.0;
    for (int c = 0; c < s; ++c) Z[lane][c] = lane == c ? 1.0 : 0.0;
  }
  __syncthreads();
  int h = s - 1, iters = 0;
  bool bad = false;
  while (h > 0) {
    if (fabs(se[h - 1]) <= kEps * (fabs(sd[h - 1]) + fabs(sd[h]))) {
      se[h - 1] = 0.0;
      --h;
      continue;
    }
    if (++iters > 30 * s) {   // also ends a NaN-filled leaf
      bad = true;
      break;
    }
    int l = h - 1;
    while (l > 0 && fabs(se[l - 1]) > kEps * (fabs(sd[l - 1]) + fabs(sd[l]))) --l;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 nearer d_h
    const double dd = 0.5 * (sd[h - 1] - sd[h]), b = se[h - 1];
    const double mu = sd[h] - b * (b / (dd + copysign(hypot(dd, b), dd)));
    double x = sd[l] - mu, y = se[l];
    for (int k = l; k < h; ++k) {
      // rotation G on (k, k+1): first column along (x, y) at k = l, else
      // chosen to clear the bulge at (k-1, k+1)
      const double r = hypot(x, y);
      const double c = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : -y / r;
      const double a0 = sd[k], b0 = se[k], c0 = sd[k + 1];
      const double cs = c * sn;
      const double nk = a0 * c * c - 2.0 * b0 * cs + c0 * sn * sn;
      const double nk1 = a0 * sn * sn + 2.0 * b0 * cs + c0 * c * c;
      const double ne = (a0 - c0) * cs + b0 * (c * c - sn * sn);
      sd[k] = nk;
      sd[k + 1] = nk1;
      se[k] = ne;
      if (k > l) se[k - 1] = r;
      if (k + 1 < h) {
        const double e1 = se[k + 1];
        y = -sn * e1;            // new bulge at (k, k+2)
        se[k + 1] = c * e1;
        x = ne;
      }
      if (lane < s) {
        const double zk = Z[lane][k], zk1 = Z[lane][k + 1];
        Z[lane][k] = c * zk - sn * zk1;
        Z[lane][k + 1] = sn * zk + c * zk1;
      }
    }
  }
  if (bad && lane == 0) atomicExch(a.err, 1);
  // ascending order (selection sort, columns of Z along)
  for (int i = 0; i + 1 < s; ++i) {
    int mi = i;
    double mv = sd[i];
    for (int j = i + 1; j < s; ++j)
      if (sd[j] < mv) { mv = sd[j]; mi = j; }
    if (mi != i) {
      const double t = sd[i];
      sd[i] = mv;
      sd[mi] = t;
      if (lane < s) {
        const double u = Z[lane][i];
        Z[lane][i] = Z[lane][mi];
        Z[lane][mi] = u;
      }
    }
  }
  if (lane < s) {
    a.d[lo + lane] = sd[lane];
    for (int c = 0; c < s; ++c) Zt[(long)(lo + c) * n + lo + lane] = Z[lane][c];
  }
}

// Merge step 1-2 for every merge of level t: one workgroup each.
__global__ __launch_bounds__(256) void k_tdc_deflate(TdcArgs a, int t, const double* __restrict__ Zt) {
  extern __shared__ double sm[];
  const int n = a.n, tid = threadIdx.x;
  const long p = blockIdx.x;
  const int lo = cut(n, t, p), hi = cut(n, t, p + 1), m = cut(n, t + 1, 2 * p + 1);
  const int s = hi - lo, n1 = m - lo, n2 = hi - m;
  double* sd = sm;                  // [s] sorted poles
  double* sz = sd + s;              // [s] sorted z
  double* dv = sz + s;              // [s] deflated values (scan order)
  int* src = (int*)(dv + s);        // [s] source row of sorted entry
  int* nd = src + s;                // [s] survivors (sorted index)
  int* df = nd + s;                 // [s] deflated (sorted index)
  __shared__ double red[256];
  __shared__ int cnt[2];
  const double ev = a.e[m - 1];
  const double beta = fabs(ev), sg = ev < 0.0 ? -1.0 : 1.0;
  const double rho = 2.0 * beta, rs2 = 0.70710678118654752440;   // 1/sqrt(2)
  // sorted position: left entries before equal right ones
  for (int i = tid; i < s; i += 256) {
    double x, z;
    int r;
    if (i < n1) {
      x = a.d[lo + i];
      z = Zt[(long)(lo + i) * n + (m - 1)] * rs2;
      int l0 = 0, l1 = n2;           // count of right entries < x
      while (l0 < l1) {
        const int md = (l0 + l1) >> 1;
        if (a.d[m + md] < x) l0 = md + 1; else l1 = md;
      }
      r = i + l0;
    } else {
      const int j = i - n1;
      x = a.d[m + j];
      z = sg * Zt[(long)(m + j) * n + m] * rs2;
      int l0 = 0, l1 = n1;           // count of left entries <= x
      while (l0 < l1) {
        const int md = (l0 + l1) >> 1;
        if (a.d[lo + md] <= x) l0 = md + 1; else l1 = md;
      }
      r = j + l0;
    }
    r = min(max(r, 0), s - 1);       // NaN input: keep the write in range
    sd[r] = x;
    sz[r] = z;
    src[r] = i;
  }
  double mx = 0.0;
  for (int i = tid; i < s; i += 256) {
    const double v = i < n1 ? a.d[lo + i] : a.d[m + (i - n1)];
    mx = fmax(mx, fabs(v));
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double tol = 8.0 * kEps * fmax(red[0], rho);
  if (tid == 0) {
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
  for (int u = tid; u < nm; u += 256) dv[u] = sd[df[u]];
  __syncthreads();
  // deflated values in ascending order (rank sort, ties by scan order)
  for (int u = tid; u < nm; u += 256) {
    const double x = dv[u];
    int r = 0;
    for (int v = 0; v < nm; ++v) r += (dv[v] < x || (dv[v] == x && v < u)) ? 1 : 0;
    r = min(r, nm - 1);
    a.dvs[lo + r] = x;
    a.dvrow[lo + r] = src[df[u]];
  }
}

// f at tau from origin pole o (every lane gets the same value)
__device__ __forceinline__ double secular(const double* dk, const double* zk, int k, int o, double tau, double rho,
                                          int lane) {
  const double dorg = dk[o];
  double s = 0.0;
  for (int j = lane; j < k; j += 64) {
    const double z = zk[j];
    s += z * z / ((dk[j] - dorg) - tau);
  }
  return 1.0 + rho * wave_sum_dpp(s);
}

// Merge step 3: one wave per root; the merge's poles and z in LDS.
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
  const double rho = a.rho[lo];
  int o = i;
  double sgn = 1.0, hi;
  if (i + 1 < k) {
    const double gap = dk[i + 1] - dk[i];
    if (secular(dk, zk, k, i, 0.5 * gap, rho, lane) >= 0.0) {
      hi = 0.5 * gap;
    } else {
      o = i + 1;
      sgn = -1.0;
      hi = gap;
    }
  } else {
    double s2 = 0.0;
    for (int j = lane; j < k; j += 64) s2 += zk[j] * zk[j];
    hi = rho * wave_sum_dpp(s2);
  }
  // invariant: the root's |tau| lies in (lo, hi] in the order of bit patterns
  long long lb = 0, hb = __double_as_longlong(hi);
  while (hb - lb > 1) {
    const long long mb = lb + ((hb - lb) >> 1);
    const double tt = __longlong_as_double(mb);
    const double v = secular(dk, zk, k, o, sgn * tt, rho, lane);
    if ((v < 0.0) == (sgn > 0.0)) lb = mb; else hb = mb;
  }
  if (lane == 0) {
    a.org[lo + i] = o;
    a.tau[lo + i] = sgn * __longlong_as_double(hb);
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
    double* row = B + (long)a.ndrow[lo + w] * n;
    for (int c = lane; c < s; c += 64) {
      const int i = a.colsrc[lo + c];
      double v = 0.0;
      if (i >= 0) v = zj / ((dj - a.dk[lo + a.org[lo + i]]) - a.tau[lo + i]) * a.invn[lo + i];
      row[c] = v;
    }
  } else {
    const int u = w - k;
    double* row = B + (long)a.dvrow[lo + u] * n;
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

__global__ __launch_bounds__(256) void k_tdc_zero(long count, double* x, double* y, int* err) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
    x[i] = 0.0;
    y[i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

size_t deflate_lds(int s) { return (size_t)s * (3 * sizeof(double) + 3 * sizeof(int)); }
}  // namespace

size_t tdc_scratch_bytes(int n) {   // B, then 10 double and 9 int arrays of n
  return (size_t)n * n * sizeof(double) + 10 * (size_t)n * sizeof(double) + 9 * (size_t)n * sizeof(int);
}
int tdc_max_n() { return kTdcMaxN; }

rif_status op_tdc(rif_ctx* c, int n, double* d, const double* e, double* Z0, double* Z1, void* scratch, int* err) {
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
  take(dn);   // spare, keeps the int arrays 8-byte aligned
  a.kcnt = (int*)take(in_);
  a.nrot = (int*)take(in_);
  a.ndrow = (int*)take(in_);
  a.dvrow = (int*)take(in_);
  a.rp = (int*)take(in_);
  a.rj = (int*)take(in_);
  a.org = (int*)take(in_);
  a.colsrc = (int*)take(in_);
  take(in_);
  a.err = err;
  const int T = tdc_levels(n);
  double* cur = (T % 2 == 0) ? Z0 : Z1;   // the last level writes Z0
  double* nxt = cur == Z0 ? Z1 : Z0;
  rif_status st;
  {
    const long cnt = (long)n * n;
    hipLaunchKernelGGL(k_tdc_zero, dim3((unsigned)std::min(1024L, (cnt + 255) / 256)), dim3(256), 0, c->stream, cnt,
                       Z0, Z1, a.err);
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
    for (int q = 0; q < nmerge; ++q) {   // Zt_new = B^T Zt on the merge's diagonal block
      const int lo = cut(n, t, q), sz = cut(n, t, q + 1) - lo;
      const long off = (long)lo * n + lo;
      if ((st = op_gemm_kn(c, sz, sz, sz, a.B + off, n, cur + off, n, nxt + off, n))) return st;
    }
    std::swap(cur, nxt);
  }
  return RIF_OK;   // cur == Z0
}

}  // namespace rif
