// Rounding (Sec. 3) of the MPO that Algorithm 4.1 builds: the linear-algebra
// kernels.
//
// Once the selection cores 2..d are orthogonalised (an exact relabelling, done
// in kernels_sparse.hip), the rounding needs the truncated SVD of core 1, a
// tall panel P with I_1 J_1 rows and one column per nonzero block, and then of
// a chain of small panels.  P is factorised by TSQR: independent workgroups
// take the blocked Householder QR of row tiles ("leaves"), the R factors are
// stacked in pairs and factorised again up a binary tree, and the root R is
// diagonalised by one-sided Jacobi (Hestenes).  The kept left singular vectors
// are formed by applying the tree's reflectors top-down to those of R, so they
// are orthonormal to working accuracy however small the kept singular values
// are.  Each small panel is handled by one workgroup: Householder QR when it
// is taller than wide, Jacobi, reflector application, sign convention.
#include "tnrsvd_internal.h"
#include "wg_linalg.h"

namespace tnr {

namespace {

constexpr int AR = kSweepArena;
constexpr int RC = AR - 64 - 2 * QBMAX * QBMAX;   // LDS for the panel and the GEMM tiles

__device__ inline double* lds_Ts(double* a) { return a + AR - 32 - 2 * QBMAX * QBMAX; }
__device__ inline double* lds_Gs(double* a) { return a + AR - 32 - QBMAX * QBMAX; }
__device__ inline double* lds_red(double* a) { return a + AR - 16; }

__host__ __device__ inline int pick_qb(int64_t m) { return m * (QBMAX + 1) <= RC ? QBMAX : QB; }

// Householder QR (diag(R) >= 0) of the m x n column-major X (ld ld) in place.
// ws holds qr_ws_doubles(m, n): the blocked update's workspace, then m doubles
// for the reflector of an unblocked step when m exceeds the LDS (else LDS).
__device__ void wg_qr(double* X, int m, int n, int64_t ld, double* tau, double* ws, double* arena) {
  const int qb = pick_qb(m);
  double* v = m <= RC ? arena : ws + (int64_t)m * qb + 2 * (int64_t)qb * n;
  wg_geqrf(X, m, n, tau, v, lds_red(arena), ws, arena, RC, lds_Ts(arena), lds_Gs(arena), ld, qb);
}

// Y <- H_0 ... H_{k-1} Y for the m x s matrix Y with element (r, c) at
// Y[r ys + c], reflectors stored as by wg_geqr2 in V (ld ldv).  One wave per
// column of Y.
__device__ void wg_apply_q_rows(const double* V, const double* tau, int m, int k, double* Y, int s,
                                int64_t ldv, int64_t ys) {
  const int lane = threadIdx.x & 63, w = wave_id();
  for (int c = w; c < s; c += NW) {
    double* yc = Y + c;
    for (int j = k - 1; j >= 0; --j) {
      const double tj = tau[j];
      if (tj == 0.0) continue;
      const double* vj = V + (int64_t)j * ldv;
      const int r0 = j & ~63;
      double part = 0.0;
      for (int r = r0 + lane; r < m; r += 64) {
        if (r == j) part += yc[(int64_t)r * ys];
        else if (r > j) part += vj[r] * yc[(int64_t)r * ys];
      }
      part = wave_sum(part);
      const double f = tj * part;
      for (int r = r0 + lane; r < m; r += 64) {
        if (r == j) yc[(int64_t)r * ys] -= f;
        else if (r > j) yc[(int64_t)r * ys] -= f * vj[r];
      }
    }
  }
  __syncthreads();
}

// Smallest rank >= 1 whose discarded tail satisfies sum_{l >= rho} sig_l^2 <=
// delta^2 (sig descending, kk values), then capped at rmax (> 0) and at kk.
__device__ int tail_rank(const double* sig, int kk, double delta, int rmax) {
  const double d2 = delta * delta;
  double tail = 0.0;
  int rho = kk;
  for (int cand = kk - 1; cand >= 1; --cand) {
    tail += sig[cand] * sig[cand];
    if (tail <= d2)
      rho = cand;
    else
      break;
  }
  if (rmax > 0 && rho > rmax) rho = rmax;
  return rho < 1 ? 1 : rho;
}

// ------------------------------------------------------------------- TSQR

// Leaf l: QR of the h x N column-major tile l of Pw; R goes to the parent's
// 2N x N stack (rows (l & 1) N ..), or to the root (ld N) when there is one leaf.
__global__ __launch_bounds__(NT) void k_tsqr_leaf(double* Pw, int h, int N, double* tau,
                                                  double* ws, int64_t wss, double* up, int single) {
  __shared__ double arena[AR];
  const int l = blockIdx.x;
  double* X = Pw + (int64_t)l * h * N;
  wg_qr(X, h, N, h, tau + (int64_t)l * N, ws + (int64_t)l * wss, arena);
  double* S = single ? up : up + (int64_t)(l >> 1) * 2 * N * N + (l & 1) * N;
  const int64_t ls = single ? N : 2 * (int64_t)N;
  for (int64_t e = threadIdx.x; e < (int64_t)N * N; e += NT) {
    const int64_t c = e / N, r = e % N;
    S[c * ls + r] = r <= c ? X[c * h + r] : 0.0;
  }
}

// Tree node i of one level: QR of its stacked pair (2N x N, ld 2N); R to the
// parent's stack, or to the root when the level has one node.
__global__ __launch_bounds__(NT) void k_tsqr_node(double* S, int N, double* tau, double* ws,
                                                  int64_t wss, double* up, int single) {
  __shared__ double arena[AR];
  const int i = blockIdx.x;
  const int64_t m = 2 * (int64_t)N;
  double* X = S + (int64_t)i * m * N;
  wg_qr(X, (int)m, N, m, tau + (int64_t)i * N, ws + (int64_t)i * wss, arena);
  double* D = single ? up : up + (int64_t)(i >> 1) * m * N + (i & 1) * N;
  const int64_t ls = single ? N : m;
  for (int64_t e = threadIdx.x; e < (int64_t)N * N; e += NT) {
    const int64_t c = e / N, r = e % N;
    D[c * ls + r] = r <= c ? X[c * m + r] : 0.0;
  }
}

// SVD of the root R (N x N, column-major) by one-sided Jacobi on its rows:
// R = U diag(sig) V^T.  Rank by the tail rule with delta = eps |R|_F /
// sqrt(d - 1) (|R|_F = |A|_F), capped at rmax and min(n1, N).  Writes rho,
// delta, Y0 = U(:, kept) (N x rho, ld N) and T = diag(sig) V^T (rho x N,
// row-major).  Signs are fixed later on the full left vectors.
__global__ __launch_bounds__(NT) void k_root_svd(const double* Rf, int N, int64_t n1, double eps,
                                                 int dm1, int rmax, double* B, double* U,
                                                 double* nrm, double* sig, int* perm, int* flag,
                                                 double* Y0, double* T, int* rho_out,
                                                 double* delta_out) {
  __shared__ double red[16];
  __shared__ int srho;
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int64_t e = tid; e < (int64_t)N * N; e += NT) {
    const int64_t p = e / N, c = e % N;
    const double x = Rf[c * N + p];
    B[e] = x;                         // vector p = row p of R
    part += x * x;
  }
  const double nrm2 = block_sum(part, red);
  const double delta = eps * sqrt(nrm2) / sqrt((double)dm1);
  wg_jacobi(B, N, N, N, U, flag, red, delta * delta / (double)N);
  wg_norms_sorted(B, N, N, N, sig, perm, nrm);
  if (tid == 0) {
    const int kk = (int)(n1 < N ? n1 : N);
    srho = tail_rank(sig, kk, delta, rmax);
    rho_out[0] = srho;
    delta_out[0] = delta;
  }
  __syncthreads();
  const int rho = srho;
  for (int64_t e = tid; e < (int64_t)N * rho; e += NT) {
    const int64_t k = e / N, r = e % N;
    Y0[e] = U[(int64_t)perm[k] * N + r];
    T[k * N + r] = B[(int64_t)perm[k] * N + r];
  }
}

// Top-down application of a tree level: node i takes rows (i & 1) N .. of its
// parent's Y (2N x rho, ld 2N; Y0 with ld N at the root), pads them with N zero
// rows and applies its reflectors.
__global__ __launch_bounds__(NT) void k_tsqr_apply_node(const double* S, const double* tau, int N,
                                                        int rho, const double* Yup, int root,
                                                        double* Yl) {
  const int i = blockIdx.x;
  const int64_t m = 2 * (int64_t)N;
  const double* src = root ? Yup : Yup + (int64_t)(i >> 1) * m * rho + (i & 1) * N;
  const int64_t ls = root ? N : m;
  double* Y = Yl + (int64_t)i * m * rho;
  for (int64_t e = threadIdx.x; e < m * rho; e += NT) {
    const int64_t c = e / m, r = e % m;
    Y[e] = r < N ? src[c * ls + r] : 0.0;
  }
  __syncthreads();
  wg_apply_q(S + (int64_t)i * m * N, tau + (int64_t)i * N, (int)m, N, Y, rho, m);
}

// Leaf l: rows l h .. of core 1 (row-major n1 x rho) = the leaf's reflectors
// applied to [its rows of the parent's Y; 0].  Only the leaf's rows that exist
// (< n1) are touched: padding rows of P are zero, so no reflector reaches them.
__global__ __launch_bounds__(NT) void k_tsqr_apply_leaf(const double* Pw, const double* tau, int h,
                                                        int N, int rho, int64_t n1,
                                                        const double* Yup, int single,
                                                        double* core1) {
  const int l = blockIdx.x;
  const int64_t row0 = (int64_t)l * h;
  const int ml = (int)((n1 - row0) < h ? (n1 - row0) : h);
  const double* src = single ? Yup : Yup + (int64_t)(l >> 1) * 2 * N * rho + (l & 1) * N;
  const int64_t ls = single ? N : 2 * (int64_t)N;
  double* Y = core1 + row0 * rho;
  for (int64_t e = threadIdx.x; e < (int64_t)ml * rho; e += NT) {
    const int64_t r = e / rho, c = e % rho;
    Y[e] = r < N ? src[c * ls + r] : 0.0;
  }
  __syncthreads();
  wg_apply_q_rows(Pw + (int64_t)l * h * N, tau + (int64_t)l * N, ml, ml < N ? ml : N, Y, rho, h,
                  rho);
}

// Per chunk of 1024 rows and per column of the row-major n1 x rho matrix X:
// the largest magnitude and the first row holding it.
constexpr int kColChunk = 1024;
__global__ __launch_bounds__(NT) void k_colmax(const double* X, int64_t n1, int rho, double* pv,
                                               int64_t* pi) {
  const int lane = threadIdx.x & 63, w = wave_id();
  const int64_t r0 = (int64_t)blockIdx.x * kColChunk;
  const int64_t r1 = (r0 + kColChunk) < n1 ? (r0 + kColChunk) : n1;
  for (int c = w; c < rho; c += NW) {
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t r = r0 + lane; r < r1; r += 64) {
      const double a = fabs(X[r * rho + c]);
      if (a > best) {       // rows rise along a lane, so the first maximum is kept
        best = a;
        bi = r;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int64_t oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      pv[(int64_t)blockIdx.x * rho + c] = best;
      pi[(int64_t)blockIdx.x * rho + c] = bi;
    }
  }
}

// Sign of the largest-magnitude entry of every column (first row on ties),
// from the per-chunk maxima; sgn[c] = +-1.
__global__ __launch_bounds__(NT) void k_colsign(const double* X, int rho, const double* pv,
                                                const int64_t* pi, int nchunk, double* sgn) {
  for (int c = threadIdx.x; c < rho; c += NT) {
    double best = -1.0;
    int64_t bi = 0;
    for (int k = 0; k < nchunk; ++k) {
      const double v = pv[(int64_t)k * rho + c];
      if (v > best) {     // chunks in row order: a tie keeps the earlier row
        best = v;
        bi = pi[(int64_t)k * rho + c];
      }
    }
    sgn[c] = X[bi * rho + c] < 0.0 ? -1.0 : 1.0;
  }
}

// X (row-major n1 x rho) columns and T (rho x N) rows times sgn.
__global__ void k_apply_sign(double* X, int64_t n1, int rho, double* T, int N, const double* sgn) {
  const int64_t tot = n1 * rho, tt = (int64_t)rho * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot + tt;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < tot)
      X[e] *= sgn[e % rho];
    else
      T[e - tot] *= sgn[(e - tot) / N];
  }
}

// ------------------------------------------------------------ small panels

// Truncated SVD of the nv x q column-major panel M (rows: carried rank x
// mode, columns: the next bond): QR first when it is taller than wide, then
// one-sided Jacobi, rank by the tail rule, left vectors sign-fixed (largest-
// magnitude entry positive).  core = those vectors (row-major nv x rho), Tn =
// diag(sig) V^T with the same signs (row-major rho x q); *rho_out = rho.
__device__ void panel_svd(double* M, int64_t nv, int q, double delta, int rmax, double* ws,
                          double* tau, double* B, double* U, double* nrm, double* sig, int* perm,
                          double* sgn, int* flag, double* Y, double* core, double* Tn,
                          int* rho_out, double* arena, int* srho_s) {
  const int tid = threadIdx.x;
  int& srho = *srho_s;
  const bool tall = nv > q;
  const int nvv = tall ? q : (int)nv;   // Jacobi vectors: rows of R, or rows of M
  if (tall) {
    wg_qr(M, (int)nv, q, nv, tau, ws, arena);
    for (int64_t e = tid; e < (int64_t)q * q; e += NT) {
      const int64_t p = e / q, c = e % q;
      B[e] = c >= p ? M[c * nv + p] : 0.0;
    }
  } else {
    for (int64_t e = tid; e < nv * q; e += NT) {
      const int64_t p = e / q, c = e % q;
      B[e] = M[c * nv + p];
    }
  }
  __syncthreads();
  wg_jacobi(B, nvv, q, q, U, flag, lds_red(arena), delta * delta / (double)nvv);
  wg_norms_sorted(B, nvv, q, q, sig, perm, nrm);
  if (tid == 0) {
    const int kk = (int)(nv < q ? nv : q);
    srho = tail_rank(sig, kk, delta, rmax);
    rho_out[0] = srho;
  }
  __syncthreads();
  const int rho = srho;
  // left vectors, column-major nv x rho
  for (int64_t e = tid; e < nv * rho; e += NT) {
    const int64_t k = e / nv, r = e % nv;
    Y[e] = r < nvv ? U[(int64_t)perm[k] * nvv + r] : 0.0;
  }
  __syncthreads();
  if (tall) wg_apply_q(M, tau, (int)nv, q, Y, rho, nv);
  for (int k = tid; k < rho; k += NT) sgn[k] = sign_of_max(Y + (int64_t)k * nv, (int)nv, 1);
  __syncthreads();
  for (int64_t e = tid; e < nv * rho; e += NT) {
    const int64_t r = e / rho, k = e % rho;
    core[e] = Y[k * nv + r] * sgn[k];
  }
  for (int64_t e = tid; e < (int64_t)rho * q; e += NT) {
    const int64_t k = e / q, c = e % q;
    Tn[e] = B[(int64_t)perm[k] * q + c] * sgn[k];
  }
}

// One core k of the left-to-right truncation (1 < k < d).  T (rp x cp,
// row-major) is the carried factor; column c of it belongs to class c of the
// orthogonalised selection core, whose single unit entry sits at mode index
// pm[c] and right class nx[c] (an injective map, so the panel is a scatter):
//   M[(a n + pm[c]), nx[c]] = T[a, c],   M is (rp n) x q,
// then its truncated SVD (panel_svd).
__global__ __launch_bounds__(NT) void k_round_level(const double* T, int rp, int cp, const int* pm,
                                                    const int* nx, int n, int q,
                                                    const double* delta_p, int rmax, double* M,
                                                    double* ws, double* tau, double* B, double* U,
                                                    double* nrm, double* sig, int* perm,
                                                    double* sgn, int* flag, double* Y,
                                                    double* core, double* Tn, int* rho_out) {
  __shared__ double arena[AR];
  __shared__ int srho;
  const int tid = threadIdx.x;
  const int64_t nv = (int64_t)rp * n;
  const double delta = delta_p[0];
  for (int64_t e = tid; e < nv * q; e += NT) M[e] = 0.0;
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)rp * cp; e += NT) {
    const int64_t a = e / cp, c = e % cp;
    M[(int64_t)nx[c] * nv + a * n + pm[c]] = T[e];
  }
  __syncthreads();
  panel_svd(M, nv, q, delta, rmax, ws, tau, B, U, nrm, sig, perm, sgn, flag, Y, core, Tn, rho_out,
            arena, &srho);
}

// The last core: core[a n + pm[c]] = T[a, c] (row-major rp x n), zero elsewhere.
__global__ __launch_bounds__(NT) void k_round_last(const double* T, int rp, int cp, const int* pm,
                                                   int n, double* core) {
  for (int64_t e = threadIdx.x; e < (int64_t)rp * n; e += NT) core[e] = 0.0;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)rp * cp; e += NT) {
    const int64_t a = e / cp, c = e % cp;
    core[a * n + pm[c]] = T[e];
  }
}

// ------------------------------------------------- rounding of any MPO

// Z (m x s column-major, ld m) <- H_0 H_1 ... H_{k-1} Z for the reflectors
// stored as by wg_geqr2 in V (ld m), applied in blocks of QBMAX from the last
// one: a block is I - Vb T Vb^T (compact WY; T by the forward recurrence from
// Vb^T Vb, as in wg_geqrf), so each block costs three matrix-core GEMMs.
// ws holds m QBMAX + 2 QBMAX s doubles.
__device__ void wg_apply_q_blocked(const double* V, const double* tau, int m, int k, double* Z,
                                   int s, double* ws, double* arena) {
  const int tid = threadIdx.x;
  double* Ts = lds_Ts(arena);
  double* Gs = lds_Gs(arena);
  for (int j0 = ((k - 1) / QBMAX) * QBMAX; j0 >= 0; j0 -= QBMAX) {
    const int jb = (k - j0) < QBMAX ? (k - j0) : QBMAX, mp = m - j0;
    double* Vp = ws;                                   // explicit V (mp x jb, column-major)
    double* W = ws + (int64_t)mp * QBMAX;              // Vp^T Z (jb x s, row-major)
    double* W2 = W + (int64_t)QBMAX * s;               // T W
    for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
      const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
      Vp[e] = r > c ? V[(int64_t)(j0 + c) * m + j0 + r] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    wg_gemm<double>(jb, jb, mp, 1.0, Vp, mp, 1, Vp, 1, mp, 0.0, Gs, QBMAX, 1, arena);
    if (tid < 64) {
      for (int i = 0; i < jb; ++i) {
        const double ti = tau[j0 + i];
        if (tid < i) {
          double acc = 0.0;
          for (int c = tid; c < i; ++c) acc += Ts[tid * QBMAX + c] * Gs[c * QBMAX + i];
          Ts[tid * QBMAX + i] = -ti * acc;
        } else if (tid < QBMAX) {
          Ts[tid * QBMAX + i] = tid == i ? ti : 0.0;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    wg_gemm<double>(jb, s, mp, 1.0, Vp, mp, 1, Z + j0, 1, m, 0.0, W, s, 1, arena);
    wg_gemm<double>(jb, s, jb, 1.0, Ts, QBMAX, 1, W, s, 1, 0.0, W2, s, 1, arena);
    wg_gemm<double>(mp, s, jb, -1.0, Vp, 1, mp, W2, s, 1, 1.0, Z + j0, 1, m, arena);
  }
  __syncthreads();
}

// Right-to-left step at core k >= 1 of the rounding of a general MPO: the LQ
// of core k (r rows, m = n r' columns, row-major) as the QR with diag(R) >= 0
// of its transpose X (m x r column-major: the same memory), rk = min(m, r).
// X keeps the reflectors (the new core k is Q^T, rk x m, never formed: the
// left-to-right pass applies them); Gpo (pn x rk) = Gp (pn x r) R^T is the
// previous core with L = R^T absorbed.
__global__ __launch_bounds__(NT) void k_lq_absorb(const double* G, int r, int m, const double* Gp,
                                                  int pn, double* X, double* tau, double* ws,
                                                  double* Rt, double* Gpo) {
  __shared__ double arena[AR];
  const int tid = threadIdx.x;
  const int rk = m < r ? m : r;
  for (int64_t e = tid; e < (int64_t)m * r; e += NT) X[e] = G[e];
  __syncthreads();
  wg_qr(X, m, r, m, tau, ws, arena);
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)r * rk; e += NT) {   // Rt[b][c] = R[c][b]
    const int64_t b = e / rk, c = e % rk;
    Rt[e] = c <= b ? X[b * m + c] : 0.0;
  }
  __syncthreads();
  wg_gemm<double>(pn, rk, r, 1.0, Gp, r, 1, Rt, rk, 1, 0.0, Gpo, rk, 1, arena);
}

// |G|_F of the first core after the right-to-left pass (= |A|_F) and the
// truncation threshold delta = eps |A|_F / sqrt(d - 1): out[0] = delta, out[1] = |A|_F.
__global__ __launch_bounds__(NT) void k_norm_delta(const double* G, int64_t len, double eps,
                                                   int dm1, double* out) {
  __shared__ double red[NW];
  double part = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += NT) part += G[e] * G[e];
  const double nrm = sqrt(block_sum(part, red));
  if (threadIdx.x == 0) {
    out[0] = dm1 > 0 ? eps * nrm / sqrt((double)dm1) : 0.0;
    out[1] = nrm;
  }
}

// Left-to-right step at core 0: the panel M = core 0 (n x q, as (1 n) x q)
// times the 1 x 1 carried factor T, column-major, then its truncated SVD.
__global__ __launch_bounds__(NT) void k_round_first(const double* T, const double* G, int n, int q,
                                                    const double* delta_p, int rmax, double* M,
                                                    double* ws, double* tau, double* B, double* U,
                                                    double* nrm, double* sig, int* perm,
                                                    double* sgn, int* flag, double* Y,
                                                    double* core, double* Tn, int* rho_out) {
  __shared__ double arena[AR];
  __shared__ int srho;
  const double t = T[0];
  for (int64_t e = threadIdx.x; e < (int64_t)n * q; e += NT) {
    const int64_t i = e / q, c = e % q;
    M[c * n + i] = t * G[e];
  }
  __syncthreads();
  panel_svd(M, n, q, delta_p[0], rmax, ws, tau, B, U, nrm, sig, perm, sgn, flag, Y, core, Tn,
            rho_out, arena, &srho);
}

// Left-to-right step at core 0 < k < d - 1: the carried factor T (s x rk, s
// read from the device, where the previous step left it)
// times the orthogonalised core Q^T (rk x m, m = n q), formed as
// (Q [T^T; 0])^T with the stored reflectors, reshaped (s n) x q column-major,
// then its truncated SVD.
__global__ __launch_bounds__(NT) void k_round_step(const double* T, const int* s_dev, int rk, const double* X,
                                                   const double* tq, int m, int n, int q,
                                                   const double* delta_p, int rmax, double* Z,
                                                   double* wsq, double* M, double* ws, double* tau,
                                                   double* B, double* U, double* nrm, double* sig,
                                                   int* perm, double* sgn, int* flag, double* Y,
                                                   double* core, double* Tn, int* rho_out) {
  __shared__ double arena[AR];
  __shared__ int srho;
  const int s = s_dev[0];   // the rank the previous step kept
  const int64_t nv = (int64_t)s * n;
  for (int64_t e = threadIdx.x; e < (int64_t)m * s; e += NT) {
    const int64_t a = e / m, j = e % m;
    Z[e] = j < rk ? T[a * rk + j] : 0.0;
  }
  __syncthreads();
  wg_apply_q_blocked(X, tq, m, rk, Z, s, wsq, arena);
  for (int64_t e = threadIdx.x; e < nv * q; e += NT) {   // M[(a n + i), c] = Z[(i q + c), a]
    const int64_t p = e / q, c = e % q, a = p / n, i = p % n;
    M[c * nv + p] = Z[a * m + i * q + c];
  }
  __syncthreads();
  panel_svd(M, nv, q, delta_p[0], rmax, ws, tau, B, U, nrm, sig, perm, sgn, flag, Y, core, Tn,
            rho_out, arena, &srho);
}

// The last core takes the carried factor: out (s x n) = T (s x rk) Q^T, i.e.
// the column-major n x s matrix Q [T^T; 0], which has the same memory.
__global__ __launch_bounds__(NT) void k_round_last_q(const double* T, const int* s_dev, int rk,
                                                     const double* X, const double* tq, int n,
                                                     double* wsq, double* out) {
  __shared__ double arena[AR];
  const int s = s_dev[0];
  for (int64_t e = threadIdx.x; e < (int64_t)n * s; e += NT) {
    const int64_t a = e / n, j = e % n;
    out[e] = j < rk ? T[a * rk + j] : 0.0;
  }
  __syncthreads();
  wg_apply_q_blocked(X, tq, n, rk, out, s, wsq, arena);
}

// ------------------------------------------- sketched product truncation

// Randomize-then-orthogonalize (Al Daas, Ballard et al., SIAM J. Sci. Comput.
// 2023) applied to the pending product of MPO b (one workgroup): with a
// Gaussian chain S of bond ranks l_k = min(ell, P_k) drawn from the counter
// stream, the sketch environments W_k = Y_{>=k} S_{>=k}^T (P_k x l_k) are
// formed right to left; then, left to right, the panel (C Y_k) W_{k+1}
// ((s n) x l_{k+1}) is orthogonalised by Householder QR (diag(R) >= 0), its Q
// overwrites core k and Q^T (C Y_k) is carried; the last core takes C Y_{d-1}.
// The product ranks pr are lowered to the new ones.  Nothing is done when no
// bond rank exceeds ell.  Sketch entry (c, i, c') of core k (1 <= k <= d-2)
// is the normal number at counter cbase + o_k + (c n_k + i) ell + c', with
// o_k = sum over 1 <= j < k of ell n_j ell; on the last core (c, i, kappa)
// at cbase + o_{d-1} + c n K + i K + kappa.
template <typename T>
__global__ __launch_bounds__(NT) void k_sketch_pass(const MpoDesc* mpos, const CoreDesc* cores,
                                                    int op, int* pr, T* Z, int ell, uint64_t seed,
                                                    uint64_t cbase, const int* nm_d,
                                                    const int64_t* ws_off, double* wsb, int* err) {
  __shared__ double arena[AR];
  __shared__ int Pold[kSketchMaxD + 1];
  const int b = blockIdx.x, tid = threadIdx.x;
  const MpoDesc md = mpos[b];
  const int d = md.d, K = md.K, pc = md.pcap, nm = nm_d[b];
  if (d < 2) return;
  if (d > kSketchMaxD) {
    if (tid == 0) atomicOr(err, 4);
    return;
  }
  for (int k = tid; k <= d; k += NT) Pold[k] = pr[md.r0 + k];
  __syncthreads();
  int pmax = 0;
  for (int k = 1; k < d; ++k) pmax = Pold[k] > pmax ? Pold[k] : pmax;
  if (pmax <= ell) return;
  if (pmax > pc) {   // the plan's capacity bounds every product rank
    if (tid == 0) atomicOr(err, 4);
    return;
  }
  const uint64_t s_seed = seed + (uint64_t)b;
  double* Wb = wsb + ws_off[b];
  double* S = Wb + (int64_t)(d - 1) * pc * ell;
  double* U2 = S + (int64_t)ell * nm * (ell > K ? ell : K);
  double* Zt = U2 + (int64_t)nm * pc * ell;
  double* M = Zt + (int64_t)ell * nm * (pc > K ? pc : K);
  double* Qm = M + (int64_t)ell * nm * ell;
  double* tau = Qm + (int64_t)ell * nm * ell;
  double* C = tau + ell;
  double* C2 = C + (int64_t)ell * pc;
  double* qws = C2 + (int64_t)ell * pc;
  auto Wk = [&](int k) { return Wb + (int64_t)(k - 1) * pc * ell; };
  auto nmode = [&](int k) {
    const CoreDesc& cd = cores[md.c0 + k];
    return op == 0 ? cd.I : cd.J;
  };
  auto counter_off = [&](int k) {   // o_k
    uint64_t o = 0;
    for (int j = 1; j < k; ++j) o += (uint64_t)ell * nmode(j) * ell;
    return o;
  };
  auto lr = [&](int k) { return Pold[k] < ell ? Pold[k] : ell; };

  // right to left: W_{d-1}, then W_k from W_{k+1}
  {
    const int k = d - 1, n = nmode(k), P = Pold[k], lk = lr(k);
    const int64_t nK = (int64_t)n * K;
    const uint64_t o = cbase + counter_off(k);
    for (int64_t e = tid; e < lk * nK; e += NT) S[e] = gaussian_at(s_seed, o + (uint64_t)e);
    __syncthreads();
    const T* Y = Z + cores[md.c0 + k].z_off;
    wg_gemm<T>(lk, P, (int)nK, 1.0, S, nK, 1, Y, 1, nK, 0.0, Wk(k), 1, lk, arena);
  }
  for (int k = d - 2; k >= 1; --k) {
    const int n = nmode(k), P = Pold[k], P2 = Pold[k + 1], lk = lr(k), lk2 = lr(k + 1);
    const uint64_t o = cbase + counter_off(k);
    for (int64_t e = tid; e < (int64_t)lk * n * lk2; e += NT) {
      const int64_t c2 = e % lk2, ci = e / lk2;
      S[e] = gaussian_at(s_seed, o + (uint64_t)(ci * ell + c2));
    }
    __syncthreads();
    for (int i = 0; i < n; ++i)   // U2[(i P2 + q) lk + c] = sum_c' W_{k+1}[q, c'] S[c, i, c']
      wg_gemm<double>(P2, lk, lk2, 1.0, Wk(k + 1), lk2, 1, S + (int64_t)i * lk2, 1,
                      (int64_t)n * lk2, 0.0, U2 + (int64_t)i * P2 * lk, lk, 1, arena);
    const T* Y = Z + cores[md.c0 + k].z_off;
    wg_gemm<T>(lk, P, n * P2, 1.0, U2, 1, lk, Y, 1, (int64_t)n * P2, 0.0, Wk(k), 1, lk, arena);
  }

  // left to right
  if (tid == 0) C[0] = 1.0;
  __syncthreads();
  int s = 1;
  for (int k = 0; k < d - 1; ++k) {
    const int n = nmode(k), P = Pold[k], P2 = Pold[k + 1], lk2 = lr(k + 1), sn = s * n;
    const int rho = sn < lk2 ? sn : lk2;
    T* Y = Z + cores[md.c0 + k].z_off;
    wg_gemm<T>(s, n * P2, P, 1.0, C, P, 1, Y, (int64_t)n * P2, 1, 0.0, Zt, (int64_t)n * P2, 1,
               arena);
    wg_gemm<double>(sn, lk2, P2, 1.0, Zt, P2, 1, Wk(k + 1), lk2, 1, 0.0, M, 1, sn, arena);
    wg_qr(M, sn, lk2, sn, tau, qws, arena);
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)sn * rho; e += NT) Qm[e] = (e % sn) == (e / sn) ? 1.0 : 0.0;
    __syncthreads();
    wg_apply_q(M, tau, sn, rho, Qm, rho, sn);
    __syncthreads();
    wg_gemm<double>(rho, P2, sn, 1.0, Qm, sn, 1, Zt, P2, 1, 0.0, C2, P2, 1, arena);
    for (int64_t e = tid; e < (int64_t)sn * rho; e += NT) {
      const int64_t row = e / rho, r = e % rho;
      Y[e] = T(Qm[r * sn + row]);
    }
    double* t = C;
    C = C2;
    C2 = t;
    s = rho;
    if (tid == 0) pr[md.r0 + k + 1] = rho;
    __syncthreads();
  }
  {
    const int k = d - 1, n = nmode(k), P = Pold[k];
    const int64_t nK = (int64_t)n * K;
    T* Y = Z + cores[md.c0 + k].z_off;
    wg_gemm<T>(s, (int)nK, P, 1.0, C, P, 1, Y, nK, 1, 0.0, Zt, nK, 1, arena);
    for (int64_t e = tid; e < s * nK; e += NT) Y[e] = T(Zt[e]);
  }
}

}  // namespace

int64_t qr_ws_doubles(int64_t m, int64_t n) { return m * pick_qb(m) + 2 * (int64_t)pick_qb(m) * n + m; }

hipError_t launch_tsqr_leaf(double* Pw, int h, int N, int L, double* tau, double* ws, int64_t wss,
                            double* up, hipStream_t s) {
  k_tsqr_leaf<<<L, NT, 0, s>>>(Pw, h, N, tau, ws, wss, up, L == 1);
  return hipGetLastError();
}

hipError_t launch_tsqr_node(double* S, int N, int cnt, double* tau, double* ws, int64_t wss,
                            double* up, hipStream_t s) {
  k_tsqr_node<<<cnt, NT, 0, s>>>(S, N, tau, ws, wss, up, cnt == 1);
  return hipGetLastError();
}

hipError_t launch_root_svd(const double* Rf, int N, int64_t n1, double eps, int dm1, int rmax,
                           double* B, double* U, double* nrm, double* sig, int* perm, int* flag,
                           double* Y0, double* T, int* rho_out, double* delta_out, hipStream_t s) {
  k_root_svd<<<1, NT, 0, s>>>(Rf, N, n1, eps, dm1, rmax, B, U, nrm, sig, perm, flag, Y0, T,
                              rho_out, delta_out);
  return hipGetLastError();
}

hipError_t launch_tsqr_apply_node(const double* S, const double* tau, int N, int rho, int cnt,
                                  const double* Yup, int root, double* Yl, hipStream_t s) {
  k_tsqr_apply_node<<<cnt, NT, 0, s>>>(S, tau, N, rho, Yup, root, Yl);
  return hipGetLastError();
}

hipError_t launch_tsqr_apply_leaf(const double* Pw, const double* tau, int h, int N, int rho,
                                  int64_t n1, int L, const double* Yup, double* core1,
                                  hipStream_t s) {
  k_tsqr_apply_leaf<<<L, NT, 0, s>>>(Pw, tau, h, N, rho, n1, Yup, L == 1, core1);
  return hipGetLastError();
}

int64_t colsign_chunks(int64_t n1) { return (n1 + kColChunk - 1) / kColChunk; }

hipError_t launch_colsign(double* X, int64_t n1, int rho, double* T, int N, double* pv,
                          int64_t* pi, double* sgn, hipStream_t s) {
  const int64_t nch = colsign_chunks(n1);
  k_colmax<<<(unsigned)nch, NT, 0, s>>>(X, n1, rho, pv, pi);
  k_colsign<<<1, NT, 0, s>>>(X, rho, pv, pi, (int)nch, sgn);
  const int64_t tot = n1 * rho + (int64_t)rho * N;
  const int64_t g = (tot + 255) / 256;
  k_apply_sign<<<(unsigned)(g > 16384 ? 16384 : g), 256, 0, s>>>(X, n1, rho, T, N, sgn);
  return hipGetLastError();
}

hipError_t launch_round_level(const double* T, int rp, int cp, const int* pm, const int* nx, int n,
                              int q, const double* delta_p, int rmax, double* M, double* ws,
                              double* tau, double* B, double* U, double* nrm, double* sig,
                              int* perm, double* sgn, int* flag, double* Y, double* core,
                              double* Tn, int* rho_out, hipStream_t s) {
  k_round_level<<<1, NT, 0, s>>>(T, rp, cp, pm, nx, n, q, delta_p, rmax, M, ws, tau, B, U, nrm,
                                 sig, perm, sgn, flag, Y, core, Tn, rho_out);
  return hipGetLastError();
}

hipError_t launch_round_last(const double* T, int rp, int cp, const int* pm, int n, double* core,
                             hipStream_t s) {
  k_round_last<<<1, NT, 0, s>>>(T, rp, cp, pm, n, core);
  return hipGetLastError();
}

// SVD-based rounding (Sec. 3) of a general MPO: right-to-left LQ of cores
// d..2 with each L absorbed into the left neighbour (k_lq_absorb; the
// orthogonalised cores stay as Householder reflectors), delta from the first
// core's norm, then left-to-right truncated SVDs of the carried factor times
// each core (k_round_first, k_round_step); the last core takes the remaining
// factor (k_round_last_q).  One workgroup per step; each step reads the rank
// the previous one kept from the device.  The zero matrix (|A|_F = 0 after the first pass)
// gives zero rank-1 cores.  Every buffer but the result cores is carved from
// one allocation sized on the host from the ranks of the first pass (exact)
// and the caps of the second (each kept rank is at most the first pass's).
hipError_t round_mpo(int d, const int64_t* rank, const int64_t* I, const int64_t* J,
                     const double* const* cores, double eps, int rmax, RoundedMpo* out,
                     hipStream_t s) {
  DevArena A;
  hipError_t e = hipSuccess;
  std::vector<double*> res(d, nullptr);
  out->ranks.assign(d + 1, 1);
  out->cores.assign(d, nullptr);
  auto finish = [&]() {
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int k = 0; k < d; ++k) {
      A.release(res[k]);
      out->cores[k] = res[k];
    }
    return hipSuccess;
  };
  auto read_back = [&](void* host, const void* dev, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  };
  std::vector<int64_t> n(d), rr(rank, rank + d + 1), mk(d, 0);
  for (int k = 0; k < d; ++k) n[k] = I[k] * J[k];
  for (int k = d - 1; k >= 1; --k) {   // ranks after the right-to-left pass
    mk[k] = n[k] * rr[k + 1];
    rr[k] = mk[k] < rank[k] ? mk[k] : rank[k];
  }
  // ---- workspace plan (doubles, 256-byte pieces)
  int64_t tot = 0;
  auto take = [&](int64_t cnt) {
    const int64_t o = tot;
    tot += ((cnt > 0 ? cnt : 1) + 31) / 32 * 32;
    return o;
  };
  std::vector<int64_t> oX(d, 0), oT(d, 0), oG(d, 0);
  int64_t ws_rl = 1, rt_rl = 1;
  for (int k = d - 1; k >= 1; --k) {
    const int64_t r = rank[k], rk = rr[k], pn = rank[k - 1] * n[k - 1];
    oX[k] = take(mk[k] * r);
    oT[k] = take(r);
    oG[k - 1] = take(pn * rk);
    ws_rl = std::max(ws_rl, qr_ws_doubles(mk[k], r));
    rt_rl = std::max(rt_rl, r * rk);
  }
  int64_t cM = 1, cws = 1, ctau = 1, cU = 1, cmn = 1, ccap = 1, cY = 1, cTn = 1, cwsq = 1;
  auto sr_cap = [&](int k) {   // rows of the carried factor at step k
    if (k == 0) return (int64_t)1;
    return (rmax > 0 && rmax < rr[k]) ? (int64_t)rmax : rr[k];
  };
  for (int k = 0; k < d - 1; ++k) {
    const int64_t nv = sr_cap(k) * n[k], q = rr[k + 1], mn = nv < q ? nv : q;
    const int64_t cap = (rmax > 0 && rmax < mn) ? rmax : mn;
    cM = std::max(cM, nv * q);
    cws = std::max(cws, nv * (QBMAX + 1) + 2 * QBMAX * q);   // qr_ws_doubles at any m <= nv
    ctau = std::max(ctau, q);
    cU = std::max(cU, mn * mn);
    cmn = std::max(cmn, mn);
    ccap = std::max(ccap, cap);
    cY = std::max(cY, nv * cap);
    cTn = std::max(cTn, cap * q);
    if (k > 0) cwsq = std::max(cwsq, mk[k] * QBMAX + 2 * QBMAX * sr_cap(k));
  }
  if (d > 1) cwsq = std::max(cwsq, mk[d - 1] * QBMAX + 2 * QBMAX * sr_cap(d - 1));
  const int64_t o_wsrl = take(ws_rl), o_rt = take(rt_rl), o_M = take(cM), o_ws = take(cws),
                o_tau = take(ctau), o_B = take(cM), o_U = take(cU), o_nrm = take(cmn),
                o_sig = take(cmn), o_perm = take(cmn), o_sgn = take(ccap), o_Y = take(cY),
                o_Tn0 = take(cTn), o_Tn1 = take(cTn), o_Z = take(cM), o_wsq = take(cwsq),
                o_dl = take(2), o_one = take(1), o_flag = take(4), o_rho = take(d + 1);
  double* W = A.get<double>(tot);
  if ((e = A.e) != hipSuccess) return e;
  auto at = [&](int64_t o) { return W + o; };

  const double* G0 = cores[0];
  std::vector<const double*> X(d, nullptr), tq(d, nullptr);
  const double* Gk = d > 1 ? cores[d - 1] : nullptr;
  for (int k = d - 1; k >= 1 && e == hipSuccess; --k) {
    const int64_t r = rank[k], m = mk[k], pn = rank[k - 1] * n[k - 1];
    double* Xk = at(oX[k]);
    double* tk = at(oT[k]);
    double* Gpo = at(oG[k - 1]);
    k_lq_absorb<<<1, NT, 0, s>>>(Gk, (int)r, (int)m, cores[k - 1], (int)pn, Xk, tk, at(o_wsrl),
                                 at(o_rt), Gpo);
    e = hipGetLastError();
    X[k] = Xk;
    tq[k] = tk;
    Gk = Gpo;   // core k - 1 with L absorbed
  }
  if (d > 1) G0 = Gk;
  double* dl = at(o_dl);
  if (e == hipSuccess) {
    k_norm_delta<<<1, NT, 0, s>>>(G0, n[0] * rr[1], eps, d - 1, dl);
    e = hipGetLastError();
  }
  double hd[2] = {0.0, 0.0};
  read_back(hd, dl, sizeof(hd));
  if (e != hipSuccess) return e;
  if (hd[1] == 0.0) {   // the zero matrix
    for (int k = 0; k < d && e == hipSuccess; ++k) {
      res[k] = A.get<double>(n[k]);
      if ((e = A.e) == hipSuccess) e = hipMemsetAsync(res[k], 0, sizeof(double) * n[k], s);
    }
    return finish();
  }
  if (d == 1) {   // a single core is the matrix itself
    res[0] = A.get<double>(n[0]);
    if ((e = A.e) == hipSuccess)
      e = hipMemcpyAsync(res[0], G0, sizeof(double) * n[0], hipMemcpyDeviceToDevice, s);
    return finish();
  }
  double* one = at(o_one);
  int* flag = (int*)at(o_flag);
  int* rho_d = (int*)at(o_rho);
  const double h_one = 1.0;
  e = hipMemcpyAsync(one, &h_one, sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 4 * sizeof(int), s);
  // no host round trip between steps: each kernel reads the rank the previous
  // one kept from rho_d, and the result cores are sized by the caps
  const double* T = one;
  for (int k = 0; k < d - 1 && e == hipSuccess; ++k) {
    const int64_t q = rr[k + 1], nv = sr_cap(k) * n[k];
    const int64_t mn = nv < q ? nv : q;
    const int64_t cap = (rmax > 0 && rmax < mn) ? rmax : mn;
    res[k] = A.get<double>(nv * cap);
    if ((e = A.e) != hipSuccess) break;
    double* Tn = at((k & 1) ? o_Tn1 : o_Tn0);
    if (k == 0)
      k_round_first<<<1, NT, 0, s>>>(T, G0, (int)n[0], (int)q, dl, rmax, at(o_M), at(o_ws),
                                     at(o_tau), at(o_B), at(o_U), at(o_nrm), at(o_sig),
                                     (int*)at(o_perm), at(o_sgn), flag, at(o_Y), res[k], Tn,
                                     rho_d + 1);
    else
      k_round_step<<<1, NT, 0, s>>>(T, rho_d + k, (int)rr[k], X[k], tq[k], (int)mk[k], (int)n[k],
                                    (int)q, dl, rmax, at(o_Z), at(o_wsq), at(o_M), at(o_ws),
                                    at(o_tau), at(o_B), at(o_U), at(o_nrm), at(o_sig),
                                    (int*)at(o_perm), at(o_sgn), flag, at(o_Y), res[k], Tn,
                                    rho_d + k + 1);
    e = hipGetLastError();
    T = Tn;
  }
  if (e == hipSuccess) {
    const int k = d - 1;
    res[k] = A.get<double>(sr_cap(k) * n[k]);
    if ((e = A.e) == hipSuccess) {
      k_round_last_q<<<1, NT, 0, s>>>(T, rho_d + k, (int)rr[k], X[k], tq[k], (int)n[k], at(o_wsq),
                                      res[k]);
      e = hipGetLastError();
    }
  }
  std::vector<int> kept(d + 1, 1);
  read_back(kept.data() + 1, rho_d + 1, sizeof(int) * (d - 1));
  for (int k = 1; k < d; ++k) out->ranks[k] = kept[k];
  return finish();
}

hipError_t launch_sketch(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op, int* pr,
                         void* Z, int dtype, int ell, uint64_t seed, uint64_t cbase,
                         const int* nm, const int64_t* off, double* ws, int* err, hipStream_t s) {
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_sketch_pass<T><<<batch, NT, 0, s>>>(mpos, cores, op, pr, (T*)Z, ell, seed, cbase, nm, off,
                                          ws, err);
  });
  return hipGetLastError();
}

}  // namespace tnr
