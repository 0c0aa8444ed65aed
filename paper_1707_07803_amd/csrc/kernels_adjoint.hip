// Reverse-mode derivative of the whole TNrSVD pipeline on the GPU (gfx950).
//
// L = sum_{j<k} dsigma_j sigma_j of the solve (Algorithm 5.4: Y = A Omega,
// rounding + orthogonalisation after every product, q power steps, B^T = A^T Q
// and its rounding with the SVD of the last core, Sec. 5.4), differentiated
// with respect to the merged cores of A with Omega fixed and every rounding's
// ranks frozen at the values the forward solve chose.  Nothing of the forward
// solve is kept besides those ranks: the products and roundings are computed
// again here, in FP64, from A and Omega.
//
// Each rounding is differentiated in its Gram (environment) form, which
// computes the same map as the QR/SVD sweep of Sec. 3 (rounding) and
// Algorithms 5.2-5.3 but stays differentiable when a product has lower rank
// than its bond dimensions:
//   G_d = I_K, G_i = sum_x Y_i[:, x, :] G_{i+1} Y_i[:, x, :]^T   (right Grams)
//   left to right: M_i = (T_i Y_i) as (s_i n_i) x P_{i+1};
//   H_i = M_i G_{i+1} M_i^T = U diag(lam) U^T, the kept columns U_r (largest
//   entry of each positive) form the output core, T_{i+1} = U_r^T M_i;
//   last core: QR with diag(R) >= 0 (orthogonalise) or SVD (solve).
// The reverse pass runs these steps backwards (eigenvector derivative with
// F_aj = 1 / (lam_j - lam_a), the QR derivative, dM = X diag(dsigma) W^T for
// the SVD), then the Gram recursion from left to right, then the product's
// bilinear adjoint, stage by stage from the solve back to Y = A Omega.
//
// Building blocks: a tiled FP64 matrix-core GEMM with arbitrary element
// strides (k_dgemm, one 64 x 64 tile per workgroup), the product and its
// adjoints (one thread per output), a one-workgroup symmetric eigensolver
// (one-sided Jacobi on the rows of H), the last-core QR and SVD and their
// adjoints (one workgroup).  The host code orchestrates them with the shapes
// read back once from the recorded ranks.
#include <vector>

#include "tnrsvd_internal.h"
#include "wg_linalg.h"

namespace tnr {

namespace {

// C (M x N) = beta C + alpha A B with element (i, k) of A at A[i sai + k sak],
// (k, j) of B at B[k sbk + j sbj], (i, j) of C at C[i sci + j scj]; one 64 x 64
// tile of C per workgroup.
__global__ __launch_bounds__(NT) void k_dgemm(int M, int N, int K, double alpha,
                                              const double* A, int64_t sai, int64_t sak,
                                              const double* B, int64_t sbk, int64_t sbj,
                                              double beta, double* C, int64_t sci, int64_t scj,
                                              int tiles_n) {
  __shared__ double lds[GEMM_LDS];
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int i0 = 64 * tm, j0 = 64 * tn;
  const int mt = M - i0 < 64 ? M - i0 : 64;
  const int nt = N - j0 < 64 ? N - j0 : 64;
  wg_gemm_t<64, 64, double>(mt, nt, K, alpha, A + (int64_t)i0 * sai, sai, sak,
                            B + (int64_t)j0 * sbj, sbk, sbj, beta,
                            C + (int64_t)i0 * sci + (int64_t)j0 * scj, sci, scj, lds);
}

// dst (rows x cols, ld ldd) = src (rows x cols, ld lds)
__global__ void k_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                         int cols) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[(int64_t)r * ldd + c] = src[(int64_t)r * lds + c];
  }
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// x (n x n, row-major) <- x + x^T ... into out (out may not alias x)
__global__ void k_sym(const double* x, double* out, int n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), c = (int)(e % n);
    out[e] = x[e] + x[(int64_t)c * n + r];
  }
}

// Product of one core (Sec. 5.2), FP64: op 0 Y[(a,c), x, (b,e)] = sum_y
// A[a,x,y,b] X[c,y,e]; op 1 Y[(a,c), y, (b,e)] = sum_x A[a,x,y,b] X[c,x,e].
template <int OP>
__global__ void k_prod(const double* __restrict__ A, const double* __restrict__ X, double* Y,
                       int Ra, int I, int J, int Rb, int rc, int re) {
  const int n = OP == 0 ? I : J, ns = OP == 0 ? J : I;
  const int64_t tot = (int64_t)Ra * rc * n * Rb * re;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < tot;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = o;
    const int e = (int)(t % re);
    t /= re;
    const int b = (int)(t % Rb);
    t /= Rb;
    const int x = (int)(t % n);
    t /= n;
    const int c = (int)(t % rc);
    const int a = (int)(t / rc);
    double acc = 0.0;
    for (int y = 0; y < ns; ++y) {
      const int ii = OP == 0 ? x : y, jj = OP == 0 ? y : x;
      acc += A[(((int64_t)a * I + ii) * J + jj) * Rb + b] * X[((int64_t)c * ns + y) * re + e];
    }
    Y[o] = acc;
  }
}

// Adjoint of k_prod with respect to A (accumulated): dA[a,x,y,b] +=
// sum_{c,e} dY[(a,c), n, (b,e)] X[c, s, e] with (n, s) = (x, y) for op 0 and
// (y, x) for op 1.
template <int OP>
__global__ void k_prod_dA(const double* __restrict__ dY, const double* __restrict__ X, double* dA,
                          int Ra, int I, int J, int Rb, int rc, int re) {
  const int n = OP == 0 ? I : J, ns = OP == 0 ? J : I;
  const int64_t tot = (int64_t)Ra * I * J * Rb;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < tot;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = o;
    const int b = (int)(t % Rb);
    t /= Rb;
    const int y = (int)(t % J);
    t /= J;
    const int x = (int)(t % I);
    const int a = (int)(t / I);
    const int ni = OP == 0 ? x : y, si = OP == 0 ? y : x;
    double acc = 0.0;
    for (int c = 0; c < rc; ++c)
      for (int e = 0; e < re; ++e)
        acc += dY[((((int64_t)a * rc + c) * n + ni) * Rb + b) * re + e] *
               X[((int64_t)c * ns + si) * re + e];
    dA[o] += acc;
  }
}

// Adjoint of k_prod with respect to X: dX[c, s, e] = sum_{a, n, b}
// dY[(a,c), n, (b,e)] A[a, x, y, b] with (x, y) = (n, s) for op 0, (s, n) for op 1.
template <int OP>
__global__ void k_prod_dX(const double* __restrict__ dY, const double* __restrict__ A, double* dX,
                          int Ra, int I, int J, int Rb, int rc, int re) {
  const int n = OP == 0 ? I : J, ns = OP == 0 ? J : I;
  const int64_t tot = (int64_t)rc * ns * re;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < tot;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = o;
    const int e = (int)(t % re);
    t /= re;
    const int si = (int)(t % ns);
    const int c = (int)(t / ns);
    double acc = 0.0;
    for (int a = 0; a < Ra; ++a)
      for (int ni = 0; ni < n; ++ni) {
        const int x = OP == 0 ? ni : si, y = OP == 0 ? si : ni;
        for (int b = 0; b < Rb; ++b)
          acc += dY[((((int64_t)a * rc + c) * n + ni) * Rb + b) * re + e] *
                 A[(((int64_t)a * I + x) * J + y) * Rb + b];
      }
    dX[o] = acc;
  }
}

// Eigen-decomposition of the symmetric positive semidefinite H (nv x nv,
// row-major; symmetrised here) by one-sided Jacobi on its rows: the rows of
// V^T H are orthogonal with norms lam when V holds the eigenvectors.  Writes
// lam (descending) and U (nv x nv, row-major, column j the eigenvector of
// lam_j); the first rho columns are flipped so that their entry of largest
// magnitude (the first on ties) is positive.  B and W: nv x nv doubles of
// scratch (global); one workgroup.
__global__ __launch_bounds__(NT) void k_sym_eig(const double* H, int nv, int rho, double* lam,
                                                double* U, double* B, double* W, double* nrm,
                                                double* sg, int* perm) {
  __shared__ double red[16];
  __shared__ int flag[2];
  const int tid = threadIdx.x;
  for (int e = tid; e < nv * nv; e += NT) {
    const int r = e / nv, c = e % nv;
    B[e] = 0.5 * (H[e] + H[c * nv + r]);
  }
  __syncthreads();
  wg_jacobi(B, nv, nv, nv, W, flag, red);
  wg_norms_sorted(B, nv, nv, nv, sg, perm, nrm);
  for (int j = tid; j < nv; j += NT) lam[j] = sg[j];
  __syncthreads();
  for (int j = tid; j < nv; j += NT)
    nrm[j] = j < rho ? sign_of_max(W + (int64_t)perm[j] * nv, nv, 1) : 1.0;
  __syncthreads();
  for (int e = tid; e < nv * nv; e += NT) {
    const int r = e / nv, j = e % nv;
    U[e] = W[(int64_t)perm[j] * nv + r] * nrm[j];
  }
}

// Economy QR with diag(R) >= 0 of the last core's panel M (m x K, row-major,
// m >= K): Q (m x K, row-major) and R (K x K, row-major, zero lower triangle).
// X: m K doubles, E: m K doubles of scratch; one workgroup.
__global__ __launch_bounds__(NT) void k_last_qr(const double* M, int m, int K, double* Q, double* R,
                                                double* X, double* E, double* tau) {
  __shared__ double v[4096 + 16];
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)m * K; e += NT) {
    const int c = (int)(e / m), r = (int)(e % m);
    X[e] = M[(int64_t)r * K + c];   // column-major copy
  }
  __syncthreads();
  wg_geqr2(X, m, K, tau, v, v + 4096);
  for (int e = tid; e < K * K; e += NT) {
    const int r = e / K, c = e % K;
    R[e] = c >= r ? X[(int64_t)c * m + r] : 0.0;
  }
  for (int64_t e = tid; e < (int64_t)m * K; e += NT) {
    const int c = (int)(e / m), r = (int)(e % m);
    E[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_apply_q(X, tau, m, K, E, K);
  for (int64_t e = tid; e < (int64_t)m * K; e += NT) {
    const int r = (int)(e / K), c = (int)(e % K);
    Q[e] = E[(int64_t)c * m + r];
  }
}

// Economy SVD of the last core's panel M (m x K, row-major, m >= K) by one-sided
// Jacobi on its columns: S descending, X (m x K, row-major) the left vectors
// (largest entry of each positive), Wt (K x K, row-major) the right ones
// transposed, M = X diag(S) Wt.  B: m K, W: K K doubles of scratch.
__global__ __launch_bounds__(NT) void k_last_svd(const double* M, int m, int K, double* S,
                                                 double* X, double* Wt, double* B, double* W,
                                                 double* nrm, double* sg, int* perm) {
  __shared__ double red[16];
  __shared__ int flag[2];
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)m * K; e += NT) {
    const int c = (int)(e / m), r = (int)(e % m);
    B[e] = M[(int64_t)r * K + c];   // column c of M as vector c
  }
  __syncthreads();
  wg_jacobi(B, K, m, m, W, flag, red);
  wg_norms_sorted(B, K, m, m, sg, perm, nrm);
  for (int j = tid; j < K; j += NT) S[j] = sg[j];
  __syncthreads();
  for (int j = tid; j < K; j += NT) nrm[j] = sign_of_max(B + (int64_t)perm[j] * m, m, 1);
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)m * K; e += NT) {
    const int r = (int)(e / K), j = (int)(e % K);
    const double sj = sg[j];
    X[e] = sj > 0.0 ? B[(int64_t)perm[j] * m + r] * nrm[j] / sj : 0.0;
  }
  for (int e = tid; e < K * K; e += NT) {
    const int j = e / K, c = e % K;
    Wt[e] = W[(int64_t)perm[j] * K + c] * nrm[j];
  }
}

// QR derivative: dM = (dQ + Q copyltu(-dQ^T Q)) R^{-T} for M = Q R (m x K,
// R invertible), copyltu(C) the symmetric matrix with C's lower triangle.
// All row-major; C: K K doubles of scratch.  One workgroup.
__global__ __launch_bounds__(NT) void k_qr_adjoint(const double* Q, const double* R,
                                                   const double* dQ, int m, int K, double* dM,
                                                   double* C) {
  const int tid = threadIdx.x;
  for (int e = tid; e < K * K; e += NT) {
    const int a = e / K, b = e % K;
    double acc = 0.0;
    for (int r = 0; r < m; ++r) acc -= dQ[(int64_t)r * K + a] * Q[(int64_t)r * K + b];
    C[e] = acc;
  }
  __syncthreads();
  for (int r = tid; r < m; r += NT) {
    double* out = dM + (int64_t)r * K;
    // B row r = dQ[r] + Q[r] S, S[a][b] = C[max][min]
    for (int b = 0; b < K; ++b) {
      double acc = dQ[(int64_t)r * K + b];
      for (int a = 0; a < K; ++a) {
        const double sab = a >= b ? C[a * K + b] : C[b * K + a];
        acc += Q[(int64_t)r * K + a] * sab;
      }
      out[b] = acc;
    }
    // x R^T = B_r  <=>  R x^T = B_r^T (R upper triangular): back substitution
    for (int i = K - 1; i >= 0; --i) {
      double acc = out[i];
      for (int j = i + 1; j < K; ++j) acc -= R[i * K + j] * out[j];
      out[i] = acc / R[i * K + i];
    }
  }
}

// dM = X diag(w) Wt for the SVD of the last core (m x K, row-major).
__global__ void k_svd_adjoint(const double* X, const double* w, const double* Wt, int m, int K,
                              double* dM) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)m * K;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / K), c = (int)(e % K);
    double acc = 0.0;
    for (int j = 0; j < K; ++j) acc += X[(int64_t)r * K + j] * w[j] * Wt[(int64_t)j * K + c];
    dM[e] = acc;
  }
}

// Z (nv x rho, row-major) <- F o Z, F_aj = 1 / (lam_j - lam_a) for a != j
// (0 on the diagonal and where the difference vanishes).
__global__ void k_eig_f(double* Z, const double* lam, int nv, int rho) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)nv * rho;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / rho), j = (int)(e % rho);
    const double diff = lam[j] - lam[a];
    Z[e] = (a == j || diff == 0.0) ? 0.0 : Z[e] / diff;
  }
}

int grid1(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------

struct Ctx {
  hipStream_t s;
  DevArena* A;
  hipError_t e = hipSuccess;
  double* get(int64_t n) {
    double* p = A->get<double>(n);
    if (!p && e == hipSuccess) e = A->e != hipSuccess ? A->e : hipErrorOutOfMemory;
    return p;
  }
  void gemm(int M, int N, int K, double alpha, const double* a, int64_t sai, int64_t sak,
            const double* b, int64_t sbk, int64_t sbj, double beta, double* c, int64_t sci,
            int64_t scj) {
    if (e != hipSuccess || M <= 0 || N <= 0) return;
    const int tn = (N + 63) / 64, tm = (M + 63) / 64;
    k_dgemm<<<tm * tn, NT, 0, s>>>(M, N, K, alpha, a, sai, sak, b, sbk, sbj, beta, c, sci, scj, tn);
    e = hipGetLastError();
  }
  // row-major shorthands: C (MxN) = beta C + alpha op(A) op(B)
  void mm(int M, int N, int K, double alpha, const double* a, int lda, bool ta, const double* b,
          int ldb, bool tb, double beta, double* c, int ldc) {
    gemm(M, N, K, alpha, a, ta ? 1 : lda, ta ? lda : 1, b, tb ? 1 : ldb, tb ? ldb : 1, beta, c,
         ldc, 1);
  }
  void fill(double* p, int64_t n, double v) {
    if (e != hipSuccess || n <= 0) return;
    k_fill<<<grid1(n), 256, 0, s>>>(p, n, v);
    e = hipGetLastError();
  }
  void copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows, int cols) {
    if (e != hipSuccess || rows <= 0 || cols <= 0) return;
    k_copy2d<<<grid1((int64_t)rows * cols), 256, 0, s>>>(src, lds, dst, ldd, rows, cols);
    e = hipGetLastError();
  }
};

// One rounding in Gram form, with everything its reverse pass needs.
struct Rec {
  int op = 0;
  bool svd = false;
  std::vector<int> x;          // ranks of the basis that entered the product (d + 1)
  std::vector<int> rho;        // ranks kept (d + 1): rho[0] = 1, rho[d] = K
  std::vector<int> P, n;       // product ranks (d + 1) and mode sizes (d)
  std::vector<double*> X;      // basis cores entering the product (x_i, ns_i, x_{i+1})
  std::vector<double*> Y;      // product cores (P_i, n_i, P_{i+1})
  std::vector<double*> G;      // right Grams G_i (P_i x P_i), G_d = I_K
  std::vector<double*> M, U, lam, T;   // per core i < d - 1 (M, T also for d - 1)
  double *Q = nullptr, *R = nullptr, *Xs = nullptr, *S = nullptr, *Wt = nullptr;
  std::vector<double*> out;    // output cores (rho_i, n_i, rho_{i+1})
};

void run_round(Ctx& c, Rec& r, int d, int K, double* eig_ws, int64_t eig_n) {
  const std::vector<int>& P = r.P;
  r.G.assign(d + 1, nullptr);
  for (int i = 0; i <= d; ++i) r.G[i] = c.get((int64_t)P[i] * P[i]);
  if (c.e != hipSuccess) return;
  // G_d = I_K
  c.fill(r.G[d], (int64_t)K * K, 0.0);
  for (int j = 0; j < K && c.e == hipSuccess; ++j) {
    k_fill<<<1, 1, 0, c.s>>>(r.G[d] + (int64_t)j * K + j, 1, 1.0);
    c.e = hipGetLastError();
  }
  for (int i = d - 1; i >= 0; --i) {
    const int p = P[i], n = r.n[i], p2 = P[i + 1];
    double* T1 = c.get((int64_t)p * n * p2);
    // T1 = Y_i (p n x p2) G_{i+1};  G_i = T1 (p x n p2) Y_i (p x n p2)^T
    c.mm(p * n, p2, p2, 1.0, r.Y[i], p2, false, r.G[i + 1], p2, false, 0.0, T1, p2);
    c.mm(p, p, n * p2, 1.0, T1, n * p2, false, r.Y[i], n * p2, true, 0.0, r.G[i], p);
  }
  r.M.assign(d, nullptr);
  r.U.assign(d, nullptr);
  r.lam.assign(d, nullptr);
  r.T.assign(d, nullptr);
  r.out.assign(d, nullptr);
  // T_0 = [[1]]
  r.T[0] = c.get(1);
  c.fill(r.T[0], 1, 1.0);
  for (int i = 0; i + 1 < d && c.e == hipSuccess; ++i) {
    const int p = P[i], n = r.n[i], p2 = P[i + 1], s = r.rho[i];
    const int nv = s * n, rk = r.rho[i + 1];
    r.M[i] = c.get((int64_t)nv * p2);
    r.U[i] = c.get((int64_t)nv * nv);
    r.lam[i] = c.get(nv);
    double* W1 = c.get((int64_t)nv * p2);
    double* H = c.get((int64_t)nv * nv);
    r.out[i] = c.get((int64_t)s * n * rk);
    r.T[i + 1] = c.get((int64_t)rk * p2);
    if (c.e != hipSuccess) return;
    // M = T Y_i (s x n p2) = (s n) x p2
    c.mm(s, n * p2, p, 1.0, r.T[i], p, false, r.Y[i], n * p2, false, 0.0, r.M[i], n * p2);
    // H = M G M^T
    c.mm(nv, p2, p2, 1.0, r.M[i], p2, false, r.G[i + 1], p2, false, 0.0, W1, p2);
    c.mm(nv, nv, p2, 1.0, W1, p2, false, r.M[i], p2, true, 0.0, H, nv);
    if (c.e != hipSuccess) return;
    double* B = eig_ws;
    double* Wm = eig_ws + eig_n * eig_n;
    double* nrm = Wm + eig_n * eig_n;
    double* sg = nrm + eig_n;
    int* perm = (int*)(sg + eig_n);
    k_sym_eig<<<1, NT, 0, c.s>>>(H, nv, rk, r.lam[i], r.U[i], B, Wm, nrm, sg, perm);
    c.e = hipGetLastError();
    // output core = U_r (nv x rk), row-major (c n + y, k) = core (c, y, k)
    c.copy2d(r.U[i], nv, r.out[i], rk, nv, rk);
    // T_{i+1} = U_r^T M (rk x p2)
    c.mm(rk, p2, nv, 1.0, r.U[i], nv, true, r.M[i], p2, false, 0.0, r.T[i + 1], p2);
  }
  // last core
  const int i = d - 1, p = P[i], n = r.n[i], s = r.rho[i], nv = s * n;
  r.M[i] = c.get((int64_t)nv * K);
  if (c.e != hipSuccess) return;
  c.mm(s, n * K, p, 1.0, r.T[i], p, false, r.Y[i], n * K, false, 0.0, r.M[i], n * K);
  if (!r.svd) {
    r.Q = c.get((int64_t)nv * K);
    r.R = c.get((int64_t)K * K);
    double* Xc = c.get((int64_t)nv * K);
    double* E = c.get((int64_t)nv * K);
    double* tau = c.get(K);
    if (c.e != hipSuccess) return;
    k_last_qr<<<1, NT, 0, c.s>>>(r.M[i], nv, K, r.Q, r.R, Xc, E, tau);
    c.e = hipGetLastError();
    r.out[i] = r.Q;
  } else {
    r.Xs = c.get((int64_t)nv * K);
    r.S = c.get(K);
    r.Wt = c.get((int64_t)K * K);
    double* B = c.get((int64_t)nv * K);
    double* W = c.get((int64_t)K * K);
    double* nrm = c.get(K);
    double* sg = c.get(K);
    double* pm = c.get(K);
    if (c.e != hipSuccess) return;
    k_last_svd<<<1, NT, 0, c.s>>>(r.M[i], nv, K, r.S, r.Xs, r.Wt, B, W, nrm, sg, (int*)pm);
    c.e = hipGetLastError();
  }
}

// Reverse pass of one rounding: dY (per core, allocated here) from the
// cotangents of its output cores dout (nullptr entries: zero) or of sigma (dw).
void round_adjoint(Ctx& c, Rec& r, int d, int K, const std::vector<double*>& dout,
                   const double* dw, std::vector<double*>& dY) {
  const std::vector<int>& P = r.P;
  dY.assign(d, nullptr);
  std::vector<double*> dG(d + 1, nullptr);
  for (int i = 0; i < d; ++i) {
    dY[i] = c.get((int64_t)P[i] * r.n[i] * P[i + 1]);
    c.fill(dY[i], (int64_t)P[i] * r.n[i] * P[i + 1], 0.0);
  }
  for (int i = 1; i < d; ++i) {
    dG[i] = c.get((int64_t)P[i] * P[i]);
    c.fill(dG[i], (int64_t)P[i] * P[i], 0.0);
  }
  if (c.e != hipSuccess) return;
  // last core
  int i = d - 1;
  int p = P[i], n = r.n[i], s = r.rho[i], nv = s * n;
  double* dM = c.get((int64_t)nv * K);
  double* dT = c.get((int64_t)s * p);
  if (c.e != hipSuccess) return;
  if (!r.svd) {
    double* C = c.get((int64_t)K * K);
    double* dQ = dout[i];
    double* zq = nullptr;
    if (!dQ) {
      zq = c.get((int64_t)nv * K);
      c.fill(zq, (int64_t)nv * K, 0.0);
      dQ = zq;
    }
    if (c.e != hipSuccess) return;
    k_qr_adjoint<<<1, NT, 0, c.s>>>(r.Q, r.R, dQ, nv, K, dM, C);
    c.e = hipGetLastError();
  } else {
    k_svd_adjoint<<<grid1((int64_t)nv * K), 256, 0, c.s>>>(r.Xs, dw, r.Wt, nv, K, dM);
    c.e = hipGetLastError();
  }
  // dM as dMr (s x n K): dT = dMr Y^T (s x p);  dY += T^T dMr (p x n K)
  c.mm(s, p, n * K, 1.0, dM, n * K, false, r.Y[i], n * K, true, 0.0, dT, p);
  c.mm(p, n * K, s, 1.0, r.T[i], p, true, dM, n * K, false, 1.0, dY[i], n * K);
  for (i = d - 2; i >= 0 && c.e == hipSuccess; --i) {
    p = P[i];
    n = r.n[i];
    s = r.rho[i];
    nv = s * n;
    const int p2 = P[i + 1], rk = r.rho[i + 1];
    double* dMi = c.get((int64_t)nv * p2);
    double* dU = c.get((int64_t)nv * rk);
    double* Z = c.get((int64_t)nv * rk);
    double* Zu = c.get((int64_t)nv * rk);
    double* dH = c.get((int64_t)nv * nv);
    double* Sd = c.get((int64_t)nv * nv);
    double* W1 = c.get((int64_t)nv * p2);
    double* W2 = c.get((int64_t)p2 * nv);
    double* dTn = c.get((int64_t)s * p);
    if (c.e != hipSuccess) return;
    // dU = cotangent of the output core (nv x rk) + M dT^T
    if (dout[i]) {
      c.copy2d(dout[i], rk, dU, rk, nv, rk);
    } else {
      c.fill(dU, (int64_t)nv * rk, 0.0);
    }
    c.mm(nv, rk, p2, 1.0, r.M[i], p2, false, dT, p2, true, 1.0, dU, rk);
    // dM = U_r dT
    c.mm(nv, p2, rk, 1.0, r.U[i], nv, false, dT, p2, false, 0.0, dMi, p2);
    // dH = U (F o (U^T dU)) U_r^T
    c.mm(nv, rk, nv, 1.0, r.U[i], nv, true, dU, rk, false, 0.0, Z, rk);
    if (c.e != hipSuccess) return;
    k_eig_f<<<grid1((int64_t)nv * rk), 256, 0, c.s>>>(Z, r.lam[i], nv, rk);
    c.e = hipGetLastError();
    c.mm(nv, rk, nv, 1.0, r.U[i], nv, false, Z, rk, false, 0.0, Zu, rk);
    c.mm(nv, nv, rk, 1.0, Zu, rk, false, r.U[i], nv, true, 0.0, dH, nv);
    // dM += (dH + dH^T) M G_{i+1}
    if (c.e != hipSuccess) return;
    k_sym<<<grid1((int64_t)nv * nv), 256, 0, c.s>>>(dH, Sd, nv);
    c.e = hipGetLastError();
    c.mm(nv, p2, p2, 1.0, r.M[i], p2, false, r.G[i + 1], p2, false, 0.0, W1, p2);
    c.mm(nv, p2, nv, 1.0, Sd, nv, false, W1, p2, false, 1.0, dMi, p2);
    // dG_{i+1} += M^T dH M
    c.mm(p2, nv, nv, 1.0, r.M[i], p2, true, dH, nv, false, 0.0, W2, nv);
    c.mm(p2, p2, nv, 1.0, W2, nv, false, r.M[i], p2, false, 1.0, dG[i + 1], p2);
    // dT_i = dMr Y_i^T (s x p), dY_i += T_i^T dMr
    c.mm(s, p, n * p2, 1.0, dMi, n * p2, false, r.Y[i], n * p2, true, 0.0, dTn, p);
    c.mm(p, n * p2, s, 1.0, r.T[i], p, true, dMi, n * p2, false, 1.0, dY[i], n * p2);
    dT = dTn;
  }
  // the right Grams, left to right: G_i = sum_x Y_x G_{i+1} Y_x^T
  for (i = 1; i < d && c.e == hipSuccess; ++i) {
    p = P[i];
    n = r.n[i];
    const int p2 = P[i + 1];
    double* Sd = c.get((int64_t)p * p);
    double* YG = c.get((int64_t)p * n * p2);
    double* DY = c.get((int64_t)p * n * p2);
    if (c.e != hipSuccess) return;
    k_sym<<<grid1((int64_t)p * p), 256, 0, c.s>>>(dG[i], Sd, p);
    c.e = hipGetLastError();
    c.mm(p * n, p2, p2, 1.0, r.Y[i], p2, false, r.G[i + 1], p2, false, 0.0, YG, p2);
    c.mm(p, n * p2, p, 1.0, Sd, p, false, YG, n * p2, false, 1.0, dY[i], n * p2);
    if (i + 1 < d) {
      c.mm(p, n * p2, p, 1.0, dG[i], p, false, r.Y[i], n * p2, false, 0.0, DY, n * p2);
      c.mm(p2, p2, p * n, 1.0, r.Y[i], p2, true, DY, p2, false, 1.0, dG[i + 1], p2);
    }
  }
}

}  // namespace

// Gradient of sum_{j<k} dsigma_j sigma_j with respect to the merged cores of one
// MPO (FP64 device cores A[i] of shape (Ra, I, J, Rb)), written to dA[i]
// (overwritten).  omega: the device Omega of the MPO (vectors of the first d-1
// cores, then the J_last x K matrix).  ranks[t]: the bond ranks (d + 1) kept by
// rounding t of the forward solve (t = 0 .. 2q+1); ops: the product of each
// rounding (0: A X, 1: A^T X); the last rounding is the solve's (SVD).
hipError_t pipeline_adjoint(int d, const CoreShape* shapes, const double* const* A,
                            double* const* dA, const double* omega, int K, int k,
                            const double* dsigma_host,
                            const std::vector<std::vector<int>>& ranks,
                            const std::vector<int>& ops, hipStream_t s) {
  DevArena arena;
  Ctx c;
  c.s = s;
  c.A = &arena;
  const int T = (int)ranks.size();
  std::vector<Rec> rec(T);
  // scratch of the eigensolver: the largest s n of any rounding
  int64_t eig_n = 1;
  for (int t = 0; t < T; ++t)
    for (int i = 0; i + 1 < d; ++i) {
      const int n = ops[t] == 0 ? shapes[i].I : shapes[i].J;
      eig_n = std::max<int64_t>(eig_n, (int64_t)ranks[t][i] * n);
    }
  double* eig_ws = c.get(2 * eig_n * eig_n + 3 * eig_n + 8);
  // forward, recomputed: X_0 = Omega
  std::vector<double*> X(d, nullptr);
  std::vector<int> xr(d + 1, 1);
  xr[d] = K;
  {
    int64_t off = 0;
    for (int i = 0; i < d; ++i) {
      X[i] = const_cast<double*>(omega) + off;
      off += (int64_t)shapes[i].J * (i == d - 1 ? K : 1);
    }
  }
  for (int t = 0; t < T && c.e == hipSuccess; ++t) {
    Rec& r = rec[t];
    r.op = ops[t];
    r.svd = t == T - 1;
    r.x = xr;
    r.rho = ranks[t];
    r.X = X;
    r.n.resize(d);
    r.P.resize(d + 1);
    for (int i = 0; i < d; ++i) {
      r.n[i] = r.op == 0 ? shapes[i].I : shapes[i].J;
      r.P[i] = shapes[i].Ra * xr[i];
    }
    r.P[d] = K;
    // product
    r.Y.assign(d, nullptr);
    for (int i = 0; i < d && c.e == hipSuccess; ++i) {
      const CoreShape& cs = shapes[i];
      const int re = xr[i + 1];
      const int64_t len = (int64_t)r.P[i] * r.n[i] * (i == d - 1 ? K : cs.Rb * re);
      r.Y[i] = c.get(len);
      if (c.e != hipSuccess) break;
      if (r.op == 0)
        k_prod<0><<<grid1(len), 256, 0, s>>>(A[i], X[i], r.Y[i], cs.Ra, cs.I, cs.J, cs.Rb, xr[i],
                                             re);
      else
        k_prod<1><<<grid1(len), 256, 0, s>>>(A[i], X[i], r.Y[i], cs.Ra, cs.I, cs.J, cs.Rb, xr[i],
                                             re);
      c.e = hipGetLastError();
    }
    if (c.e != hipSuccess) break;
    run_round(c, r, d, K, eig_ws, eig_n);
    X = r.out;
    xr = r.rho;
  }
  // reverse
  std::vector<double*> dXo(d, nullptr);   // cotangent of the basis a rounding produced
  double* dw = c.get(K);
  if (c.e == hipSuccess) {
    std::vector<double> w(K, 0.0);
    for (int j = 0; j < k && j < K; ++j) w[j] = dsigma_host ? dsigma_host[j] : 1.0;
    c.e = hipMemcpyAsync(dw, w.data(), sizeof(double) * K, hipMemcpyHostToDevice, s);
    if (c.e == hipSuccess) c.e = hipStreamSynchronize(s);
  }
  for (int i = 0; i < d && c.e == hipSuccess; ++i)
    c.fill(dA[i], (int64_t)shapes[i].Ra * shapes[i].I * shapes[i].J * shapes[i].Rb, 0.0);
  for (int t = T - 1; t >= 0 && c.e == hipSuccess; --t) {
    Rec& r = rec[t];
    std::vector<double*> dY;
    round_adjoint(c, r, d, K, dXo, dw, dY);
    std::vector<double*> dX(d, nullptr);
    for (int i = 0; i < d && c.e == hipSuccess; ++i) {
      const CoreShape& cs = shapes[i];
      const int rc = r.x[i], re = (i == d - 1) ? K : r.x[i + 1];
      const int Rb = cs.Rb;
      const int ns = r.op == 0 ? cs.J : cs.I;
      const int64_t na = (int64_t)cs.Ra * cs.I * cs.J * Rb;
      const int64_t nx = (int64_t)rc * ns * re;
      if (r.op == 0)
        k_prod_dA<0><<<grid1(na), 256, 0, s>>>(dY[i], r.X[i], dA[i], cs.Ra, cs.I, cs.J, Rb, rc, re);
      else
        k_prod_dA<1><<<grid1(na), 256, 0, s>>>(dY[i], r.X[i], dA[i], cs.Ra, cs.I, cs.J, Rb, rc, re);
      c.e = hipGetLastError();
      if (t > 0 && c.e == hipSuccess) {
        dX[i] = c.get(nx);
        if (c.e != hipSuccess) break;
        if (r.op == 0)
          k_prod_dX<0><<<grid1(nx), 256, 0, s>>>(dY[i], A[i], dX[i], cs.Ra, cs.I, cs.J, Rb, rc, re);
        else
          k_prod_dX<1><<<grid1(nx), 256, 0, s>>>(dY[i], A[i], dX[i], cs.Ra, cs.I, cs.J, Rb, rc, re);
        c.e = hipGetLastError();
      }
    }
    dXo = dX;
  }
  if (c.e == hipSuccess) c.e = hipStreamSynchronize(s);
  return c.e;
}

}  // namespace tnr
