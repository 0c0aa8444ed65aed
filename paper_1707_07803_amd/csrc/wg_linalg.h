// Workgroup-level FP64 linear algebra shared by the sweep and rounding kernels
// (gfx950, 512-thread workgroups): wave and workgroup sums, Householder QR
// (unblocked and blocked), application of the reflectors, LDS-tiled GEMM, and
// one-sided Jacobi.  Every function is called by a whole workgroup.
#pragma once

#include "tnrsvd_internal.h"

namespace tnr {

namespace {

constexpr int NT = kSweepThreads;
constexpr int NW = NT / 64;

// DPP move of a double (both 32-bit halves), zero where the source lane is invalid.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(h2, l2);
}

// Sum over the 64 lanes of a wave, returned to every lane: shift-adds within
// each row of 16 lanes, row broadcasts 15 and 31 to fold the four rows into
// lane 63, then a read of lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0x111>(v);          // row_shr:1
  v += dpp_d<0x112>(v);          // row_shr:2
  v += dpp_d<0x114>(v);          // row_shr:4
  v += dpp_d<0x118>(v);          // row_shr:8
  v += dpp_d<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);     // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Three wave sums in lockstep (their DPP chains interleave); every lane
// receives the totals.
__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
  a += dpp_d<0x111>(a);
  b += dpp_d<0x111>(b);
  c += dpp_d<0x111>(c);
  a += dpp_d<0x112>(a);
  b += dpp_d<0x112>(b);
  c += dpp_d<0x112>(c);
  a += dpp_d<0x114>(a);
  b += dpp_d<0x114>(b);
  c += dpp_d<0x114>(c);
  a += dpp_d<0x118>(a);
  b += dpp_d<0x118>(b);
  c += dpp_d<0x118>(c);
  a += dpp_d<0x142, 0xa>(a);
  b += dpp_d<0x142, 0xa>(b);
  c += dpp_d<0x142, 0xa>(c);
  a += dpp_d<0x143, 0xc>(a);
  b += dpp_d<0x143, 0xc>(b);
  c += dpp_d<0x143, 0xc>(c);
  a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(a), 63),
                       __builtin_amdgcn_readlane(__double2loint(a), 63));
  b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(b), 63),
                       __builtin_amdgcn_readlane(__double2loint(b), 63));
  c = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(c), 63),
                       __builtin_amdgcn_readlane(__double2loint(c), 63));
}

// Sum over the 16 lanes of each DPP row, returned to every lane of the row:
// shift-adds within the row leave the total in its lane 15 (src), which is
// then read back by the row's lanes.
__device__ __forceinline__ double row16_sum(double v, int src) {
  v += dpp_d<0x111>(v);          // row_shr:1
  v += dpp_d<0x112>(v);          // row_shr:2
  v += dpp_d<0x114>(v);          // row_shr:4
  v += dpp_d<0x118>(v);          // row_shr:8
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Three row sums in lockstep, as row16_sum.
__device__ __forceinline__ void row16_sum3(double& a, double& b, double& c, int src) {
  a += dpp_d<0x111>(a);
  b += dpp_d<0x111>(b);
  c += dpp_d<0x111>(c);
  a += dpp_d<0x112>(a);
  b += dpp_d<0x112>(b);
  c += dpp_d<0x112>(c);
  a += dpp_d<0x114>(a);
  b += dpp_d<0x114>(b);
  c += dpp_d<0x114>(c);
  a += dpp_d<0x118>(a);
  b += dpp_d<0x118>(b);
  c += dpp_d<0x118>(c);
  const int s4 = src << 2;
  a = __hiloint2double(__builtin_amdgcn_ds_bpermute(s4, __double2hiint(a)),
                       __builtin_amdgcn_ds_bpermute(s4, __double2loint(a)));
  b = __hiloint2double(__builtin_amdgcn_ds_bpermute(s4, __double2hiint(b)),
                       __builtin_amdgcn_ds_bpermute(s4, __double2loint(b)));
  c = __hiloint2double(__builtin_amdgcn_ds_bpermute(s4, __double2hiint(c)),
                       __builtin_amdgcn_ds_bpermute(s4, __double2loint(c)));
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Workgroup barrier that orders LDS only: global stores still in flight are
// not waited for (a plain __syncthreads drains them, which costs an L2 round
// trip).  Only for loops whose global writes nobody reads before the next full
// barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Sum over the workgroup; every thread receives the total.  `red` holds NW doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = wave_id();
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) t += red[k];
  return t;
}

// Maximum over the workgroup; every thread receives it.  `red` holds NW doubles.
__device__ double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, w = wave_id();
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) t = fmax(t, red[k]);
  return t;
}

// Householder QR with nonnegative diagonal of the m x n column-major X (ld m
// unless given),
// in place: R on and above the diagonal of the first min(m,n) rows, the
// Householder vectors (unit leading entry implicit) below it, scalars in tau.
// Each reflector maps its column x to +||x|| e_1, using Parlett's form of the
// leading entry when x_1 > 0 so that no cancellation occurs.
__device__ void wg_geqr2(double* X, int m, int n, double* tau, double* v, double* red,
                         int64_t ld = -1) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  const int kmax = m < n ? m : n;
  if (ld < 0) ld = m;
  for (int j = 0; j < kmax; ++j) {
    double* col = X + (int64_t)j * ld;
    double alpha = col[j];
    double s2 = 0.0;
    for (int r = j + 1 + tid; r < m; r += NT) {
      const double t = col[r];
      s2 += t * t;
    }
    s2 = block_sum(s2, red);
    // Columns whose squares approach the underflow range are handled scaled
    // by their largest magnitude (the reflector depends only on the
    // direction); a column below 2^-1000 counts as zero.
    double scl = 1.0;
    if (s2 > 0.0 && s2 < 0x1p-900 && !(alpha > 0.0 && s2 <= 0x1p-106 * alpha * alpha)) {
      double mx = fabs(alpha);
      for (int r = j + 1 + tid; r < m; r += NT) mx = fmax(mx, fabs(col[r]));
      mx = block_max(mx, red);
      if (mx < 0x1p-1000) {
        s2 = 0.0;
      } else {
        const double inv = 1.0 / mx;
        double t2 = 0.0;
        for (int r = j + 1 + tid; r < m; r += NT) {
          const double t = col[r] * inv;
          t2 += t * t;
        }
        s2 = block_sum(t2, red);
        alpha *= inv;
        scl = mx;
      }
    }
    double tj, beta, inv_v0;
    // s2 at most (2^-53 alpha)^2 with alpha > 0: the column already points
    // along e_j to working accuracy, and Parlett's form of the leading entry
    // would divide by a value of order s2 / alpha; the identity is taken (the
    // dropped part is below the rounding of alpha).
    if (s2 == 0.0 || (alpha > 0.0 && s2 <= 0x1p-106 * alpha * alpha)) {
      inv_v0 = 0.0;
      if (alpha >= 0.0) {
        tj = 0.0;
        beta = alpha;
      } else {
        tj = 2.0;
        beta = -alpha;
      }
    } else {
      const double nrm = sqrt(alpha * alpha + s2);
      const double v0 = (alpha <= 0.0) ? alpha - nrm : -s2 / (alpha + nrm);
      tj = 2.0 * v0 * v0 / (s2 + v0 * v0);
      beta = nrm;
      inv_v0 = 1.0 / v0;
    }
    beta *= scl;
    inv_v0 /= scl;
    for (int r = j + 1 + tid; r < m; r += NT) {
      const double vr = col[r] * inv_v0;
      v[r] = vr;
      col[r] = vr;
    }
    if (tid == 0) {
      v[j] = 1.0;
      col[j] = beta;
      tau[j] = tj;
    }
    __syncthreads();
    if (tj != 0.0) {
      const int r0 = j & ~63;
      for (int c = j + 1 + w; c < n; c += NW) {
        double* xc = X + (int64_t)c * ld;
        double part = 0.0;
        for (int r = r0 + lane; r < m; r += 64)
          if (r >= j) part += v[r] * xc[r];
        part = wave_sum(part);
        const double f = tj * part;
        for (int r = r0 + lane; r < m; r += 64)
          if (r >= j) xc[r] -= f * v[r];
      }
    }
    __syncthreads();
  }
}

// C (M x N) = beta C + alpha A (M x K) B (K x N) in FP64 by the whole
// workgroup, on the FP64 matrix cores (v_mfma_f64_16x16x4f64: a wave
// multiplies a 16 x 4 block of A by a 4 x 16 block of B into a 16 x 16
// accumulator; lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// holds D[4 j + l / 16][l % 16] in its j-th accumulator double).  Element
// (i, k) of A is A[i sai + k sak], (k, j) of B is B[k sbk + j sbj] (type TB,
// widened to FP64) and (i, j) of C is C[i sci + j scj]; C may be in global
// memory or LDS.  TM x TN output tiles (64 x 64, or 128 x 32 for products
// only a few columns wide): the eight waves form a 4 x 2 grid, each owning
// TM/64 x TN/32 accumulator blocks.  K goes through LDS GK at a time, the next
// chunk's loads (clamped in-bounds addresses, mapped so the unit-stride index
// runs across lanes) held in registers while the current one is multiplied.
// beta == 0 never reads C.  `lds` holds GEMM_LDS doubles.  Ends with a barrier.
constexpr int GK = 32;
constexpr int GEMM_LDS = GK * (128 + 1) + GK * (64 + 1);
typedef double dbl4 __attribute__((ext_vector_type(4)));
template <int TM, int TN, typename TB>
__device__ void wg_gemm_t(int M, int N, int K, double alpha, const double* A, int64_t sai,
                          int64_t sak, const TB* B, int64_t sbk, int64_t sbj, double beta,
                          double* C, int64_t sci, int64_t scj, double* lds) {
  static_assert((TM == 64 || TM == 128) && (TN == 32 || TN == 64), "tile shapes");
  constexpr int WR = TM / 64, CB = TN / 32;          // accumulator blocks per wave
  constexpr int ALD = TM + 1, BLD = TN + 1;
  constexpr int NA = TM * GK / NT, NB = TN * GK / NT;  // loads per thread and chunk
  static_assert(GK * (ALD + BLD) <= GEMM_LDS, "LDS tiles");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w & 3, wc = w >> 2;
  const int r16 = lane & 15, q4 = lane >> 4;
  double* As = lds;             // As[k * ALD + i]
  double* Bs = lds + GK * ALD;  // Bs[k * BLD + j]
  const bool a_ifast = sai == 1, b_jfast = sbj == 1;
  int ai[NA], ak[NA], bk[NB], bj[NB];
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    const int e = tid + t * NT;
    ai[t] = a_ifast ? (e % TM) : (e / GK);
    ak[t] = a_ifast ? (e / TM) : (e % GK);
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int e = tid + t * NT;
    bj[t] = b_jfast ? (e % TN) : (e / GK);
    bk[t] = b_jfast ? (e / TN) : (e % GK);
  }
  for (int i0 = 0; i0 < M; i0 += TM) {
    for (int j0 = 0; j0 < N; j0 += TN) {
      dbl4 acc[WR][CB];
#pragma unroll
      for (int a = 0; a < WR; ++a)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[a][c] = dbl4{0.0, 0.0, 0.0, 0.0};
      double av[NA], bv[NB];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < NA; ++t) {
          const bool oka = i0 + ai[t] < M && k0 + ak[t] < K;
          const double va = A[oka ? (int64_t)(i0 + ai[t]) * sai + (int64_t)(k0 + ak[t]) * sak : 0];
          av[t] = oka ? va : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const bool okb = j0 + bj[t] < N && k0 + bk[t] < K;
          const double vb =
              (double)B[okb ? (int64_t)(k0 + bk[t]) * sbk + (int64_t)(j0 + bj[t]) * sbj : 0];
          bv[t] = okb ? vb : 0.0;
        }
      };
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int t = 0; t < NA; ++t) As[ak[t] * ALD + ai[t]] = av[t];
#pragma unroll
        for (int t = 0; t < NB; ++t) Bs[bk[t] * BLD + bj[t]] = bv[t];
        __syncthreads();
        if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
          const int k = kk + q4;
          double b[CB];
#pragma unroll
          for (int c = 0; c < CB; ++c) b[c] = Bs[k * BLD + wc * (TN / 2) + c * 16 + r16];
#pragma unroll
          for (int a = 0; a < WR; ++a) {
            const double x = As[k * ALD + wr * (TM / 4) + a * 16 + r16];
#pragma unroll
            for (int c = 0; c < CB; ++c)
              acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, b[c], acc[a][c], 0, 0, 0);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < WR; ++a)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int i = i0 + wr * (TM / 4) + a * 16 + 4 * jj + q4;
            const int j = j0 + wc * (TN / 2) + c * 16 + r16;
            if (i < M && j < N) {
              double* cp = C + (int64_t)i * sci + (int64_t)j * scj;
              *cp = alpha * acc[a][c][jj] + (beta != 0.0 ? beta * *cp : 0.0);
            }
          }
    }
  }
  __syncthreads();
}

// C (M x N) = A^T B for a long reduction dimension K, with A (K x M, element
// (k, i) at A[i lda + k]) and B (K x N, element (k, j) at B[j ldb + k]),
// M <= 16 MB, N <= 16 NBK, on the FP64 matrix cores without LDS staging: the
// waves take interleaved 16-deep slices of K, each loading its MFMA operands
// straight from memory (four k-steps in flight) and accumulating all of C;
// the partial results are then added into acc (LDS, row-major, ld 16 NBK)
// one wave after the other, in wave order, so the result does not depend on
// timing.  Within a slice, the lanes of one row (or column) group read four
// consecutive k each, so a slice of a row is one contiguous 128-byte run; A
// and B use the same k order, so the sum is unchanged.  Ends with a barrier.
template <int MB, int NBK>
__device__ void wg_atb(int M, int N, int K, const double* __restrict__ A, int64_t lda,
                       const double* __restrict__ B, int64_t ldb, double* acc) {
  constexpr int LDC = 16 * NBK;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  dbl4 c[MB][NBK];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NBK; ++j) c[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 16 * w; k0 < K; k0 += 16 * NW) {
    // each lane reads its four consecutive k (two 16-byte loads when all four
    // are in range), so a load instruction covers whole 128-byte lines
    const int kb = k0 + 4 * q4;
    double a[MB][4], b[NBK][4];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const int row = 16 * i + r16;
      const double* p = A + (int64_t)(row < M ? row : 0) * lda + kb;
      if (row < M && kb + 3 < K) {
        double2 u0, u1;
        __builtin_memcpy(&u0, p, 16);
        __builtin_memcpy(&u1, p + 2, 16);
        a[i][0] = u0.x;
        a[i][1] = u0.y;
        a[i][2] = u1.x;
        a[i][3] = u1.y;
      } else {
#pragma unroll
        for (int st = 0; st < 4; ++st) a[i][st] = (row < M && kb + st < K) ? p[st] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < NBK; ++j) {
      const int col = 16 * j + r16;
      const double* p = B + (int64_t)(col < N ? col : 0) * ldb + kb;
      if (col < N && kb + 3 < K) {
        double2 u0, u1;
        __builtin_memcpy(&u0, p, 16);
        __builtin_memcpy(&u1, p + 2, 16);
        b[j][0] = u0.x;
        b[j][1] = u0.y;
        b[j][2] = u1.x;
        b[j][3] = u1.y;
      } else {
#pragma unroll
        for (int st = 0; st < 4; ++st) b[j][st] = (col < N && kb + st < K) ? p[st] : 0.0;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NBK; ++j)
          c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][st], b[j][st], c[i][j], 0, 0, 0);
  }
  __syncthreads();   // acc may still be read by the caller's previous step
  for (int q = 0; q < NW; ++q) {
    if (w == q) {
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NBK; ++j)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int row = 16 * i + 4 * jj + q4, col = 16 * j + r16;
            if (row < 16 * MB && col < LDC)
              acc[row * LDC + col] = (q == 0 ? 0.0 : acc[row * LDC + col]) + c[i][j][jj];
          }
    }
    __syncthreads();
  }
}

// C (mp x N, column-major, ld ldc) += alpha A B with A (mp x KK, column-major,
// ld lda), KK <= 32, and B small (element (k, j) at B[k sbk + j sbj], usually
// LDS), N <= 16 NBK, on the FP64 matrix cores: each wave takes 16-row blocks
// of C in turn, with no barrier.  The caller orders B's writes before the call
// and C's use after it.
template <int NBK>
__device__ void wg_ab_rows(int mp, int N, int KK, double alpha, const double* __restrict__ A,
                           int64_t lda, const double* B, int sbk, int sbj, double* C,
                           int64_t ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  // the 16 x 16 blocks are formed transposed, C^T = B^T A^T, so that a lane's
  // four results are four columns of one row and every read-modify-write
  // instruction covers 16 consecutive rows of four columns; B (small, usually
  // LDS) is read at each product rather than held, to leave registers for the
  // old values of C
  for (int r0 = 16 * w; r0 < mp; r0 += 16 * NW) {
    const int row = r0 + r16;
    // the old values of C are loaded first, so their reads overlap the products
    double old[NBK][4];
#pragma unroll
    for (int j = 0; j < NBK; ++j)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int col = 16 * j + 4 * jj + q4;
        const bool ok = row < mp && col < N;
        const double v = C[ok ? (int64_t)col * ldc + row : 0];
        old[j][jj] = v;
      }
    double av[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int k = 4 * st + q4;
      const bool ok = k < KK && row < mp;
      const double v = A[ok ? (int64_t)k * lda + row : 0];
      av[st] = ok ? v : 0.0;   // A^T[k][row]
    }
    dbl4 c[NBK];
#pragma unroll
    for (int j = 0; j < NBK; ++j) c[j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int k = 4 * st + q4;
#pragma unroll
      for (int j = 0; j < NBK; ++j) {
        const int col = 16 * j + r16;   // B^T[col][k] = B[k][col]
        const double bv = (k < KK && col < N) ? B[k * sbk + col * sbj] : 0.0;
        c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av[st], c[j], 0, 0, 0);
      }
    }
    // c[j][jj] = (A B)[row][16 j + 4 jj + q4]
#pragma unroll
    for (int j = 0; j < NBK; ++j)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int col = 16 * j + 4 * jj + q4;
        if (row < mp && col < N) C[(int64_t)col * ldc + row] = old[j][jj] + alpha * c[j][jj];
      }
  }
}

template <typename TB>
__device__ void wg_gemm(int M, int N, int K, double alpha, const double* A, int64_t sai,
                        int64_t sak, const TB* B, int64_t sbk, int64_t sbj, double beta, double* C,
                        int64_t sci, int64_t scj, double* lds) {
  wg_gemm_t<64, 64, TB>(M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, sci, scj, lds);
}

constexpr int QB = 16;      // block width of the left-to-right pass
constexpr int QBMAX = 32;   // widest block; Ts and Gs are QBMAX x QBMAX

// T of the compact WY form from G = V^T V already in Gs: the forward
// recurrence T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i] (one wave).
// Ends with a barrier.
__device__ void wg_t_from_gram(int jb, const double* tau, double* Ts, const double* Gs) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    for (int i = 0; i < jb; ++i) {
      const double ti = tau[i];
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
}

// Compact WY factor of jb <= QBMAX reflectors held explicitly in Vp (mp x jb,
// column-major, unit diagonal, zeros above it): H_0 ... H_{jb-1} = I - V T V^T
// with T upper triangular (row-major in Ts, ld QBMAX); G = V^T V by the
// split-K matrix-core product (wg_atb) into Gs, then wg_t_from_gram.
__device__ void wg_build_t_splitk(const double* Vp, int mp, int jb, const double* tau, double* Ts,
                                  double* Gs) {
  wg_atb<2, 2>(jb, jb, mp, Vp, mp, Vp, mp, Gs);
  wg_t_from_gram(jb, tau, Ts, Gs);
}

// Blocked Householder QR (same output as wg_geqr2: R on and above the
// diagonal, reflectors below it, tau) of the m x n column-major X (ld ld,
// default m), for
// panels too large for registers.  Each block of QB columns is factorised by
// wg_geqr2; its reflectors are applied to the trailing columns at once in the
// compact WY form H_0 ... H_{b-1} = I - V T V^T (T upper triangular):
//   C <- C - V (C^T V T)^T,  three GEMMs (the two skinny ones in 128 x 32 tiles).
// A panel that fits in lds (lds_cap doubles, at least GEMM_LDS) is factorised
// there; otherwise in place in global memory with v as the LDS vector.
// qb: block width (<= QBMAX).  ws: m qb + 2 qb n doubles of global workspace;
// Ts, Gs: QBMAX x QBMAX doubles each in LDS outside lds.
// A panel too tall for LDS at width qb is itself factorised in QB-wide blocks
// in LDS (NEST) when those fit, else column by column in global memory.
template <bool NEST>
__device__ void wg_geqrf_impl(double* X, int m, int n, double* tau, double* v, double* red,
                              double* ws, double* lds, int64_t lds_cap, double* Ts, double* Gs,
                              int64_t ld, int qb) {
  const int tid = threadIdx.x;
  const int kmax = m < n ? m : n;
  for (int j0 = 0; j0 < kmax; j0 += qb) {
    const int jb = (kmax - j0) < qb ? (kmax - j0) : qb;
    const int mp = m - j0;
    double* P0 = X + (int64_t)j0 * ld + j0;  // panel (mp x jb), ld ld
    const int nc = n - j0 - jb;
    double* Vp = ws;                          // explicit V (mp x jb, column-major)
    if ((int64_t)mp * (jb + 1) <= lds_cap) {
      // factorise the panel in LDS (v in lds[0, mp), panel after it, ld mp)
      double* PL = lds + mp;
      for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
        const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
        PL[e] = P0[(int64_t)c * ld + r];
      }
      __syncthreads();
      wg_geqr2(PL, mp, jb, tau + j0, lds, red, mp);
      for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
        const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
        P0[(int64_t)c * ld + r] = PL[e];
        if (nc > 0) Vp[e] = r > c ? PL[e] : (r == c ? 1.0 : 0.0);
      }
      __syncthreads();
      if (nc <= 0) continue;
    } else {
      if (NEST && jb > QB && (int64_t)mp * (QB + 1) <= lds_cap)
        wg_geqrf_impl<false>(P0, mp, jb, tau + j0, v, red, ws, lds, lds_cap, Ts, Gs, ld, QB);
      else
        wg_geqr2(P0, mp, jb, tau + j0, v, red, ld);
      if (nc <= 0) continue;
      for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
        const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
        Vp[e] = r > c ? P0[(int64_t)c * ld + r] : (r == c ? 1.0 : 0.0);
      }
      __syncthreads();
    }
    // G = V^T V (jb x jb, row-major in LDS), then T by the forward recurrence
    //   T_ii = tau_i,  T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
    wg_gemm<double>(jb, jb, mp, 1.0, Vp, mp, 1, Vp, 1, mp, 0.0, Gs, QBMAX, 1, lds);
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
    double* C = X + (int64_t)(j0 + jb) * ld + j0;  // trailing block (mp x nc), ld ld
    double* Wt = ws + (int64_t)mp * qb;             // W^T = C^T V, nc x jb (ld qb)
    double* Wt2 = Wt + (int64_t)qb * n;             // W^T T, nc x jb (ld qb)
    wg_gemm_t<128, 32, double>(nc, jb, mp, 1.0, C, ld, 1, Vp, 1, mp, 0.0, Wt, qb, 1, lds);
    wg_gemm_t<128, 32, double>(nc, jb, jb, 1.0, Wt, qb, 1, Ts, QBMAX, 1, 0.0, Wt2, qb, 1, lds);
    // C -= V (W^T T)^T
    wg_gemm<double>(mp, nc, jb, -1.0, Vp, 1, mp, Wt2, 1, qb, 1.0, C, 1, ld, lds);
  }
  __syncthreads();
}

__device__ void wg_geqrf(double* X, int m, int n, double* tau, double* v, double* red, double* ws,
                         double* lds, int64_t lds_cap, double* Ts, double* Gs, int64_t ld = -1,
                         int qb = QB) {
  wg_geqrf_impl<true>(X, m, n, tau, v, red, ws, lds, lds_cap, Ts, Gs, ld < 0 ? m : ld, qb);
}

// Y <- H_0 H_1 ... H_{k-1} Y for the m x s column-major Y (ld m), with the
// reflectors stored as by wg_geqr2 in V (ld ldv, default m).  One wave per column of Y;
// columns are independent, so no barrier is needed between reflectors.
__device__ void wg_apply_q(const double* V, const double* tau, int m, int k, double* Y, int s,
                           int64_t ldv = -1) {
  const int lane = threadIdx.x & 63, w = wave_id();
  if (ldv < 0) ldv = m;
  for (int c = w; c < s; c += NW) {
    double* yc = Y + (int64_t)c * m;
    for (int j = k - 1; j >= 0; --j) {
      const double tj = tau[j];
      if (tj == 0.0) continue;
      const double* vj = V + (int64_t)j * ldv;
      const int r0 = j & ~63;
      double part = 0.0;
      for (int r = r0 + lane; r < m; r += 64) {
        if (r == j) part += yc[r];
        else if (r > j) part += vj[r] * yc[r];
      }
      part = wave_sum(part);
      const double f = tj * part;
      for (int r = r0 + lane; r < m; r += 64) {
        if (r == j) yc[r] -= f;
        else if (r > j) yc[r] -= f * vj[r];
      }
    }
  }
  __syncthreads();
}

// One-sided Jacobi (Hestenes 1958): rotate the nv vectors b_k = B + k*ldb (length
// len) pairwise until they are mutually orthogonal to working accuracy, and
// accumulate the rotations in U (nv x nv, column-major).  Pairs follow the
// round-robin (circle) ordering so a round's pairs are disjoint and each is
// handled by one wave.  Returns the number of sweeps.
__device__ int wg_jacobi(double* B, int nv, int len, int ldb, double* U, int* flag, double* red,
                          double skip2 = 0.0) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  for (int t = tid; t < nv * nv; t += NT) U[t] = ((t % nv) == (t / nv)) ? 1.0 : 0.0;
  __syncthreads();
  if (nv < 2) return 0;
  // Vectors whose norm is below 16 eps |B|_F (rotations keep |B|_F) are
  // rounding noise, e.g. the null space when nv > len; rotating them cannot
  // change any singular value above that level, and their relative
  // orthogonality would never converge, so pairs with one are left alone.
  double part = 0.0;
  for (int e = tid; e < nv * len; e += NT) {
    const double x = B[(int64_t)(e / len) * ldb + e % len];
    part += x * x;
  }
  const double tiny = 256.0 * 4.930380657631324e-32 * block_sum(part, red);
  // A pair whose squared norms sum to at most skip2 (the caller passes
  // delta^2 / nv when the rank will be cut at tail delta^2) needs no rotation:
  // every vector that small ends in the discarded tail (nv of them sum to at
  // most delta^2), and the tail's Frobenius norm does not depend on rotations
  // among its vectors.
  // Convergence threshold len * eps on |<b_p,b_q>| / (|b_p| |b_q|): above the
  // rounding level of the computed inner products, so a converged pair is
  // never rotated again and the sweep count stays small.
  const double tol = 2.220446049250313e-16 * (double)(len > 16 ? len : 16);
  const int nn = nv + (nv & 1);
  // More pairs per round than waves and short vectors: one 16-lane row of a
  // wave per pair (32 pairs at once), row sums by DPP shifts within the row.
  const bool rows16 = nn / 2 > NW && len <= 256;
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    if (rows16) {
      const int g = tid >> 4, r16 = tid & 15, src = (lane & ~15) | 15;
      for (int rnd = 0; rnd < nn - 1; ++rnd) {
        for (int t = g; t < nn / 2; t += NT / 16) {
          int p, q;
          if (t == 0) {
            p = nn - 1;
            q = rnd;
          } else {
            p = (rnd + t) % (nn - 1);
            q = (rnd - t + nn - 1) % (nn - 1);
          }
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q >= nv) continue;
          double* bp = B + (int64_t)p * ldb;
          double* bq = B + (int64_t)q * ldb;
          double a = 0.0, b = 0.0, c = 0.0;
          for (int e = r16; e < len; e += 16) {
            const double x = bp[e], y = bq[e];
            a += x * x;
            b += y * y;
            c += x * y;
          }
          a = row16_sum(a, src);
          b = row16_sum(b, src);
          c = row16_sum(c, src);
          if (a <= tiny || b <= tiny || a + b <= skip2 || fabs(c) <= tol * sqrt(a) * sqrt(b))
            continue;
          const double zeta = (b - a) / (2.0 * c);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          for (int e = r16; e < len; e += 16) {
            const double x = bp[e], y = bq[e];
            bp[e] = cs * x - sn * y;
            bq[e] = sn * x + cs * y;
          }
          double* up = U + (int64_t)p * nv;
          double* uq = U + (int64_t)q * nv;
          for (int e = r16; e < nv; e += 16) {
            const double x = up[e], y = uq[e];
            up[e] = cs * x - sn * y;
            uq[e] = sn * x + cs * y;
          }
          if (r16 == 0) *flag = 1;
        }
        __syncthreads();
      }
      const int any = *flag;
      __syncthreads();
      if (!any) break;
      continue;
    }
    for (int rnd = 0; rnd < nn - 1; ++rnd) {
      for (int t = w; t < nn / 2; t += NW) {
        int p, q;
        if (t == 0) {
          p = nn - 1;
          q = rnd;
        } else {
          p = (rnd + t) % (nn - 1);
          q = (rnd - t + nn - 1) % (nn - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q >= nv) continue;
        double* bp = B + (int64_t)p * ldb;
        double* bq = B + (int64_t)q * ldb;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = lane; r < len; r += 64) {
          const double x = bp[r], y = bq[r];
          a += x * x;
          b += y * y;
          c += x * y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        if (a <= tiny || b <= tiny || a + b <= skip2 || fabs(c) <= tol * sqrt(a) * sqrt(b))
          continue;
        const double zeta = (b - a) / (2.0 * c);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int r = lane; r < len; r += 64) {
          const double x = bp[r], y = bq[r];
          bp[r] = cs * x - sn * y;
          bq[r] = sn * x + cs * y;
        }
        double* up = U + (int64_t)p * nv;
        double* uq = U + (int64_t)q * nv;
        for (int r = lane; r < nv; r += 64) {
          const double x = up[r], y = uq[r];
          up[r] = cs * x - sn * y;
          uq[r] = sn * x + cs * y;
        }
        if (lane == 0) *flag = 1;
      }
      __syncthreads();
    }
    const int any = *flag;
    __syncthreads();
    if (!any) break;
  }
  return sweep;
}

// The same one-sided Jacobi for the left-to-right pass, with each pair's
// vectors held in registers between the inner products and the rotation, and
// B and U addressed as LDS when they live there (ds reads the compiler can
// batch, instead of flat accesses that wait on both memory counters).  A
// pair takes one 16-lane DPP row (LN = 16, 32 pairs at once) or one wave
// (LN = 64); lane li holds elements li + LN i (i < E) of the two vectors and
// li + LN i (i < EU) of their rotation rows.  Same pairs, rotations and
// stopping rule as wg_jacobi, with the orthogonality test taken on squares.
typedef __attribute__((address_space(3))) double lds_double;
template <bool L>
struct jac_ptr {
  using type = double*;
};
template <>
struct jac_ptr<true> {
  using type = lds_double*;
};

template <int LN, int E, int EU, bool BL, bool UL, bool ACC = true>
__device__ int jacobi_regs(double* Bg, int nv, int len, int ldb, double* Ug, int* flag,
                           double tiny, double skip2, double tol) {
  using PB = typename jac_ptr<BL>::type;
  using PU = typename jac_ptr<UL>::type;
  PB B = (PB)Bg;
  PU U = (PU)Ug;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = tid / LN, li = tid & (LN - 1);
  constexpr int NG = NT / LN;
  const int src = (lane & ~15) | 15;
  const double tol2 = tol * tol;
  const int nn = nv + (nv & 1);
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int rnd = 0; rnd < nn - 1; ++rnd) {
      for (int t = g; t < nn / 2; t += NG) {
        int p, q;
        if (t == 0) {
          p = nn - 1;
          q = rnd;
        } else {
          p = (rnd + t) % (nn - 1);
          q = (rnd - t + nn - 1) % (nn - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q >= nv) continue;
        PB bp = B + (int64_t)p * ldb;
        PB bq = B + (int64_t)q * ldb;
        // the rotation rows are loaded with the vectors, off the path that
        // waits for the sums
        PU up = nullptr, uq = nullptr;
        double ux[ACC ? EU : 1], uy[ACC ? EU : 1];
        if constexpr (ACC) {
          up = U + (int64_t)p * nv;
          uq = U + (int64_t)q * nv;
#pragma unroll
          for (int i = 0; i < EU; ++i) {
            const int e = li + LN * i;
            const bool ok = e < nv;
            ux[i] = up[ok ? e : 0];
            uy[i] = uq[ok ? e : 0];
          }
        }
        double x[E], y[E];
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int e = li + LN * i;
          const bool ok = e < len;
          const double xv = bp[ok ? e : 0], yv = bq[ok ? e : 0];
          x[i] = ok ? xv : 0.0;
          y[i] = ok ? yv : 0.0;
          a += x[i] * x[i];
          b += y[i] * y[i];
          c += x[i] * y[i];
        }
        if constexpr (LN == 16)
          row16_sum3(a, b, c, src);
        else
          wave_sum3(a, b, c);
        if (a <= tiny || b <= tiny || a + b <= skip2 || c * c <= tol2 * a * b) continue;
        const double zeta = (b - a) / (2.0 * c);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = rsqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int e = li + LN * i;
          if (e < len) {
            bp[e] = cs * x[i] - sn * y[i];
            bq[e] = sn * x[i] + cs * y[i];
          }
        }
        if constexpr (ACC) {
#pragma unroll
          for (int i = 0; i < EU; ++i) {
            const int e = li + LN * i;
            if (e < nv) {
              up[e] = cs * ux[i] - sn * uy[i];
              uq[e] = sn * ux[i] + cs * uy[i];
            }
          }
        }
        if (li == 0) *flag = 1;
      }
      __syncthreads();
    }
    const int any = *flag;
    __syncthreads();
    if (!any) break;
  }
  return sweep;
}

template <bool BL, bool UL>
__device__ int jacobi_pick(double* B, int nv, int len, int ldb, double* U, int* flag, double tiny,
                           double skip2, double tol) {
  const int nn = nv + (nv & 1);
  const int mx = len > nv ? len : nv;
  if (nn / 2 > NW) {
    if (mx <= 64) return jacobi_regs<16, 4, 4, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
    if (mx <= 128) return jacobi_regs<16, 8, 8, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
    return jacobi_regs<16, 16, 16, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  }
  if (mx <= 64) return jacobi_regs<64, 1, 1, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  if (mx <= 128) return jacobi_regs<64, 2, 2, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  return jacobi_regs<64, 4, 4, BL, UL>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
}

// wg_jacobi for vectors of at most 256 entries (b_lds / u_lds: B / U lie in
// LDS); longer ones take wg_jacobi itself.  jacobi_rows_lr: the same on the
// nv rows (of len <= 256 entries) of B in LDS without accumulating the
// rotations (U unused).
__device__ int wg_jacobi_lr(double* B, int nv, int len, int ldb, double* U, int* flag,
                            double* red, double skip2, bool b_lds, bool u_lds) {
  if (len > 256 || nv > 256) return wg_jacobi(B, nv, len, ldb, U, flag, red, skip2);
  const int tid = threadIdx.x;
  for (int t = tid; t < nv * nv; t += NT) U[t] = ((t % nv) == (t / nv)) ? 1.0 : 0.0;
  __syncthreads();
  if (nv < 2) return 0;
  double part = 0.0;
  for (int e = tid; e < nv * len; e += NT) {
    const double x = B[(int64_t)(e / len) * ldb + e % len];
    part += x * x;
  }
  const double tiny = 256.0 * 4.930380657631324e-32 * block_sum(part, red);
  const double tol = 2.220446049250313e-16 * (double)(len > 16 ? len : 16);
  if (b_lds && u_lds) return jacobi_pick<true, true>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  if (b_lds) return jacobi_pick<true, false>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  if (u_lds) return jacobi_pick<false, true>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
  return jacobi_pick<false, false>(B, nv, len, ldb, U, flag, tiny, skip2, tol);
}

__device__ int jacobi_rows_lr(double* B, int nv, int len, int ldb, int* flag, double* red,
                              double skip2) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (nv < 2) return 0;
  double part = 0.0;
  for (int e = tid; e < nv * len; e += NT) {
    const double x = B[(int64_t)(e / len) * ldb + e % len];
    part += x * x;
  }
  const double tiny = 256.0 * 4.930380657631324e-32 * block_sum(part, red);
  const double tol = 2.220446049250313e-16 * (double)(len > 16 ? len : 16);
  const int nn = nv + (nv & 1);
  if (nn / 2 > NW) {
    if (len <= 64)
      return jacobi_regs<16, 4, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                       tol);
    if (len <= 128)
      return jacobi_regs<16, 8, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                       tol);
    return jacobi_regs<16, 16, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                      tol);
  }
  if (len <= 64)
    return jacobi_regs<64, 1, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                     tol);
  if (len <= 128)
    return jacobi_regs<64, 2, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                     tol);
  return jacobi_regs<64, 4, 1, true, false, false>(B, nv, len, ldb, nullptr, flag, tiny, skip2,
                                                   tol);
}

// Norms of the nv vectors, then a stable descending sort: sig[pos], perm[pos].
__device__ void wg_norms_sorted(const double* B, int nv, int len, int ldb, double* sig, int* perm,
                                double* nrm) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  for (int k = w; k < nv; k += NW) {
    const double* bk = B + (int64_t)k * ldb;
    double part = 0.0;
    for (int r = lane; r < len; r += 64) part += bk[r] * bk[r];
    part = wave_sum(part);
    if (lane == 0) nrm[k] = sqrt(part);
  }
  __syncthreads();
  for (int k = tid; k < nv; k += NT) {
    const double sk = nrm[k];
    int pos = 0;
    for (int j = 0; j < nv; ++j) {
      const double sj = nrm[j];
      if (sj > sk || (sj == sk && j < k)) ++pos;
    }
    perm[pos] = k;
    sig[pos] = sk;
  }
  __syncthreads();
}

// Sign of the entry of largest magnitude (first one on ties) of x[0..n).
__device__ inline double sign_of_max(const double* x, int n, int stride) {
  double best = -1.0, val = 1.0;
  for (int r = 0; r < n; ++r) {
    const double a = fabs(x[(int64_t)r * stride]);
    if (a > best) {
      best = a;
      val = x[(int64_t)r * stride];
    }
  }
  return val < 0.0 ? -1.0 : 1.0;
}

}  // namespace

}  // namespace tnr
