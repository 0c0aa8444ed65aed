// FP64 sweeps of the TNrSVD hot path on gfx950.
//
// ROUND + ORTH of a product MPS (Sec. 3 rounding fused with Algorithm 5.2 as
// described in Sec. 5.4, mirrored so that the K leg sits on the last core):
//   k_rl_pass  right-to-left: absorb L_{i+1} into product core i and take the
//              Householder QR of the transposed panel (= an LQ of the core).
//   k_lr_pass  left-to-right: apply the stored reflectors to the carried
//              factor, one-sided Jacobi SVD of the (s n) x rho panel, rank
//              decision in FP64, then a Householder QR (orthogonalise) or a
//              Jacobi SVD (solve, Algorithm 5.3) of the last core.
// One workgroup handles one MPO for a whole pass, so a batch of independent
// MPOs runs as one persistent launch and a single MPO needs one launch per
// pass.  Every row of a vector is always touched by the same lane (row r is
// owned by lane r % 64), so no cross-lane read-after-write goes through memory
// without a workgroup barrier.
#include <type_traits>

#include "tnrsvd_internal.h"
#include "wg_linalg.h"

namespace tnr {

namespace {

// ---------------------------------------------------------------------------
// Register-resident Householder QR (panels up to 256 x 128).
// Layout: lane l of wave w is in 16-lane row g = l / 16 at position h = l % 16;
// o = 4 w + g (0 .. QOWN-1) owns columns o + QOWN u (slots u < QNC) and lane h
// holds rows h + 16 t (t < 16) of them: x[t][u] = X[h + 16 t][o + QOWN u].
// A column's inner product is then a butterfly over one DPP row (4 steps,
// every lane gets the sum), the four rows of a wave work on four columns at
// once, and columns are dealt cyclically so the shrinking trailing matrix
// stays balanced.  One barrier per column step: the owner row builds the
// reflector and publishes it in a double-buffered LDS vector.
// ---------------------------------------------------------------------------
constexpr int QMR = 16;                // row slots    -> 256 rows
constexpr int QOWN = 4 * NW;           // column owners: four 16-lane rows per wave
constexpr int QNC = 128 / QOWN;        // column slots -> 128 columns
constexpr int QROWS = 16 * QMR;
constexpr int QCOLS = QOWN * QNC;
constexpr int ARENA = 19456;           // doubles of static LDS per workgroup (152 KiB)
static_assert(2 * QROWS + QCOLS + QCOLS * QCOLS <= ARENA - 32,
              "register QR: reflector buffers, diagonal, R gather");
static_assert(QOWN * QROWS + QOWN <= QCOLS * QCOLS, "register QR: a block's reflectors in the R gather");

// Sum over the 16 lanes of a DPP row; every lane of the row receives it.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// Two such sums in lockstep (independent DPP chains interleave).
__device__ __forceinline__ void row16_sum2(double& a, double& b) {
  a += dpp_d<0xB1>(a);
  b += dpp_d<0xB1>(b);
  a += dpp_d<0x4E>(a);
  b += dpp_d<0x4E>(b);
  a += dpp_d<0x141>(a);
  b += dpp_d<0x141>(b);
  a += dpp_d<0x140>(a);
  b += dpp_d<0x140>(b);
}

// Compile-time loop: f(integral_constant<int, B>), ..., f(<E - 1>).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Householder reflector of column jj, held in col by the calling owner row
// (Parlett's form: diag(R) >= 0, v[jj] = 1).  Writes v (zeros above the
// diagonal, 1 on it) to LDS, tau to LDS and to tau_g, and the diagonal entry
// of R to bt[jj].  Sums use partial accumulators to keep the dependent FP64
// chains short.
__device__ __forceinline__ void reg_reflect(const double (&col)[QMR], int jj, int m, int h,
                                            double* v, double* tbs, double* tau_g, double* bt) {
  double sq[4] = {0.0, 0.0, 0.0, 0.0}, dg[2] = {0.0, 0.0};
#pragma unroll
  for (int t = 0; t < QMR; ++t) {
    const int r = h + 16 * t;
    const double c = col[t];
    const double cm = (r > jj && r < m) ? c : 0.0;
    sq[t & 3] += cm * cm;
    dg[t & 1] += (r == jj) ? c : 0.0;
  }
  double s2 = (sq[0] + sq[1]) + (sq[2] + sq[3]);
  double al = dg[0] + dg[1];
  row16_sum2(s2, al);
  double tj, beta, inv_v0;
  if (s2 == 0.0) {
    inv_v0 = 0.0;
    if (al >= 0.0) {
      tj = 0.0;
      beta = al;
    } else {
      tj = 2.0;
      beta = -al;
    }
  } else {
    // v0 = al - nrm (for al > 0 as -s2 / (al + nrm), without cancellation);
    // 1 / v0 and tau = 2 v0^2 / (s2 + v0^2) = -v0 / nrm are both formed from
    // nrm, so a single division lies on the path to v
    const double nrm = sqrt(al * al + s2);
    if (al <= 0.0) {
      const double v0 = al - nrm;
      inv_v0 = 1.0 / v0;
      tj = -v0 / nrm;
    } else {
      const double ap = al + nrm;
      inv_v0 = -ap / s2;
      tj = s2 / (ap * nrm);
    }
    beta = nrm;
  }
#pragma unroll
  for (int t = 0; t < QMR; ++t) {
    const int r = h + 16 * t;
    const bool below = r > jj && r < m;
    v[r] = below ? col[t] * inv_v0 : (r == jj ? 1.0 : 0.0);
  }
  if (h == 0) {
    tbs[0] = tj;
    tau_g[jj] = tj;
    bt[jj] = beta;
  }
}

// Householder QR of the register panel, blocked by column slots: block ub is
// the columns 32 ub .. 32 ub + 31 (slot ub of every owner row).  Within a
// block, one barrier per column step: the owner of column j + 1 builds its
// reflector (look-ahead) as soon as reflector j has updated it, and only the
// block's own columns are updated step by step.  The reflectors of the block
// stay in LDS (over the R gather buffer, free until the end) and are then
// applied in order to the columns right of the block, with no barrier between
// them; the next block starts after one barrier.  Every column still receives
// the reflectors in the unblocked order, so the arithmetic per element is the
// same.  A wave that does not hold column j + 1 copies reflector j from LDS to
// V (column-major, ld ldv, whole column: zeros above the diagonal, 1 on it).
// R (row-major k x n, k = min(m, n), zero lower triangle) is read off the
// registers at the end: rows above the diagonal of column c are final once
// reflectors 0..c-1 are applied, the diagonal comes from bt.  It is gathered in
// LDS (Rl, k n doubles) and written out coalesced.
__device__ __forceinline__ void reg_geqr(double (&x)[QMR][QNC], int m, int n, double* tau_g,
                                         double* V, int ldv, double* R, double* bt, double* Rl) {
  const int tid = threadIdx.x, lane = tid & 63, h = lane & 15, g = lane >> 4;
  const int w = wave_id();
  const int o = 4 * w + g;
  const int kmax = m < n ? m : n;
  double* Vk = Rl;                    // QOWN reflectors of QROWS rows
  double* Tk = Rl + QOWN * QROWS;     // and their scalars
  static_for<0, QNC>([&](auto UB) {
    constexpr int ub = decltype(UB)::value;
    constexpr int j0 = QOWN * ub;
    if (j0 >= kmax) return;
    const int jend = (j0 + QOWN) < kmax ? (j0 + QOWN) : kmax;
    // the previous block's reflectors are no longer read
    if (ub > 0) lds_barrier();
    if (o == 0) {
      double col[QMR];
#pragma unroll
      for (int t = 0; t < QMR; ++t) col[t] = x[t][ub];
      reg_reflect(col, j0, m, h, Vk, Tk, tau_g, bt);
    }
    for (int j = j0; j < jend; ++j) {
      lds_barrier();
      const int k = j - j0;
      const double tj = Tk[k];
      const double* vh = Vk + k * QROWS + h;
      const int jn = j + 1;
      const bool la = jn < jend && ((jn - j0) >> 2) == w;   // this wave holds column j + 1
      if (!la && w == (((k >> 2) + NW / 2) % NW)) {
        // reflector j to global memory (rows lane + 64 r)
        double* Vc = V + j * ldv;
#pragma unroll
        for (int r4 = 0; r4 < QROWS / 64; ++r4) {
          const int r = lane + 64 * r4;
          if (r < m) Vc[r] = vh[r - h];
        }
      }
      // some column of this wave in slot ub lies right of j (wave uniform)
      if (4 * w + 3 + j0 > j && 4 * w + j0 < n) {
        const int c = o + j0;
        if (tj != 0.0) {
          // four partial sums shorten the dependent FP64 chain
          double ac4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < QMR; ++t) ac4[t & 3] += vh[16 * t] * x[t][ub];
          const double acc = row16_sum((ac4[0] + ac4[1]) + (ac4[2] + ac4[3]));
          const double f = (c > j && c < n) ? tj * acc : 0.0;
#pragma unroll
          for (int t = 0; t < QMR; ++t) x[t][ub] -= f * vh[16 * t];
        }
        if (la && o == jn - j0) {
          double col[QMR];
#pragma unroll
          for (int t = 0; t < QMR; ++t) col[t] = x[t][ub];
          reg_reflect(col, jn, m, h, Vk + (k + 1) * QROWS, Tk + k + 1, tau_g, bt);
        }
      }
    }
    // the block's reflectors, in order, to the columns right of it (every
    // reflector was published before the last step's barrier)
    const int nb = jend - j0;
    static_for<ub + 1, QNC>([&](auto U) {
      constexpr int u = decltype(U)::value;
      if (4 * w + QOWN * u < n) {
        const bool live = o + QOWN * u < n;
        for (int k = 0; k < nb; ++k) {
          // compiler-only fence: the reflector is re-read from LDS for every
          // slot instead of being held in 16 more registers
          asm volatile("" ::: "memory");
          const double tk = Tk[k];
          if (tk != 0.0) {
            const double* vh = Vk + k * QROWS + h;
            double ac4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < QMR; ++t) ac4[t & 3] += vh[16 * t] * x[t][u];
            const double acc = row16_sum((ac4[0] + ac4[1]) + (ac4[2] + ac4[3]));
            const double f = live ? tk * acc : 0.0;
#pragma unroll
            for (int t = 0; t < QMR; ++t) x[t][u] -= f * vh[16 * t];
          }
        }
      }
    });
  });
  lds_barrier();
  // R off the registers: rows above the diagonal as they stand, the diagonal
  // from bt, zeros below
#pragma unroll
  for (int t = 0; t < QMR; ++t) {
    const int r = h + 16 * t;
#pragma unroll
    for (int u = 0; u < QNC; ++u) {
      const int c = o + QOWN * u;
      if (r < kmax && c < n) Rl[r * n + c] = r < c ? x[t][u] : (r == c ? bt[c] : 0.0);
    }
  }
  lds_barrier();
  for (int e = tid; e < kmax * n; e += NT) R[e] = Rl[e];
}


// Rows [r0, r0 + mr) of the last core's panel (no absorption):
// x[t][u] = Z[p][r0 + r], the panel row being (y, kappa) of an m-row panel.
template <typename T>
__device__ __forceinline__ void reg_load_plain(double (&x)[QMR][QNC], const T* __restrict__ Zc, int m, int P,
                               int r0 = 0, int mr = -1) {
  const int lane = threadIdx.x & 63, h = lane & 15, g = lane >> 4;
  const int o = 4 * wave_id() + g;
  if (mr < 0) mr = m;
  // branch-free: every load has a clamped in-bounds address, so all of them
  // are in flight before the first use; out-of-range elements are zeroed after
  const T* base = Zc + r0;
#pragma unroll
  for (int t = 0; t < QMR; ++t) {
    const int r = h + 16 * t;
#pragma unroll
    for (int u = 0; u < QNC; ++u) {
      const int c = o + QOWN * u;
      const bool ok = r < mr && c < P;
      const double val = (double)base[ok ? c * m + r : 0];   // 32-bit in-core index
      x[t][u] = ok ? val : 0.0;
    }
  }
}

// Absorbed panel Zt^T = (Z x_3 L)^T in the padded layout: slot t holds
// y = t / SPY and f = h + 16 (t % SPY) (each y block padded to 16 SPY rows):
//   x[t][u] = sum_{q >= f} R[f][q] Z[p_u][y][q],  L = R^T (rho x Pn, row-major),
// p_u = o + QOWN u.  Chunks of q are staged in LDS as RT[q][f] and ZL[q][y][p].
template <typename T, int SPY>
__device__ __forceinline__ void reg_absorb(double (&x)[QMR][QNC], const T* __restrict__ Zc, int P, int n, int Pn,
                           const double* __restrict__ Rn, int rho, double* stage, int stage_cap) {
  const int tid = threadIdx.x, lane = tid & 63, h = lane & 15, g = lane >> 4;
  const int o = 4 * wave_id() + g;
  constexpr int FP = 16 * SPY;
  constexpr int NY = QMR / SPY;
#pragma unroll
  for (int t = 0; t < QMR; ++t)
#pragma unroll
    for (int u = 0; u < QNC; ++u) x[t][u] = 0.0;
  const int per_q = FP + n * QCOLS;
  int QC = stage_cap / per_q;
  if (QC > 32) QC = 32;
  double* RT = stage;
  double* ZL = stage + QC * FP;
  for (int q0 = 0; q0 < Pn; q0 += QC) {
    const int qc = (Pn - q0) < QC ? (Pn - q0) : QC;
    __syncthreads();
    // staging with eight clamped loads in flight per thread
#pragma unroll 1
    for (int e0 = 0; e0 < FP * qc; e0 += 8 * NT) {
      double val[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + tid + k * NT;
        const int f = e / qc, q = q0 + e % qc;
        const bool ok = e < FP * qc && f < rho && q >= f;
        const double raw = Rn[ok ? f * Pn + q : 0];
        val[k] = ok ? raw : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + tid + k * NT;
        if (e < FP * qc) RT[(e % qc) * FP + e / qc] = val[k];
      }
    }
#pragma unroll 1
    for (int e0 = 0; e0 < QCOLS * n * qc; e0 += 8 * NT) {
      double val[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + tid + k * NT;
        const int qq = e % qc, py = e / qc;
        const int y = py % n, p = py / n;
        const bool ok = e < QCOLS * n * qc && p < P;
        const double raw = (double)Zc[ok ? (p * n + y) * Pn + q0 + qq : 0];
        val[k] = ok ? raw : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + tid + k * NT;
        if (e < QCOLS * n * qc) {
          const int qq = e % qc, py = e / qc;
          ZL[(qq * n + py % n) * QCOLS + py / n] = val[k];
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int qq = 0; qq < qc; ++qq) {
      double rv[SPY];
#pragma unroll
      for (int s = 0; s < SPY; ++s) rv[s] = RT[qq * FP + h + 16 * s];
#pragma unroll
      for (int y = 0; y < NY; ++y) {
        if (y < n) {
          const double* zp = ZL + (qq * n + y) * QCOLS + o;
          double z[QNC];
#pragma unroll
          for (int u = 0; u < QNC; ++u) z[u] = zp[QOWN * u];
#pragma unroll
          for (int s = 0; s < SPY; ++s)
#pragma unroll
            for (int u = 0; u < QNC; ++u) x[y * SPY + s][u] += rv[s] * z[u];
        }
      }
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void reg_absorb_dispatch(int spy, double (&x)[QMR][QNC], const T* Zc, int P, int n,
                                    int Pn, const double* Rn, int rho, double* stage, int cap) {
  switch (spy) {
    case 1: reg_absorb<T, 1>(x, Zc, P, n, Pn, Rn, rho, stage, cap); break;
    case 2: reg_absorb<T, 2>(x, Zc, P, n, Pn, Rn, rho, stage, cap); break;
    case 4: reg_absorb<T, 4>(x, Zc, P, n, Pn, Rn, rho, stage, cap); break;
    default: reg_absorb<T, 8>(x, Zc, P, n, Pn, Rn, rho, stage, cap); break;
  }
}

// TSQR of a tall panel (m rows > 256, n <= 128 columns), run by the
// right-to-left pass as register QR jobs: leaf QRs of consecutive 256-row
// chunks (k_rl_leaves, all leaves at once), then a binary tree of merges, each
// the QR of two stacked R factors (k_rl_merge_level per level, the root in the
// last-core phase).  Workspace layout (in the core's W slab):
//   leaf c reflectors   W + c * 256 * n            (column-major, ld = rows of leaf c)
//   merge c reflectors  W + (nc + c) * 256 * n     (ld = rows of node c), c >= 1
//   R of the range led by leaf 0   W + 2 nc 256 n   (row-major; n * n after it unused)
//   taus                W + (2 nc 256 + 2 n) n: leaf c at + c n, merge c at + (nc + c) n
//   R of the range led by leaf c >= 1   W + (2 nc 256 + 2 n) n + 2 nc n + (c - 1) n n
// The final R goes to the L slab; tsqr_apply replays the tree in the
// left-to-right pass.

// TSQR leaves of the last core's tall panel, one workgroup per (MPO, leaf):
// leaf c is the register QR of rows [256 c, 256 c + 256) of the panel.  Its
// reflectors and scalars go where the tree keeps them, its R to Racc
// (leaf 0) or to the slot of leaf c >= 1 after the taus:
//   W + (2 nc 256 + 2 n) n + 2 nc n + (c - 1) n n   (row-major n x n).
// The merge tree then runs level by level.  The test for the TSQR path
// repeats the pass's own, on the same descriptors; other MPOs exit at once.
template <typename T>
__global__ __launch_bounds__(NT) void k_rl_leaves(const MpoDesc* mpos, const CoreDesc* cores,
                                                  int op, const int* pr, const T* __restrict__ Z,
                                                  double* Wd, const int* wflag) {
  __shared__ double arena[ARENA];
  if (wflag && wflag[blockIdx.x]) return;   // taken by the multi-workgroup path
  const MpoDesc md = mpos[blockIdx.x];
  const int i = md.d - 1;
  const CoreDesc cd = cores[md.c0 + i];
  const int n = op == 0 ? cd.I : cd.J;
  const int P = pr[md.r0 + i];
  const int Pn = pr[md.r0 + i + 1];
  const int m = n * md.K;
  if (P < 1 || P > cd.RA * cd.xcap || Pn < 1 || Pn > cd.RA2 * cd.xcap2 || md.K > Pn ||
      m > ARENA - 64 - 2 * QBMAX * QBMAX)
    return;                                   // the pass reports the shape error
  if (!(i > 0 && P <= QCOLS && m > QROWS && m <= 16 * QROWS)) return;
  const int nc = (m + QROWS - 1) / QROWS;
  const int c = blockIdx.y;
  if (c >= nc) return;
  double* Xt = Wd + cd.w_off;
  double* ws_tau = Xt + (int64_t)(2 * nc * QROWS + 2 * P) * P;
  double* Rdst = c == 0 ? Xt + (int64_t)2 * nc * QROWS * P
                        : ws_tau + (int64_t)2 * nc * P + (int64_t)(c - 1) * P * P;
  const int r0 = c * QROWS;
  const int mrows = (m - r0) < QROWS ? (m - r0) : QROWS;
  double x[QMR][QNC];
  reg_load_plain<T>(x, Z + cd.z_off, m, P, r0, mrows);
  reg_geqr(x, mrows, P, ws_tau + (int64_t)c * P,
           Xt + (int64_t)c * QROWS * P, mrows, Rdst, arena + 2 * QROWS,
           arena + 2 * QROWS + QCOLS);
}

// Binary merge tree over the leaves 0 .. nc-1: node c (1 <= c < nc) at level
// l = ctz(c) merges the ranges [c - 2^l, c) and [c, min(c + 2^l, nc)); its
// reflectors and scalars sit in merge slot c.  A range's R is kept in the slot
// of its first leaf (slot 0 = Racc) and has min(P, rows of the range) rows.
// The root is the node c = 2^floor(log2(nc - 1)); levels are processed bottom
// up, and the nodes of one level are independent.
__device__ __forceinline__ int tsqr_rows(int m, int P, int lo, int hi) {
  const int r = (hi * QROWS < m ? hi * QROWS : m) - lo * QROWS;
  return r < P ? r : P;
}

__device__ __forceinline__ int tsqr_root_level(int nc) { return 31 - __clz(nc - 1); }

// Stacks [R of the left range; R of the right range] of node c column-major
// into merge slot c (not yet written) and loads it into the register panel;
// returns its row count.  *Rleft receives the left range's R slot.
__device__ __forceinline__ int tsqr_stack(double (&x)[QMR][QNC], double* Xt, int m, int P,
                                          int nc, int c, double** Rleft) {
  const int l = __ffs(c) - 1, a = c - (1 << l);
  const int hi = (c + (1 << l)) < nc ? (c + (1 << l)) : nc;
  const int kl = tsqr_rows(m, P, a, c), kr = tsqr_rows(m, P, c, hi);
  double* ws_tau = Xt + (int64_t)(2 * nc * QROWS + 2 * P) * P;
  double* Racc = Xt + (int64_t)2 * nc * QROWS * P;
  double* Rleaf = ws_tau + (int64_t)2 * nc * P;
  double* Ra = a == 0 ? Racc : Rleaf + (int64_t)(a - 1) * P * P;
  const double* Rc = Rleaf + (int64_t)(c - 1) * P * P;
  const int mrows = kl + kr;
  double* Vdst = Xt + (int64_t)(nc + c) * QROWS * P;
  for (int e = threadIdx.x; e < mrows * P; e += NT) {
    const int col = e / mrows, r = e % mrows;
    Vdst[e] = r < kl ? Ra[r * P + col] : Rc[(r - kl) * P + col];
  }
  __syncthreads();
  reg_load_plain<double>(x, Vdst, mrows, P);
  __syncthreads();
  *Rleft = Ra;
  return mrows;
}

// One level l below the root of every MPO's merge tree: node j of the level
// (c = (2 j + 1) 2^l) per workgroup.  MPOs whose root is at level l or below,
// or whose last core takes another path, exit at once.
__global__ __launch_bounds__(NT) void k_rl_merge_level(const MpoDesc* mpos, const CoreDesc* cores,
                                                       int op, const int* pr, double* Wd,
                                                       int level, const int* wflag) {
  __shared__ double arena[ARENA];
  if (wflag && wflag[blockIdx.x]) return;
  const MpoDesc md = mpos[blockIdx.x];
  const int i = md.d - 1;
  const CoreDesc cd = cores[md.c0 + i];
  const int n = op == 0 ? cd.I : cd.J;
  const int P = pr[md.r0 + i];
  const int Pn = pr[md.r0 + i + 1];
  const int m = n * md.K;
  if (P < 1 || P > cd.RA * cd.xcap || Pn < 1 || Pn > cd.RA2 * cd.xcap2 || md.K > Pn ||
      m > ARENA - 64 - 2 * QBMAX * QBMAX)
    return;
  if (!(i > 0 && P <= QCOLS && m > QROWS && m <= 16 * QROWS)) return;
  const int nc = (m + QROWS - 1) / QROWS;
  if (level >= tsqr_root_level(nc)) return;
  const int c = (2 * (int)blockIdx.y + 1) << level;
  if (c >= nc) return;
  double* Xt = Wd + cd.w_off;
  double* ws_tau = Xt + (int64_t)(2 * nc * QROWS + 2 * P) * P;
  double x[QMR][QNC];
  double* Rdst;
  const int mrows = tsqr_stack(x, Xt, m, P, nc, c, &Rdst);
  reg_geqr(x, mrows, P, ws_tau + (int64_t)(nc + c) * P,
           Xt + (int64_t)(nc + c) * QROWS * P, mrows, Rdst, arena + 2 * QROWS,
           arena + 2 * QROWS + QCOLS);
}

// ---------------------------------------------------------------------------
// Right-to-left pass: absorb + QR of every core, one workgroup per MPO.
// ldm[i] records the row stride of one y block of core i's panel (rho_{i+1},
// or its multiple of 64 when the padded register layout was used).
// ---------------------------------------------------------------------------
// PH 0 handles the last core only (plain register panel, TSQR or the global
// path); PH 1 handles cores d-2 .. 0 (absorption).  Splitting the pass keeps
// each kernel's register footprint to the paths it can take.
template <typename T, int PH>
__global__ __launch_bounds__(NT) void k_rl_pass(const MpoDesc* mpos, const CoreDesc* cores, int op,
                                                const int* pr, int* rho, int* ldm,
                                                const T* __restrict__ Z, double* Wd, double* L,
                                                double* tau, int* err, const int* wflag,
                                                const int* order) {
  __shared__ double arena[ARENA];
  double* vb = arena;                 // 2 * QROWS (register path) or m (global path)
  double* tb = arena + ARENA - 32;    // 2 doubles
  double* red = arena + ARENA - 16;   // NW doubles
  const int tid = threadIdx.x;
  // workgroups take the MPOs costliest first (order), so that the last ones
  // dispatched are short
  const int b = order ? order[blockIdx.x] : (int)blockIdx.x;
  if (wflag && wflag[b]) return;   // taken by the multi-workgroup path
  const MpoDesc md = mpos[b];
  const int d = md.d;
  if (PH == 0 && tid == 0) rho[md.r0 + d] = md.K;
  int rnext = PH == 0 ? md.K : rho[md.r0 + d - 1];
  const int i_first = PH == 0 ? d - 1 : d - 2;
  const int i_last = PH == 0 ? d - 1 : 0;
  for (int i = i_first; i >= i_last; --i) {
    const CoreDesc cd = cores[md.c0 + i];
    const int n = op == 0 ? cd.I : cd.J;
    const int P = pr[md.r0 + i];
    const int Pn = pr[md.r0 + i + 1];
    const int m = n * rnext;
    if (P < 1 || P > cd.RA * cd.xcap || Pn < 1 || Pn > cd.RA2 * cd.xcap2 || rnext > Pn ||
        m > ARENA - 64 - 2 * QBMAX * QBMAX) {
      if (tid == 0) atomicOr(err, 4);
      return;
    }
    double* Xt = Wd + cd.w_off;
    const T* Zc = Z + cd.z_off;
    const double* Rn = (i < d - 1) ? L + cores[md.c0 + i + 1].l_off : nullptr;
    int spy = 1;   // 16-row slots per y block, a power of two
    while (16 * spy < rnext) spy *= 2;
    const bool reg_abs = PH == 1 && i > 0 && i < d - 1 && P <= QCOLS && spy <= 8 &&
                         n * spy <= QMR && P <= m;
    const bool reg_plain = PH == 0 && i > 0 && P <= QCOLS && m <= QROWS;
    const bool tsqr = PH == 0 && i > 0 && P <= QCOLS && m > QROWS && m <= 16 * QROWS;
    if (reg_abs || reg_plain || tsqr) {
      // One register QR: of the absorbed or plain panel, or for a tall panel
      // the root of the TSQR merge tree (its leaves were factorised by
      // k_rl_leaves and the levels below the root by k_rl_merge_level).
      const int nc = tsqr ? (m + QROWS - 1) / QROWS : 1;
      double* ws_tau = Xt + (int64_t)(2 * nc * QROWS + 2 * P) * P;
      {
        double x[QMR][QNC];   // the register panel
        int mrows, ldv;
        double* Vdst;
        double* Rdst;
        double* taud;
        if (!tsqr) {
          if (reg_abs) {
            reg_absorb_dispatch<T>(spy, x, Zc, P, n, Pn, Rn, rnext, arena + 2 * QROWS,
                                   ARENA - 2 * QROWS - 64);
            mrows = n * spy * 16;
          } else {
            reg_load_plain<T>(x, Zc, m, P);
            mrows = m;
          }
          ldv = mrows;
          Vdst = Xt;
          Rdst = L + cd.l_off;
          taud = tau + cd.tau_off;
        } else {
          const int c = 1 << tsqr_root_level(nc);
          double* unused;
          mrows = tsqr_stack(x, Xt, m, P, nc, c, &unused);
          ldv = mrows;
          Vdst = Xt + (int64_t)(nc + c) * QROWS * P;
          Rdst = L + cd.l_off;
          taud = ws_tau + (int64_t)(nc + c) * P;
        }
        reg_geqr(x, mrows, P, taud, Vdst, ldv, Rdst, arena + 2 * QROWS,
                 arena + 2 * QROWS + QCOLS);
        __syncthreads();
      }
      const int k = m < P ? m : P;
      if (tid == 0) {
        ldm[md.r0 + i] = tsqr ? -nc : (reg_abs ? spy * 16 : rnext);
        rho[md.r0 + i] = k;
      }
      rnext = k;
      __syncthreads();
      continue;
    }
    const int64_t tot = (int64_t)m * P;
    if (PH == 0) {
      // last core: Zt = Z (the K leg is external), stored transposed
      for (int64_t o = tid; o < tot; o += NT) {
        const int p = (int)(o / m), jj = (int)(o % m);
        Xt[o] = (double)Zc[(int64_t)p * m + jj];
      }
    } else {
      // Zt^T[(y, f), p] = sum_q R_{i+1}[f, q] Z[p, y, q]   (L_{i+1} = R_{i+1}^T; R is
      // stored upper triangular with zeros below), one GEMM per y
      for (int y = 0; y < n; ++y)
        wg_gemm<T>(rnext, P, Pn, 1.0, Rn, Pn, 1, Zc + (int64_t)y * Pn, 1, (int64_t)n * Pn, 0.0,
                   Xt + (int64_t)y * rnext, 1, m, arena);
    }
    if (tid == 0) ldm[md.r0 + i] = rnext;
    __syncthreads();
    if (i == 0) break;
    {
      constexpr int RCAP = ARENA - 64 - 2 * QBMAX * QBMAX;   // LDS left for panel and tiles
      const int qb = (int64_t)m * (QBMAX + 1) <= RCAP ? QBMAX : QB;
      wg_geqrf(Xt, m, P, tau + cd.tau_off, vb, red, Xt + tot, arena, RCAP,
               arena + ARENA - 32 - 2 * QBMAX * QBMAX, arena + ARENA - 32 - QBMAX * QBMAX, m, qb);
    }
    const int k = m < P ? m : P;
    double* Ro = L + cd.l_off;
    for (int64_t o = tid; o < (int64_t)k * P; o += NT) {
      const int f = (int)(o / P), qq = (int)(o % P);
      Ro[o] = (qq >= f) ? Xt[(int64_t)qq * m + f] : 0.0;
    }
    if (tid == 0) rho[md.r0 + i] = k;
    rnext = k;
    __syncthreads();
  }
}

// Cooperative copy of n doubles from global memory into LDS with eight loads
// in flight per thread before the first store (hides L2 latency).
__device__ __forceinline__ void stage_copy(double* dst, const double* __restrict__ src, int n) {
  const int tid = threadIdx.x;
  int e = tid;
  for (; e + 7 * NT < n; e += 8 * NT) {
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = src[e + q * NT];
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[e + q * NT] = a[q];
  }
  for (; e < n; e += NT) dst[e] = src[e];
}

// Y <- H_0 ... H_{k-1} Y with the reflectors streamed through LDS in chunks
// (V in global memory, column-major ld m; Y column-major m x s, any memory).
__device__ void wg_apply_q_staged(const double* __restrict__ V, const double* __restrict__ tau,
                                  int m, int k, double* Y, int s, double* stage, int cap,
                                  double* tstage) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = wave_id();
  int CH = cap / m;
  if (CH > 64) CH = 64;
  if (CH < 1) CH = 1;
  for (int hi = k; hi > 0; hi -= CH) {
    const int lo = hi - CH > 0 ? hi - CH : 0;
    const int cnt = hi - lo;
    __syncthreads();
    stage_copy(stage, V + (int64_t)lo * m, cnt * m);
    for (int e = tid; e < cnt; e += NT) tstage[e] = tau[lo + e];
    __syncthreads();
    for (int c = w; c < s; c += NW) {
      double* yc = Y + (int64_t)c * m;
      for (int j = hi - 1; j >= lo; --j) {
        const double tj = tstage[j - lo];
        if (tj == 0.0) continue;
        const double* vj = stage + (int64_t)(j - lo) * m;
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
  }
  __syncthreads();
}

// Y <- H_0 ... H_{k-1} Y with each column of Y held in the registers of one
// wave (row r in lane r % 64, slot r / 64; m <= 64 * MT) and the reflectors
// staged through LDS in chunks.  Rows keep their lane, so the only cross-lane
// traffic is the wave reduction of each reflector's inner product.
template <int MT>
__device__ void wg_apply_q_reg(const double* __restrict__ V, const double* __restrict__ tau, int m,
                               int k, double* Y, int s, double* stage, int cap, double* tstage,
                               int ldy = -1) {
  if (ldy < 0) ldy = m;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = wave_id();
  int CH = cap / m;
  if (CH > 64) CH = 64;
  if (CH < 1) CH = 1;
  for (int cb = 0; cb < s; cb += NW) {
    const int c = cb + w;
    const bool have = c < s;
    double y[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int r = lane + 64 * t;
      const bool ok = have && r < m;
      const double raw = Y[ok ? c * ldy + r : 0];
      y[t] = ok ? raw : 0.0;
    }
    for (int hi = k; hi > 0; hi -= CH) {
      const int lo = hi - CH > 0 ? hi - CH : 0;
      const int cnt = hi - lo;
      __syncthreads();
      stage_copy(stage, V + (int64_t)lo * m, cnt * m);
      for (int e = tid; e < cnt; e += NT) tstage[e] = tau[lo + e];
      __syncthreads();
      if (have) {
        for (int j = hi - 1; j >= lo; --j) {
          const double tj = tstage[j - lo];
          if (tj == 0.0) continue;
          const double* vj = stage + (int64_t)(j - lo) * m;
          // two passes over the staged vector (re-read from LDS) keep the
          // register footprint at one column of Y
          double part = 0.0;
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            const int r = lane + 64 * t;
            const double raw = vj[r < m ? r : m - 1];   // in-bounds read, masked below
            part += ((r > j && r < m) ? raw : (r == j ? 1.0 : 0.0)) * y[t];
          }
          part = wave_sum(part);
          const double f = tj * part;
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            const int r = lane + 64 * t;
            const double raw = vj[r < m ? r : m - 1];
            y[t] -= f * ((r > j && r < m) ? raw : (r == j ? 1.0 : 0.0));
          }
        }
      }
    }
    if (have) {
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int r = lane + 64 * t;
        if (r < m) Y[c * ldy + r] = y[t];
      }
    }
  }
  __syncthreads();
}

// The same product with CPW columns of Y per wave (columns cb + w + NW q of
// each batch of CPW NW columns), so every staged reflector is read once for
// all of them: V has leading dimension ldv (its column j holds reflector j
// below row j), Y leading dimension ldy.
template <int MT, int CPW>
__device__ void wg_apply_q_cols(const double* __restrict__ V, int64_t ldv,
                                const double* __restrict__ tau, int m, int k, double* Y, int ldy,
                                int s, double* stage, int cap, double* tstage) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = wave_id();
  int CH = cap / m;
  if (CH > 64) CH = 64;
  if (CH < 1) CH = 1;
  __syncthreads();   // Y may have just been written by other threads
  for (int cb = 0; cb < s; cb += CPW * NW) {
    double y[CPW][MT];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = cb + w + NW * q;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int r = lane + 64 * t;
        const bool ok = c < s && r < m;
        const double raw = Y[ok ? (int64_t)c * ldy + r : 0];
        y[q][t] = ok ? raw : 0.0;
      }
    }
    for (int hi = k; hi > 0; hi -= CH) {
      const int lo = hi - CH > 0 ? hi - CH : 0;
      const int cnt = hi - lo;
      __syncthreads();
      for (int64_t e = tid; e < (int64_t)cnt * m; e += NT) {
        const int j = (int)(e / m), r = (int)(e - (int64_t)j * m);
        stage[e] = V[(int64_t)(lo + j) * ldv + r];
      }
      for (int e = tid; e < cnt; e += NT) tstage[e] = tau[lo + e];
      __syncthreads();
      for (int j = hi - 1; j >= lo; --j) {
        const double tj = tstage[j - lo];
        if (tj == 0.0) continue;
        const double* vj = stage + (int64_t)(j - lo) * m;
        double v[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          const int r = lane + 64 * t;
          const double raw = vj[r < m ? r : m - 1];   // in-bounds read, masked below
          v[t] = (r > j && r < m) ? raw : (r == j ? 1.0 : 0.0);
        }
        double part[CPW];
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
          double a = 0.0;
#pragma unroll
          for (int t = 0; t < MT; ++t) a += v[t] * y[q][t];
          part[q] = a;
        }
#pragma unroll
        for (int q = 0; q < CPW; ++q) part[q] = wave_sum(part[q]);
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
          const double f = tj * part[q];
#pragma unroll
          for (int t = 0; t < MT; ++t) y[q][t] -= f * v[t];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = cb + w + NW * q;
      if (c < s) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          const int r = lane + 64 * t;
          if (r < m) Y[(int64_t)c * ldy + r] = y[q][t];
        }
      }
    }
  }
  __syncthreads();
}

// M^T = Q_thin [T^T; 0] for a panel factorised by the right-to-left pass's
// TSQR (n columns, m rows, nc leaves): the nodes of the merge tree are applied
// top down, each splitting its output between its two ranges; then every leaf
// applies its reflectors to its block of rows.  On entry Y (m x s,
// column-major) holds [T^T; 0]; zbuf holds 2 n s doubles.
__device__ void tsqr_apply(const double* ws, int m, int n, double* Y, int s, int nc,
                           double* stage, int cap, double* tstage, double* zbuf) {
  const int tid = threadIdx.x;
  const double* ws_tau = ws + (int64_t)(2 * nc * QROWS + 2 * n) * n;
  // the merge tree top down: a node's input (its range's rows of the running
  // factor) sits at the head of its first leaf's row block; the root's is the
  // head of Y (= T^T)
  for (int l = tsqr_root_level(nc); l >= 0; --l) {
    for (int c = 1 << l; c < nc; c += 2 << l) {
      const int a = c - (1 << l), hi = (c + (1 << l)) < nc ? (c + (1 << l)) : nc;
      const int kl = tsqr_rows(m, n, a, c), kr = tsqr_rows(m, n, c, hi);
      const int kc = tsqr_rows(m, n, a, hi), mr = kl + kr;
      // zbuf (mr x s) = [the node's input (kc rows); 0]
      for (int e = tid; e < mr * s; e += NT) {
        const int col = e / mr, r = e % mr;
        zbuf[e] = (r < kc) ? Y[(int64_t)col * m + a * QROWS + r] : 0.0;
      }
      __syncthreads();
      const int kk = mr < n ? mr : n;
      wg_apply_q_reg<4>(ws + (int64_t)(nc + c) * QROWS * n, ws_tau + (int64_t)(nc + c) * n, mr,
                        kk, zbuf, s, stage, cap, tstage);
      // the left range's rows back to the head of leaf a's block, the right
      // range's to the head of leaf c's
      for (int e = tid; e < mr * s; e += NT) {
        const int col = e / mr, r = e % mr;
        if (r < kl)
          Y[(int64_t)col * m + a * QROWS + r] = zbuf[e];
        else
          Y[(int64_t)col * m + c * QROWS + (r - kl)] = zbuf[e];
      }
      __syncthreads();
    }
  }
  // leaves: rows [c*256, c*256 + mc): [input (kl rows); 0] -> Q_c [input; 0]
  for (int c = 0; c < nc; ++c) {
    const int mc = (m - c * QROWS) < QROWS ? (m - c * QROWS) : QROWS;
    double* Yc = Y + c * QROWS;
    const int kl = tsqr_rows(m, n, c, c + 1);
    for (int e = tid; e < mc * s; e += NT) {
      const int col = e / mc, r = e % mc;
      if (r >= kl) Yc[(int64_t)col * m + r] = 0.0;
    }
    __syncthreads();
    wg_apply_q_reg<4>(ws + (int64_t)c * QROWS * n, ws_tau + (int64_t)c * n, mc, kl, Yc, s,
                      stage, cap, tstage, m);
  }
}

// Y <- H_0 ... H_{k-1} Y (Y: mp x s, column-major, ld mp, s <= 32) for a panel
// factorised by the multi-workgroup QR (kernels_wide.hip): reflectors below the
// diagonal of V (column-major, ld mp), the compact-WY factor T_j of column block
// j (32 columns) at Tb + 1024 j (row-major 32 x 32).  Blocks from the last to
// the first: W = V_j^T Y, W = T_j W, Y -= V_j W, where the unit lower triangle
// of V_j (rows j0 .. j0 + jb) is handled apart from its dense rows below, which
// go through the matrix cores straight from V (split-K for V^T Y, 16-row
// blocks for Y -= V W).  lds: unused; Wl, W2, Ts: 1024 doubles each (LDS).
__device__ void wg_apply_wy(const double* __restrict__ V, const double* __restrict__ Tb, int mp,
                            int k, double* Y, int s, double* lds, double* Wl, double* W2,
                            double* Ts) {
  const int tid = threadIdx.x;
  const int nb = (k + 31) / 32;
  for (int j = nb - 1; j >= 0; --j) {
    const int j0 = 32 * j, jb = k - j0 < 32 ? k - j0 : 32;
    const int rb = j0 + jb, mb = mp - rb;
    for (int e = tid; e < 1024; e += NT) Ts[e] = Tb[(int64_t)j * 1024 + e];
    // W = V_bot^T Y_bot (jb x s), split over the mb dense rows
    wg_atb<2, 2>(jb, s, mb, V + (int64_t)j0 * mp + rb, mp, Y + rb, mp, Wl);
    // W[q][c] += Y[j0 + q][c] + sum_{q < r < jb} V[j0 + r][j0 + q] Y[j0 + r][c]
    for (int e = tid; e < jb * s; e += NT) {
      const int q = e / s, c = e - q * s;
      const double* vq = V + (int64_t)(j0 + q) * mp + j0;
      const double* yc = Y + (int64_t)c * mp + j0;
      double acc = yc[q];
      for (int r = q + 1; r < jb; ++r) acc += vq[r] * yc[r];
      Wl[q * 32 + c] += acc;
    }
    __syncthreads();
    // W2 = T W (T upper triangular)
    for (int e = tid; e < jb * s; e += NT) {
      const int q = e / s, c = e - q * s;
      double acc = 0.0;
      for (int r = q; r < jb; ++r) acc += Ts[q * 32 + r] * Wl[r * 32 + c];
      W2[q * 32 + c] = acc;
    }
    __syncthreads();
    // top rows: Y[j0 + r][c] -= W2[r][c] + sum_{q < r} V[j0 + r][j0 + q] W2[q][c]
    for (int e = tid; e < jb * s; e += NT) {
      const int r = e / s, c = e - r * s;
      double acc = W2[r * 32 + c];
      for (int q = 0; q < r; ++q) acc += V[(int64_t)(j0 + q) * mp + j0 + r] * W2[q * 32 + c];
      Y[(int64_t)c * mp + j0 + r] -= acc;
    }
    if (mb > 0)
      wg_ab_rows<2>(mb, s, jb, -1.0, V + (int64_t)j0 * mp + rb, mp, W2, 32, 1, Y + rb, mp);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Left-to-right pass, one workgroup per MPO.  Panels live in LDS when they fit.
// ---------------------------------------------------------------------------
constexpr int LR_MB = 6144;   // M panel / Y
constexpr int LR_VB = 6144;   // staged reflectors, E, W
constexpr int LR_UB = 4096;   // Jacobi rotations, C
constexpr int LR_SC = 990;    // sort / sign buffers (6144*2 + 4096 + 3*990 + 80 <= ARENA)

static_assert(LR_MB + LR_VB + LR_UB + 3 * LR_SC + 16 + 64 <= ARENA, "left-to-right LDS carve");
static_assert(ARENA == kSweepArena, "arena size shared with the host plan");
static_assert(QROWS == kRegRows && QCOLS == kRegCols && 16 * QROWS == kTsqrLeavesMax * kRegRows,
              "register panel shape shared with the host plan");
static_assert(LR_SC == kSortCap, "sort capacity shared with the host plan");

struct ScratchLayout {
  double* T;
  double* M;
  double* U;
  double* Q;   // QR-preconditioned Jacobi: blocked-QR workspace, then the scalars
};

template <typename TO>
__global__ __launch_bounds__(NT) void k_lr_pass(const MpoDesc* mpos, const CoreDesc* cores, int op,
                                                const int* rho, const int* ldm, int* xr,
                                                const double* Wd, const double* tau,
                                                double* scratch, TO* __restrict__ Xout,
                                                double* outs, SweepOpts so, int64_t tcap,
                                                int64_t mcap_s, int64_t ucap, int* err,
                                                const int* wflag, const int* order) {
  __shared__ double arena[ARENA];
  __shared__ int iarena[LR_SC + 16];
  double* Mb = arena;
  double* Vb = Mb + LR_MB;
  double* Ub = Vb + LR_VB;
  double* sig = Ub + LR_UB;
  double* nrmb = sig + LR_SC;
  double* sgn = nrmb + LR_SC;
  double* red = sgn + LR_SC;
  double* tst = red + 16;           // 64 doubles of staged tau
  int* perm = iarena;
  int* ibuf = iarena + LR_SC;
  const int tid = threadIdx.x;
  const int bm = order ? order[blockIdx.x] : (int)blockIdx.x;   // costliest MPOs first
  const MpoDesc md = mpos[bm];
  const int d = md.d, K = md.K;
  const bool wide = wflag && wflag[bm];   // panels factorised by kernels_wide.hip
  ScratchLayout SL;
  SL.T = scratch + md.s_off;
  SL.M = SL.T + tcap;
  SL.U = SL.M + mcap_s;
  SL.Q = SL.U + ucap;
  const CoreDesc c0 = cores[md.c0];
  const int n0 = op == 0 ? c0.I : c0.J;
  const int m0 = n0 * (d > 1 ? rho[md.r0 + 1] : K);
  const double* X0 = Wd + c0.w_off;
  double part = 0.0;
  for (int t = tid; t < m0; t += NT) part += X0[t] * X0[t];
  const double nrm = sqrt(block_sum(part, red));
  const double delta = d > 1 ? so.eps * nrm / sqrt((double)(d - 1)) : 0.0;
  int s = 1;
  if (tid == 0) {
    xr[md.r0] = 1;
    xr[md.r0 + d] = K;
  }
  for (int i = 0; i < d; ++i) {
    const CoreDesc cd = cores[md.c0 + i];
    const int n = op == 0 ? cd.I : cd.J;
    const int rn = (i == d - 1) ? K : rho[md.r0 + i + 1];
    const int ldraw = (i == 0) ? rn : ldm[md.r0 + i];
    const int ntree = ldraw < 0 ? -ldraw : 0;   // > 0: the panel was factorised by TSQR
    const int ld = ldraw < 0 ? rn : ldraw;
    const int mp = n * ld;
    const int ri = i == 0 ? 1 : rho[md.r0 + i];
    const int64_t nvg = (int64_t)s * n;
    {
      bool bad = s < 1 || s > cd.xcap || rn < 1 || rn > cd.RA2 * cd.xcap2 || ld < rn ||
                 ri < 1 || ri > cd.RA * cd.xcap || (int64_t)s * mp > mcap_s ||
                 (int64_t)s * ri > tcap || K > LR_SC || mp > ARENA;
      if (i < d - 1)
        bad = bad || nvg > LR_SC || nvg * nvg > ucap || (int64_t)cd.xcap2 * rn > tcap;
      else
        bad = bad || nvg > ARENA || 2 * nvg * K + K + (int64_t)K * K > ucap;
      if (bad) {
        if (tid == 0) atomicOr(err, 4);
        return;
      }
    }
    const bool m_in_lds = (int64_t)s * mp <= LR_MB;
    double* M = m_in_lds ? Mb : SL.M;
    if (i == 0) {
      for (int t = tid; t < mp; t += NT) M[t] = X0[t];
      __syncthreads();
    } else {
      // M^T (mp x s, column-major) = H_0 ... H_{ri-1} [T^T; 0]
      for (int64_t o = tid; o < (int64_t)mp * s; o += NT) {
        const int c = (int)(o / mp), r = (int)(o % mp);
        M[o] = (r < ri) ? SL.T[(int64_t)c * ri + r] : 0.0;
      }
      __syncthreads();
      if (ntree > 0) {
        tsqr_apply(Wd + cd.w_off, mp, ri, M, s, ntree, Vb, LR_VB, tst,
                   ((int64_t)2 * ri * s <= LR_UB) ? Ub : SL.U);
      } else if (wide && s <= 32) {
        wg_apply_wy(Wd + cd.w_off, Wd + cd.wt_off, mp, ri, M, s, Vb, Ub, Ub + 1024, Ub + 2048);
      } else if (mp <= 256)   // reflectors staged over the V and U carve (U is free here)
        wg_apply_q_reg<4>(Wd + cd.w_off, tau + cd.tau_off, mp, ri, M, s, Vb, LR_VB + LR_UB, tst);
      else if (mp <= 1024)
        wg_apply_q_reg<16>(Wd + cd.w_off, tau + cd.tau_off, mp, ri, M, s, Vb, LR_VB + LR_UB, tst);
      else if (mp <= LR_VB)
        wg_apply_q_staged(Wd + cd.w_off, tau + cd.tau_off, mp, ri, M, s, Vb, LR_VB, tst);
      else
        wg_apply_q(Wd + cd.w_off, tau + cd.tau_off, mp, ri, M, s);
    }
    // M is now s x mp row-major: row (c, y) = c * n + y of the (s n) x rn panel, stride ld.
    const int nv = s * n;
    if (i < d - 1) {
      double* U = (nvg * nvg <= LR_UB) ? Ub : SL.U;
      // A panel in global memory with fewer rows than columns is first reduced
      // by a QR of its transpose, M^T = Q R (blocked Householder, in place,
      // its panels staged in the free M and V carve):
      // the rows of M and of R^T have the same inner products, so the one-sided
      // Jacobi runs on the nv x nv R^T in LDS with the same rotations, and the
      // carried factor U^T M = (U^T R^T) Q^T is recovered by applying Q.
      // R^T stays in LDS when it fits with U, else it goes to the scratch after
      // the QR's scalars (the Jacobi then works from L2)
      const bool pre_lds = nv * nv <= LR_MB && nvg * nvg <= LR_UB;
      // larger R^T (up to 128 x 128) over the whole M, V and U carve, with U in
      // the scratch; past that R^T goes to the scratch too
      const bool pre_wide = !pre_lds && nv * nv <= LR_MB + LR_VB + LR_UB && nvg * nvg > LR_UB &&
                            rn <= LR_VB;
      const bool pre_glob = !pre_lds && !pre_wide && nv <= 256 && rn <= LR_VB &&
                            (int64_t)rn * QB + 2 * QB * nv + nv + nvg * nvg <= so.qcap;
      const bool pre = !m_in_lds && nv < rn && (pre_lds || pre_wide || pre_glob) &&
                       2 * QBMAX * QBMAX <= LR_UB &&
                       (int64_t)rn * QB + 2 * QB * nv + nv <= so.qcap;
      // Where U would sit in the scratch (R^T over the whole LDS carve), the
      // Jacobi runs on the rows of R instead and keeps no rotations: the
      // normalised rows of J R are the left singular vectors of R^T (so of
      // M), re-orthonormalised by a small QR, and the carried factor is
      // formed from R itself.  Needs room in LDS for that QR.
      int rsel = so.rmax > 0 && so.rmax < nv ? so.rmax : nv;
      if (cd.xcap2 < rsel) rsel = cd.xcap2;
      const bool noacc = pre && (pre_wide || pre_lds) && 2 * nv * rsel + nv <= LR_MB + LR_VB + LR_UB;
      // Likewise without the QR, when the panel has no more columns than rows
      // and U would sit in the scratch: the Jacobi runs on the columns of M
      // (rows of M^T, copied to LDS), whose normalised results are M's left
      // singular vectors; the carried factor is then U^T M from M itself.
      // M^T and the later small QR use the LDS after M (the V and U carve)
      // when M itself sits in LDS, else the whole carve.
      const int cst = nv + ((16 - nv % 32) + 32) % 32;
      double* wk = m_in_lds ? Vb : Mb;
      const int wcap = m_in_lds ? LR_VB + LR_UB : LR_MB + LR_VB + LR_UB;
      const bool cols = !pre && rn <= nv && nv <= 256 && (int64_t)rn * cst <= wcap &&
                        2 * nv * rsel + nv <= wcap && (int64_t)nv * rsel <= ucap;
      double* B = M;
      int blen = rn, bld = ld;
      double* tauP = SL.Q + (int64_t)rn * QB + 2 * QB * nv;
      if (pre) {
        wg_geqrf(M, rn, nv, tauP, Mb, red, SL.Q, Mb, LR_MB + LR_VB, Ub, Ub + QBMAX * QBMAX, ld,
                 QB);
        double* Bt = (pre_lds || pre_wide) ? Mb : tauP + nv;
        // in LDS, rows 16 doubles (mod 32) apart put the four rows a wave
        // reads at once (one per 16-lane group) on two bank halves, not one
        const int cap = pre_lds ? LR_MB : LR_MB + LR_VB + LR_UB;
        const int pld = nv + ((16 - nv % 32) + 32) % 32;
        const int bst = ((pre_lds || pre_wide) && nv * pld <= cap) ? pld : nv;
        for (int e = tid; e < nv * nv; e += NT) {
          const int p = e / nv, c = e - p * nv;
          if (noacc)
            Bt[p * bst + c] = c >= p ? M[(int64_t)c * ld + p] : 0.0;   // row p of R
          else
            Bt[p * bst + c] = c <= p ? M[(int64_t)p * ld + c] : 0.0;   // row p of R^T
        }
        __syncthreads();
        B = Bt;
        blen = nv;
        bld = bst;
      }
      int nvec = nv;   // the vectors the Jacobi rotates (rows of B)
      if (cols) {
        // B = M^T in LDS: row f holds column f of the panel
        for (int64_t e = tid; e < (int64_t)rn * nv; e += NT) {
          const int f = (int)(e / nv), r = (int)(e - (int64_t)f * nv);
          wk[(int64_t)f * cst + r] = M[(int64_t)r * ld + f];
        }
        B = wk;
        nvec = rn;
        blen = nv;
        bld = cst;
      }
      if (noacc || cols)
        jacobi_rows_lr(B, nvec, blen, bld, ibuf, red, delta * delta / (double)nv);
      else
        wg_jacobi_lr(B, nv, blen, bld, U, ibuf, red, delta * delta / (double)nv, B == Mb,
                     U == Ub);
      wg_norms_sorted(B, nvec, blen, bld, sig, perm, nrmb);
      if (tid == 0) {
        const int kk = nv < rn ? nv : rn;
        const double d2 = delta * delta;
        double tail = 0.0;
        int rho_new = kk;
        // smallest rho >= 1 with sum_{l >= rho} sig_l^2 <= delta^2
        for (int cand = kk - 1; cand >= 1; --cand) {
          tail += sig[cand] * sig[cand];
          if (tail <= d2)
            rho_new = cand;
          else
            break;
        }
        if (so.rmax > 0 && rho_new > so.rmax) rho_new = so.rmax;
        if (rho_new < 1) rho_new = 1;
        if (rho_new > cd.xcap2) {
          atomicOr(err, 2);
          rho_new = cd.xcap2;
        }
        ibuf[1] = rho_new;
      }
      __syncthreads();
      const int rnew = ibuf[1];
      TO* xo = Xout + cd.x_off;
      if (noacc || cols) {
        // the kept rows of J R (or of M^T J) normalised: column k of Us, nv x rnew
        double* Us = SL.U;
        for (int64_t o = tid; o < (int64_t)nv * rnew; o += NT) {
          const int k = (int)(o / nv), c = (int)(o % nv);
          const double sk = sig[k];
          Us[o] = sk > 0.0 ? B[(int64_t)perm[k] * bld + c] / sk : 0.0;
        }
        __syncthreads();
        // Householder QR (diag(R) >= 0) of Us in LDS, then E = Q [I; 0]
        double* Ul = wk;
        double* vq = wk + (int64_t)nv * rnew;
        double* E = vq + nv;
        for (int64_t o = tid; o < (int64_t)nv * rnew; o += NT) {
          Ul[o] = Us[o];
          E[o] = (o % nv) == (o / nv) ? 1.0 : 0.0;
        }
        __syncthreads();
        wg_geqr2(Ul, nv, rnew, nrmb, vq, red, nv);
        wg_apply_q(Ul, nrmb, nv, rnew, E, rnew, nv);
        for (int k = tid; k < rnew; k += NT) sgn[k] = sign_of_max(E + (int64_t)k * nv, nv, 1);
        __syncthreads();
        for (int64_t o = tid; o < (int64_t)nv * rnew; o += NT) {
          const int row = (int)(o / rnew), k = (int)(o % rnew);
          xo[o] = (TO)(E[(int64_t)k * nv + row] * sgn[k]);
        }
        // noacc: T^T (rn x rnew) = Q_M [R E sgn; 0], R read from the factorised
        // panel; cols: T (rnew x rn, row-major) = (E sgn)^T M
        for (int64_t o = tid; o < (int64_t)rnew * rn; o += NT) {
          const int k = (int)(o / rn), f = (int)(o % rn);
          const double* ek = E + (int64_t)k * nv;
          double acc = 0.0;
          if (cols) {
            for (int r = 0; r < nv; ++r) acc += ek[r] * M[(int64_t)r * ld + f];
          } else if (f < nv) {
            for (int c = f; c < nv; ++c) acc += M[(int64_t)c * ld + f] * ek[c];
          }
          SL.T[o] = acc * sgn[k];
        }
      } else {
        for (int k = tid; k < rnew; k += NT)
          sgn[k] = sign_of_max(U + (int64_t)perm[k] * nv, nv, 1);
        __syncthreads();
        for (int64_t o = tid; o < (int64_t)nv * rnew; o += NT) {
          const int row = (int)(o / rnew), k = (int)(o % rnew);
          xo[o] = (TO)(U[(int64_t)perm[k] * nv + row] * sgn[k]);
        }
      }
      if (pre) {
        // T^T (rn x rnew, column-major = T row-major) = Q [B_sel^T; 0]
        if (!noacc)
          for (int64_t o = tid; o < (int64_t)rnew * rn; o += NT) {
            const int k = (int)(o / rn), f = (int)(o % rn);
            SL.T[o] = f < nv ? B[(int64_t)perm[k] * bld + f] * sgn[k] : 0.0;
          }
        // the whole LDS carve is free again (R^T and U were last read above)
        if (rn <= 512)
          wg_apply_q_cols<8, 4>(M, ld, tauP, rn, nv, SL.T, rn, rnew, Mb, LR_MB + LR_VB + LR_UB,
                                tst);
        else if (rn <= 1024)
          wg_apply_q_cols<16, 2>(M, ld, tauP, rn, nv, SL.T, rn, rnew, Mb, LR_MB + LR_VB + LR_UB,
                                 tst);
        else {
          __syncthreads();
          wg_apply_q(M, tauP, rn, nv, SL.T, rnew, ld);
        }
      } else if (!cols) {
        for (int64_t o = tid; o < (int64_t)rnew * rn; o += NT) {
          const int k = (int)(o / rn), f = (int)(o % rn);
          SL.T[o] = M[(int64_t)perm[k] * ld + f] * sgn[k];
        }
      }
      if (tid == 0) xr[md.r0 + i + 1] = rnew;
      s = rnew;
      __syncthreads();
    } else {
      // last core: the (s n) x K panel as a column-major copy C, in LDS over
      // the V and U carve when it fits (the panel M, read while C is formed,
      // may sit in the M carve, which is free afterwards), else in the scratch
      const int64_t ck = (int64_t)nv * K;
      double* C = (ck <= LR_VB + LR_UB) ? Vb : SL.U;
      for (int64_t o = tid; o < ck; o += NT) {
        const int row = (int)(o % nv), kap = (int)(o / nv);
        C[o] = M[(int64_t)row * ld + kap];
      }
      __syncthreads();
      double* o_sig = outs + md.out_off;
      double* o_W = o_sig + K;
      double* o_R = o_W + (int64_t)K * K;
      TO* xo = Xout + cd.x_off;
      if (so.mode == 0) {
        // thin Householder QR (Algorithm 5.2, mirrored): Q_d and the K x K R
        double* tauK = sig;
        double* E = (ck <= LR_MB) ? Mb : SL.U + ck + K;
        double* vtmp = (nv <= LR_SC) ? nrmb : SL.M;
        wg_geqr2(C, nv, K, tauK, vtmp, red);
        for (int64_t o = tid; o < (int64_t)K * K; o += NT) {
          const int r = (int)(o / K), c = (int)(o % K);
          o_R[o] = (c >= r) ? C[(int64_t)c * nv + r] : 0.0;
        }
        for (int64_t o = tid; o < ck; o += NT) {
          const int row = (int)(o % nv), kap = (int)(o / nv);
          E[o] = (row == kap) ? 1.0 : 0.0;
        }
        __syncthreads();
        wg_apply_q(C, tauK, nv, K, E, K);
        for (int64_t o = tid; o < ck; o += NT) {
          const int row = (int)(o / K), kap = (int)(o % K);
          xo[o] = (TO)E[(int64_t)kap * nv + row];
        }
      } else {
        // economical SVD (Algorithm 5.3, mirrored): C W = X diag(sigma)
        double* Wr = ((int64_t)K * K <= LR_MB) ? Mb : SL.U + ck;
        wg_jacobi_lr(C, K, nv, nv, Wr, ibuf, red, 0.0, C == Vb, Wr == Mb);
        wg_norms_sorted(C, K, nv, nv, sig, perm, nrmb);
        for (int k = tid; k < K; k += NT) sgn[k] = sign_of_max(C + (int64_t)perm[k] * nv, nv, 1);
        __syncthreads();
        for (int k = tid; k < K; k += NT) o_sig[k] = sig[k];
        for (int64_t o = tid; o < (int64_t)K * K; o += NT) {
          const int kap = (int)(o / K), k = (int)(o % K);
          o_W[o] = Wr[(int64_t)perm[k] * K + kap] * sgn[k];
        }
        for (int64_t o = tid; o < ck; o += NT) {
          const int row = (int)(o / K), k = (int)(o % K);
          const double sk = sig[k];
          const double val = C[(int64_t)perm[k] * nv + row] * sgn[k];
          xo[o] = (TO)(sk > 0.0 ? val / sk : 0.0);
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_rl_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* pr, int* rho, int* ldm, const void* Z, int dtype, double* Wd,
                          double* L, double* tau, int* err, int leaf_nc, const int* wflag,
                          const int* order, hipStream_t s) {
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    if (leaf_nc > 1) {
      k_rl_leaves<T><<<dim3(batch, leaf_nc), NT, 0, s>>>(mpos, cores, op, pr, (const T*)Z, Wd,
                                                         wflag);
      // the levels below the root of the largest tree (the root: the last-core phase)
      const int lroot = 31 - __builtin_clz((unsigned)(leaf_nc - 1));
      for (int l = 0; l < lroot; ++l) {
        const int nodes = (leaf_nc + (2 << l) - 1) / (2 << l);
        k_rl_merge_level<<<dim3(batch, nodes), NT, 0, s>>>(mpos, cores, op, pr, Wd, l, wflag);
      }
    }
    k_rl_pass<T, 0><<<batch, NT, 0, s>>>(mpos, cores, op, pr, rho, ldm, (const T*)Z, Wd, L, tau,
                                         err, wflag, order);
    k_rl_pass<T, 1><<<batch, NT, 0, s>>>(mpos, cores, op, pr, rho, ldm, (const T*)Z, Wd, L, tau,
                                         err, wflag, order);
  });
  return hipGetLastError();
}

hipError_t launch_lr_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* rho, const int* ldm, int* xr, const double* Wd,
                          const double* tau, double* scratch, void* Xout, int out_dtype,
                          double* outs, SweepOpts o, int64_t tcap, int64_t mcap_s, int64_t ucap,
                          int* err, const int* wflag, const int* order, hipStream_t s) {
  by_dtype(out_dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_lr_pass<T><<<batch, NT, 0, s>>>(mpos, cores, op, rho, ldm, xr, Wd, tau, scratch, (T*)Xout,
                                      outs, o, tcap, mcap_s, ucap, err, wflag, order);
  });
  return hipGetLastError();
}

}  // namespace tnr
