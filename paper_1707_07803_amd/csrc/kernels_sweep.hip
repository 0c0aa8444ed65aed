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
#include "tnrsvd_internal.h"

namespace tnr {

namespace {

constexpr int NT = kSweepThreads;
constexpr int NW = NT / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup; every thread receives the total.  `red` holds NW doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) t += red[k];
  return t;
}

// Householder QR with nonnegative diagonal of the m x n column-major X (ld m),
// in place: R on and above the diagonal of the first min(m,n) rows, the
// Householder vectors (unit leading entry implicit) below it, scalars in tau.
// Each reflector maps its column x to +||x|| e_1, using Parlett's form of the
// leading entry when x_1 > 0 so that no cancellation occurs.
__device__ void wg_geqr2(double* X, int m, int n, double* tau, double* v, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kmax = m < n ? m : n;
  for (int j = 0; j < kmax; ++j) {
    double* col = X + (int64_t)j * m;
    const double alpha = col[j];
    double s2 = 0.0;
    for (int r = j + 1 + tid; r < m; r += NT) {
      const double t = col[r];
      s2 += t * t;
    }
    s2 = block_sum(s2, red);
    double tj, beta, inv_v0;
    if (s2 == 0.0) {
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
        double* xc = X + (int64_t)c * m;
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

// Y <- H_0 H_1 ... H_{k-1} Y for the m x s column-major Y (ld m), with the
// reflectors stored as by wg_geqr2 in V (ld m).  One wave per column of Y;
// columns are independent, so no barrier is needed between reflectors.
__device__ void wg_apply_q(const double* V, const double* tau, int m, int k, double* Y, int s) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = w; c < s; c += NW) {
    double* yc = Y + (int64_t)c * m;
    for (int j = k - 1; j >= 0; --j) {
      const double tj = tau[j];
      if (tj == 0.0) continue;
      const double* vj = V + (int64_t)j * m;
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
__device__ int wg_jacobi(double* B, int nv, int len, int ldb, double* U, int* flag) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int t = tid; t < nv * nv; t += NT) U[t] = ((t % nv) == (t / nv)) ? 1.0 : 0.0;
  __syncthreads();
  if (nv < 2) return 0;
  const double tol = 2.220446049250313e-16 * sqrt((double)(len > 4 ? len : 4));
  const int nn = nv + (nv & 1);
  int sweep = 0;
  for (; sweep < 80; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
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
        if (a == 0.0 || b == 0.0 || fabs(c) <= tol * sqrt(a) * sqrt(b)) continue;
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

// Norms of the nv vectors, then a stable descending sort: sig[pos], perm[pos].
__device__ void wg_norms_sorted(const double* B, int nv, int len, int ldb, double* sig, int* perm,
                                double* nrm) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
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

struct LdsLayout {
  double* v;      // Householder vector, vcap
  double* red;    // NW
  double* sig;    // scap
  double* nrm;    // scap
  double* sgn;    // scap
  int* perm;      // scap
  int* ibuf;      // 8 ints
};

__device__ inline LdsLayout carve(double* smem, int vcap, int scap) {
  LdsLayout L;
  L.v = smem;
  L.red = L.v + vcap;
  L.sig = L.red + NW;
  L.nrm = L.sig + scap;
  L.sgn = L.nrm + scap;
  L.perm = (int*)(L.sgn + scap);
  L.ibuf = L.perm + scap;
  return L;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_rl_pass(const MpoDesc* mpos, const CoreDesc* cores, int op,
                                                const int* pr, int* rho, const T* __restrict__ Z,
                                                double* Wd, double* L, double* tau, int vcap,
                                                int scap, int* err) {
  extern __shared__ double smem[];
  LdsLayout S = carve(smem, vcap, scap);
  const int tid = threadIdx.x;
  const MpoDesc md = mpos[blockIdx.x];
  const int d = md.d;
  if (tid == 0) rho[md.r0 + d] = md.K;
  int rnext = md.K;
  for (int i = d - 1; i >= 0; --i) {
    const CoreDesc cd = cores[md.c0 + i];
    const int n = op == 0 ? cd.I : cd.J;
    const int P = pr[md.r0 + i];
    const int Pn = pr[md.r0 + i + 1];
    const int m = n * rnext;
    // capacity guard (every value here is block uniform)
    if (P < 1 || P > cd.RA * cd.xcap || Pn < 1 || Pn > cd.RA2 * cd.xcap2 || rnext > Pn ||
        m > vcap) {
      if (tid == 0) atomicOr(err, 4);
      return;
    }
    double* Xt = Wd + cd.w_off;
    const T* Zc = Z + cd.z_off;
    const int64_t tot = (int64_t)m * P;
    if (i == d - 1) {
      // last core: Zt = Z (the K leg is external), stored transposed
      for (int64_t o = tid; o < tot; o += NT) {
        const int p = (int)(o / m), jj = (int)(o % m);
        Xt[o] = (double)Zc[(int64_t)p * m + jj];
      }
    } else {
      // Zt^T[(y, f), p] = sum_{q >= f} Z[p, y, q] R_{i+1}[f, q]   (L_{i+1} = R_{i+1}^T)
      const double* Rn = L + cores[md.c0 + i + 1].l_off;
      for (int64_t o = tid; o < tot; o += NT) {
        const int p = (int)(o / m), jj = (int)(o % m);
        const int y = jj / rnext, f = jj % rnext;
        const T* zr = Zc + ((int64_t)p * n + y) * Pn;
        const double* rr = Rn + (int64_t)f * Pn;
        double acc = 0.0;
        for (int qq = f; qq < Pn; ++qq) acc += (double)zr[qq] * rr[qq];
        Xt[o] = acc;
      }
    }
    __syncthreads();
    if (i == 0) break;
    wg_geqr2(Xt, m, P, tau + cd.tau_off, S.v, S.red);
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

// Scratch layout of one MPO (doubles): T buffer, M panel, U / C / E buffers.
struct ScratchLayout {
  double* T;
  double* M;
  double* U;
};

template <typename TO>
__global__ __launch_bounds__(NT) void k_lr_pass(const MpoDesc* mpos, const CoreDesc* cores, int op,
                                                const int* rho, int* xr, const double* Wd,
                                                const double* tau, double* scratch,
                                                TO* __restrict__ Xout, double* outs,
                                                SweepOpts so, int vcap, int scap,
                                                int64_t tcap, int64_t mcap_s, int64_t ucap,
                                                int* err) {
  extern __shared__ double smem[];
  LdsLayout S = carve(smem, vcap, scap);
  const int tid = threadIdx.x;
  const MpoDesc md = mpos[blockIdx.x];
  const int d = md.d, K = md.K;
  ScratchLayout SL;
  SL.T = scratch + md.s_off;
  SL.M = SL.T + tcap;
  SL.U = SL.M + mcap_s;
  const CoreDesc c0 = cores[md.c0];
  const int n0 = op == 0 ? c0.I : c0.J;
  const int m0 = n0 * (d > 1 ? rho[md.r0 + 1] : K);
  const double* X0 = Wd + c0.w_off;
  double part = 0.0;
  for (int t = tid; t < m0; t += NT) part += X0[t] * X0[t];
  const double nrm = sqrt(block_sum(part, S.red));
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
    const int m = n * rn;
    const int ri = i == 0 ? 1 : rho[md.r0 + i];
    const int64_t nvg = (int64_t)s * n;
    // capacity guard (every value here is block uniform)
    {
      bool bad = s < 1 || s > cd.xcap || rn < 1 || rn > cd.RA2 * cd.xcap2 || m > vcap ||
                 ri < 1 || ri > cd.RA * cd.xcap || (int64_t)s * m > mcap_s ||
                 (int64_t)s * ri > tcap || K > scap;
      if (i < d - 1)
        bad = bad || nvg > scap || nvg * nvg > ucap || (int64_t)cd.xcap2 * rn > tcap;
      else
        bad = bad || nvg > vcap || 2 * nvg * K + K + (int64_t)K * K > ucap;
      if (bad) {
        if (tid == 0) atomicOr(err, 4);
        return;
      }
    }
    double* M = SL.M;
    if (i == 0) {
      for (int t = tid; t < m; t += NT) M[t] = X0[t];
      __syncthreads();
    } else {
      // M^T (m x s, column-major) = H_0 ... H_{ri-1} [T^T; 0]
      for (int64_t o = tid; o < (int64_t)m * s; o += NT) {
        const int c = (int)(o / m), r = (int)(o % m);
        M[o] = (r < ri) ? SL.T[(int64_t)c * ri + r] : 0.0;
      }
      __syncthreads();
      wg_apply_q(Wd + cd.w_off, tau + cd.tau_off, m, ri, M, s);
    }
    // M is now s x m row-major, i.e. the (s n) x rn panel, row (c, y) = c * n + y.
    const int nv = s * n;
    if (i < d - 1) {
      double* U = SL.U;
      wg_jacobi(M, nv, rn, rn, U, S.ibuf);
      wg_norms_sorted(M, nv, rn, rn, S.sig, S.perm, S.nrm);
      if (tid == 0) {
        const int kk = nv < rn ? nv : rn;
        const double d2 = delta * delta;
        double tail = 0.0;
        int rho_new = kk;
        // smallest rho >= 1 with sum_{l >= rho} sig_l^2 <= delta^2
        for (int cand = kk - 1; cand >= 1; --cand) {
          tail += S.sig[cand] * S.sig[cand];
          if (tail <= d2) rho_new = cand;
          else break;
        }
        if (so.rmax > 0 && rho_new > so.rmax) rho_new = so.rmax;
        if (rho_new < 1) rho_new = 1;
        if (rho_new > cores[md.c0 + i].xcap2) {
          atomicOr(err, 2);
          rho_new = cores[md.c0 + i].xcap2;
        }
        S.ibuf[1] = rho_new;
      }
      __syncthreads();
      const int rnew = S.ibuf[1];
      for (int k = tid; k < rnew; k += NT)
        S.sgn[k] = sign_of_max(U + (int64_t)S.perm[k] * nv, nv, 1);
      __syncthreads();
      TO* xo = Xout + cd.x_off;
      for (int64_t o = tid; o < (int64_t)nv * rnew; o += NT) {
        const int row = (int)(o / rnew), k = (int)(o % rnew);
        xo[o] = (TO)(U[(int64_t)S.perm[k] * nv + row] * S.sgn[k]);
      }
      for (int64_t o = tid; o < (int64_t)rnew * rn; o += NT) {
        const int k = (int)(o / rn), f = (int)(o % rn);
        SL.T[o] = M[(int64_t)S.perm[k] * rn + f] * S.sgn[k];
      }
      if (tid == 0) xr[md.r0 + i + 1] = rnew;
      s = rnew;
      __syncthreads();
    } else {
      // last core: the (s n) x K panel, column-major copy C
      double* C = SL.U;
      const int64_t ck = (int64_t)nv * K;
      for (int64_t o = tid; o < ck; o += NT) {
        const int row = (int)(o % nv), kap = (int)(o / nv);
        C[o] = M[(int64_t)row * K + kap];
      }
      __syncthreads();
      double* o_sig = outs + md.out_off;
      double* o_W = o_sig + K;
      double* o_R = o_W + (int64_t)K * K;
      TO* xo = Xout + cd.x_off;
      if (so.mode == 0) {
        // thin Householder QR (Algorithm 5.2, mirrored): Q_d and the K x K R
        double* tauK = C + ck;
        double* E = tauK + K;
        wg_geqr2(C, nv, K, tauK, S.v, S.red);
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
        double* Wr = C + ck;
        wg_jacobi(C, K, nv, nv, Wr, S.ibuf);
        wg_norms_sorted(C, K, nv, nv, S.sig, S.perm, S.nrm);
        for (int k = tid; k < K; k += NT)
          S.sgn[k] = sign_of_max(C + (int64_t)S.perm[k] * nv, nv, 1);
        __syncthreads();
        for (int k = tid; k < K; k += NT) o_sig[k] = S.sig[k];
        for (int64_t o = tid; o < (int64_t)K * K; o += NT) {
          const int kap = (int)(o / K), k = (int)(o % K);
          o_W[o] = Wr[(int64_t)S.perm[k] * K + kap] * S.sgn[k];
        }
        for (int64_t o = tid; o < ck; o += NT) {
          const int row = (int)(o / K), k = (int)(o % K);
          const double sk = S.sig[k];
          const double val = C[(int64_t)S.perm[k] * nv + row] * S.sgn[k];
          xo[o] = (TO)(sk > 0.0 ? val / sk : 0.0);
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_rl_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* pr, int* rho, const void* Z, int dtype, double* Wd,
                          double* L, double* tau, int vcap, int scap, int* err, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)vcap + NW + 3 * (size_t)scap) +
                     sizeof(int) * ((size_t)scap + 8);
  if (dtype == 0)
    k_rl_pass<double><<<batch, NT, lds, s>>>(mpos, cores, op, pr, rho, (const double*)Z, Wd, L,
                                              tau, vcap, scap, err);
  else
    k_rl_pass<float><<<batch, NT, lds, s>>>(mpos, cores, op, pr, rho, (const float*)Z, Wd, L, tau,
                                             vcap, scap, err);
  return hipGetLastError();
}

hipError_t launch_lr_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* rho, int* xr, const double* Wd, const double* tau,
                          double* scratch, void* Xout, int out_dtype, double* outs, SweepOpts o,
                          int vcap, int scap, int64_t tcap, int64_t mcap_s, int64_t ucap,
                          int* err, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)vcap + NW + 3 * (size_t)scap) +
                     sizeof(int) * ((size_t)scap + 8);
  if (out_dtype == 0)
    k_lr_pass<double><<<batch, NT, lds, s>>>(mpos, cores, op, rho, xr, Wd, tau, scratch,
                                              (double*)Xout, outs, o, vcap, scap, tcap, mcap_s,
                                              ucap, err);
  else
    k_lr_pass<float><<<batch, NT, lds, s>>>(mpos, cores, op, rho, xr, Wd, tau, scratch,
                                             (float*)Xout, outs, o, vcap, scap, tcap, mcap_s, ucap,
                                             err);
  return hipGetLastError();
}

}  // namespace tnr
