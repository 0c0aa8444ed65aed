// Multi-workgroup right-to-left pass of the rounding for wide products (gfx950).
//
// The rounding applied after every product (Sec. 3 rounding, used after each
// product as in Sec. 5.4; mirrored so that the K leg sits on the last core)
// starts with a right-to-left sweep: core i of the product absorbs the factor
// L_{i+1} of its right neighbour, Zt_i = Z_i x_3 L_{i+1}, and is factorised as
// Zt_i = L_i Q_i (a Householder QR of the (n rho') x P panel Zt_i^T).  For
// product ranks P in the hundreds one workgroup per MPO (kernels_sweep.hip)
// leaves all but one compute unit idle, so for such MPOs each core is spread
// over many workgroups, one launch per phase:
//   k_wide_load     Zt_i^T as tiled FP64 GEMMs on the matrix cores, one 64 x 64
//                   output tile per workgroup, over all mode indices y at once
//                   (the last core: a copy of the product core);
//   k_wide_step(j)  the compact-WY update (I - V T V^T)^T of the trailing
//                   columns by column block j, one strip of columns per
//                   workgroup; the workgroup of the first strip then
//                   factorises block j + 1 (blocked Householder, diag(R) >= 0)
//                   and writes its explicit reflectors and its T factor;
//   k_wide_finish   R (upper trapezoid) to the L slab, the ranks rho and ldm.
// Cores stay sequential, since each absorbs its neighbour's factor.  What is
// left behind (reflectors below the diagonal of the panel, tau, R, rho, ldm)
// is what the one-workgroup path leaves, so the left-to-right pass reads both
// alike.  k_wide_classify decides per MPO, from the ranks on the device,
// whether some core's panel is wider than the register path (P > 128, or a
// last-core panel beyond the TSQR leaves); only those MPOs take these kernels,
// and only when the launch plan covers them (otherwise the one-workgroup path
// keeps them).
#include "tnrsvd_internal.h"
#include "wg_linalg.h"

namespace tnr {

namespace {

constexpr int NB = kWideNB;   // column block of the QR
constexpr int SW = 64;        // columns per update workgroup (strips after the first)
constexpr int WARENA = 19456; // doubles of static LDS per workgroup (152 KiB)
constexpr int RCAP = WARENA - 64 - 2 * QBMAX * QBMAX;   // LDS for panels and GEMM tiles
static_assert(NB == QBMAX, "one QR block is one compact-WY block");
static_assert(2 * SW * NB + NB * NB + GEMM_LDS <= WARENA, "update carve");

// True when core i's panel is wider than the one-workgroup register path:
// more than 128 columns, or a last-core panel taller than the TSQR leaves.
__device__ __forceinline__ bool wide_core(int i, int d, int n, int P, int rnext) {
  if (i == 0) return false;
  if (P > kRegCols) return true;
  return i == d - 1 && n * rnext > kTsqrLeavesMax * kRegRows;
}

// One workgroup: need[t * kWidePlan + .] = maxima over the wide MPOs of
// (column blocks, P, n rho', rho', n) at step t; wflag[b] = 1 for the MPOs the
// wide launches take.  With a plan, an MPO is taken only if every step fits
// it; without one the caller launches from `need`.
__global__ __launch_bounds__(512) void k_wide_classify(const MpoDesc* mpos,
                                                       const CoreDesc* cores, int batch, int op,
                                                       const int* pr, const int* plan,
                                                       int max_d, int* wflag, int* need) {
  for (int e = threadIdx.x; e < max_d * kWidePlan; e += blockDim.x) need[e] = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    const MpoDesc md = mpos[b];
    const int d = md.d;
    bool wide = false, ok = true;
    int rn = md.K;
    for (int i = d - 1; i >= 0 && ok; --i) {
      const CoreDesc cd = cores[md.c0 + i];
      const int n = op == 0 ? cd.I : cd.J;
      const int P = pr[md.r0 + i];
      const int64_t m = (int64_t)n * rn;
      // shapes the one-workgroup path rejects stay there (it reports them)
      if (P < 1 || P > cd.RA * cd.xcap || m > md.wmcap || m > RCAP) ok = false;
      if (wide_core(i, d, n, P, rn)) wide = true;
      rn = (int)(m < P ? m : P);
    }
    if (!(wide && ok)) {
      wflag[b] = 0;
      continue;
    }
    rn = md.K;
    bool covered = true;
    for (int i = d - 1; i >= 0; --i) {
      const CoreDesc cd = cores[md.c0 + i];
      const int n = op == 0 ? cd.I : cd.J;
      const int P = pr[md.r0 + i];
      const int m = n * rn;
      const int k = m < P ? m : P;
      const int t = d - 1 - i;
      const int v[kWidePlan] = {i >= 1 ? (k + NB - 1) / NB : 0, P, m, rn, n};
      if (plan) {
        for (int c = 0; c < kWidePlan; ++c) covered = covered && v[c] <= plan[t * kWidePlan + c];
      } else {
        for (int c = 0; c < kWidePlan; ++c) atomicMax(need + t * kWidePlan + c, v[c]);
      }
      rn = k;
    }
    wflag[b] = covered ? 1 : 0;
  }
}

// Step t, core i = d - 1 - t of every wide MPO: the absorbed panel
// Xt[(y, f), p] = sum_{q >= f} R_{i+1}[f, q] Z_i[p, y, q] (column-major,
// m = n rho' rows), one 64 x 64 tile (y, f-tile, p-tile) per workgroup; R is
// upper trapezoidal, so the reduction starts at the tile's first row.  On the
// last core (t = 0) the panel is the product core itself.
template <typename T>
__global__ __launch_bounds__(NT) void k_wide_load(const MpoDesc* mpos, const CoreDesc* cores,
                                                  int op, const int* pr, const int* rho,
                                                  const int* wflag, int t, int tf_n, int tp_n,
                                                  const T* __restrict__ Z, double* Wd,
                                                  const double* L) {
  __shared__ double lds[GEMM_LDS];
  const int b = blockIdx.y;
  if (!wflag[b]) return;
  const MpoDesc md = mpos[b];
  const int i = md.d - 1 - t;
  if (i < 0) return;
  const CoreDesc cd = cores[md.c0 + i];
  const int n = op == 0 ? cd.I : cd.J;
  const int P = pr[md.r0 + i];
  double* Xt = Wd + cd.w_off;
  const T* Zc = Z + cd.z_off;
  if (i == md.d - 1) {
    // Zt^T = Z^T: the (P, n, K) core read as the column-major (n K) x P panel
    const int64_t tot = (int64_t)n * md.K * P;
    for (int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x; o < tot; o += (int64_t)gridDim.x * NT)
      Xt[o] = (double)Zc[o];
    return;
  }
  const int rnext = rho[md.r0 + i + 1];
  const int Pn = pr[md.r0 + i + 1];
  const int m = n * rnext;
  int x = blockIdx.x;
  const int tp = x % tp_n;
  x /= tp_n;
  const int tf = x % tf_n;
  const int y = x / tf_n;
  const int f0 = 64 * tf, p0 = 64 * tp;
  if (y >= n || f0 >= rnext || p0 >= P) return;
  const double* Rn = L + cores[md.c0 + i + 1].l_off;   // rho' x Pn, row-major, zeros below
  const int mt = rnext - f0 < 64 ? rnext - f0 : 64;
  const int nt = P - p0 < 64 ? P - p0 : 64;
  wg_gemm_t<64, 64, T>(mt, nt, Pn - f0, 1.0, Rn + (int64_t)f0 * Pn + f0, Pn, 1,
                       Zc + (int64_t)y * Pn + (int64_t)p0 * n * Pn + f0, 1, (int64_t)n * Pn, 0.0,
                       Xt + (int64_t)y * rnext + f0 + (int64_t)p0 * m, 1, m, lds);
}

// Step t, column block j of core i = d - 1 - t: strip s of the trailing
// columns (s = 0: the NB columns of block j + 1; s >= 1: SW columns each
// after them) takes C <- (I - V T V^T)^T C = C - V (C^T V T)^T with the
// explicit reflectors V of block j (double buffer j & 1) and its T; then the
// workgroup of strip 0 factorises block j + 1 (rows from its diagonal down)
// in place, writes its reflectors explicitly to the other buffer and its T.
// j = -1 only factorises block 0.
__global__ __launch_bounds__(NT) void k_wide_step(const MpoDesc* mpos, const CoreDesc* cores,
                                                  int op, const int* pr, const int* rho,
                                                  const int* wflag, int t, int j, double* Wd,
                                                  double* WV, double* tau) {
  __shared__ double arena[WARENA];
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  if (!wflag[b]) return;
  const MpoDesc md = mpos[b];
  const int i = md.d - 1 - t;
  if (i < 1) return;   // core 0 is absorbed only
  const CoreDesc cd = cores[md.c0 + i];
  const int n = op == 0 ? cd.I : cd.J;
  const int P = pr[md.r0 + i];
  const int rnext = (i == md.d - 1) ? md.K : rho[md.r0 + i + 1];
  const int m = n * rnext;
  const int kmax = m < P ? m : P;
  double* Xt = Wd + cd.w_off;
  double* Vbuf = WV + md.wv_off;                           // 2 x wmcap x NB
  double* qws = Vbuf + 2 * (int64_t)md.wmcap * NB;         // wmcap * 16 + 1024
  double* Tb = Wd + cd.wt_off;                             // NB x NB per block
  double* taui = tau + cd.tau_off;
  const int s = blockIdx.x;
  if (j >= 0 && NB * j < kmax) {
    const int j0 = NB * j;
    const int jb = kmax - j0 < NB ? kmax - j0 : NB;
    const int mp = m - j0;
    const int c0 = s == 0 ? j0 + jb : j0 + jb + NB + SW * (s - 1);
    const int wcap = s == 0 ? NB : SW;
    const int cs = P - c0 < wcap ? P - c0 : wcap;
    if (cs > 0) {
      double* Wt = arena;                  // C^T V, cs x jb (ld NB)
      double* W2t = arena + SW * NB;       // C^T V T
      double* Ts = arena + 2 * SW * NB;    // T, row-major NB x NB
      double* lds = Ts + NB * NB;
      const double* Vp = Vbuf + (int64_t)(j & 1) * md.wmcap * NB;
      for (int e = tid; e < NB * NB; e += NT) Ts[e] = Tb[(int64_t)j * NB * NB + e];
      __syncthreads();
      double* C = Xt + (int64_t)c0 * m + j0;
      wg_gemm_t<64, 32, double>(cs, jb, mp, 1.0, C, m, 1, Vp, 1, mp, 0.0, Wt, NB, 1, lds);
      wg_gemm_t<64, 32, double>(cs, jb, jb, 1.0, Wt, NB, 1, Ts, NB, 1, 0.0, W2t, NB, 1, lds);
      wg_gemm<double>(mp, cs, jb, -1.0, Vp, 1, mp, W2t, 1, NB, 1.0, C, 1, m, lds);
    }
  }
  if (s != 0) return;
  const int j1 = j + 1, j10 = NB * j1;
  if (j10 >= kmax) return;
  const int jb = kmax - j10 < NB ? kmax - j10 : NB;
  const int mp = m - j10;
  double* P0 = Xt + (int64_t)j10 * m + j10;
  double* Ts = arena + WARENA - 32 - 2 * QBMAX * QBMAX;
  double* Gs = Ts + QBMAX * QBMAX;
  double* red = arena + WARENA - 16;
  __syncthreads();
  wg_geqrf_impl<true>(P0, mp, jb, taui + j10, arena, red, qws, arena, RCAP, Ts, Gs, m, QBMAX);
  double* Vp = Vbuf + (int64_t)(j1 & 1) * md.wmcap * NB;
  for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
    const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
    Vp[e] = r > c ? P0[(int64_t)c * m + r] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  wg_build_t(Vp, mp, jb, taui + j10, Ts, Gs, arena);
  for (int e = tid; e < NB * NB; e += NT) Tb[(int64_t)j1 * NB * NB + e] = Ts[e];
}

// Step t: ldm, rho and R (rows f < k of the factorised panel, q >= f) to the
// L slab as the row-major k x P matrix with zeros below the diagonal; one
// 64-column tile per workgroup, transposed through LDS.
__global__ __launch_bounds__(NT) void k_wide_finish(const MpoDesc* mpos, const CoreDesc* cores,
                                                    int op, const int* pr, int* rho, int* ldm,
                                                    const int* wflag, int t, const double* Wd,
                                                    double* L) {
  __shared__ double tile[64 * 65];
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  if (!wflag[b]) return;
  const MpoDesc md = mpos[b];
  const int i = md.d - 1 - t;
  if (i < 0) return;
  const CoreDesc cd = cores[md.c0 + i];
  const int n = op == 0 ? cd.I : cd.J;
  const int P = pr[md.r0 + i];
  const int rnext = (i == md.d - 1) ? md.K : rho[md.r0 + i + 1];
  const int m = n * rnext;
  const int k = m < P ? m : P;
  if (blockIdx.x == 0 && tid == 0) {
    ldm[md.r0 + i] = rnext;
    if (i == md.d - 1) rho[md.r0 + md.d] = md.K;
    if (i >= 1) rho[md.r0 + i] = k;
  }
  if (i < 1) return;
  const int q0 = 64 * blockIdx.x;
  if (q0 >= P) return;
  const double* Xt = Wd + cd.w_off;
  double* Ro = L + cd.l_off;
  for (int f0 = 0; f0 < k; f0 += 64) {
    // tile[qq][ff] = Xt[(q0 + qq) m + f0 + ff]  (reads run along f)
    for (int e = tid; e < 64 * 64; e += NT) {
      const int qq = e >> 6, ff = e & 63;
      const int q = q0 + qq, f = f0 + ff;
      tile[qq * 65 + ff] = (q < P && f < k && q >= f) ? Xt[(int64_t)q * m + f] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += NT) {
      const int ff = e >> 6, qq = e & 63;
      const int q = q0 + qq, f = f0 + ff;
      if (q < P && f < k) Ro[(int64_t)f * P + q] = tile[qq * 65 + ff];
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_wide_classify(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                                const int* pr, const int* plan, int max_d, int* wflag, int* need,
                                hipStream_t s) {
  k_wide_classify<<<1, 512, 0, s>>>(mpos, cores, batch, op, pr, plan, max_d, wflag, need);
  return hipGetLastError();
}

// All launches of step t for the plan entry plan_t (host ints: blocks, P, m,
// rho', n bounds over the MPOs of the step).
hipError_t launch_rl_wide_step(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                               const int* pr, int* rho, int* ldm, const int* wflag, const void* Z,
                               int dtype, double* Wd, double* WV, double* L, double* tau, int t,
                               const int* plan_t, hipStream_t s) {
  const int nb = plan_t[0], Pm = plan_t[1], mm = plan_t[2], rnm = plan_t[3], nm = plan_t[4];
  if (Pm <= 0) return hipSuccess;
  const int tp_n = (Pm + 63) / 64, tf_n = (rnm + 63) / 64;
  int gx;
  if (t == 0) {
    const int64_t tot = (int64_t)mm * Pm;
    const int64_t g = (tot + 4 * NT - 1) / (4 * NT);
    gx = (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
  } else {
    gx = nm * tf_n * tp_n;
  }
  by_dtype(dtype, [&](auto* tp) {
    using T = elem_t<decltype(tp)>;
    k_wide_load<T><<<dim3(gx, batch), NT, 0, s>>>(mpos, cores, op, pr, rho, wflag, t, tf_n, tp_n,
                                                  (const T*)Z, Wd, L);
  });
  for (int j = -1; j < nb; ++j) {
    const int rest = Pm - NB * (j + 1) - NB;   // columns after strip 0
    const int ns = j < 0 ? 1 : 1 + (rest > 0 ? (rest + SW - 1) / SW : 0);
    k_wide_step<<<dim3(ns, batch), NT, 0, s>>>(mpos, cores, op, pr, rho, wflag, t, j, Wd, WV, tau);
  }
  k_wide_finish<<<dim3(tp_n, batch), NT, 0, s>>>(mpos, cores, op, pr, rho, ldm, wflag, t, Wd, L);
  return hipGetLastError();
}

}  // namespace tnr
