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
//   k_wide_panel(j) the Householder QR (diag(R) >= 0) of 32-column block j,
//                   its columns held in registers, one workgroup per MPO; its
//                   explicit reflectors and its compact-WY factor T;
//   k_wide_update(j) the update (I - V T V^T)^T of the columns right of block
//                   j, one 64-column strip per workgroup;
//   k_wide_finish   R (upper trapezoid) to the L slab, the ranks rho and ldm.
// Cores stay sequential, since each absorbs its neighbour's factor.  What is
// left behind (reflectors below the diagonal of the panel, tau, R, rho, ldm)
// is what the one-workgroup path leaves, so the left-to-right pass reads both
// alike.  k_wide_classify decides per MPO, from the ranks on the device,
// whether some core's panel is wider than the register path (P > 128; for
// the last core P > 256), or its last-core panel lies beyond the TSQR leaves;
// only those MPOs take these kernels,
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

// Compile-time loop: f(integral_constant<int, B>), ..., f(<E - 1>).
template <int B, int E, typename F>
__device__ __forceinline__ void cfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    cfor<B + 1, E>(f);
  }
}

// Workgroups are dealt to the 8 XCDs in turn by linear id, and each XCD has
// its own L2.  For a (gx, gy) grid launched with gy rounded up to a multiple
// of 8, this maps the linear id so that every workgroup of one MPO (one
// logical y) runs on the same XCD and shares its reads of that MPO's
// reflectors or factor through one L2: logical x = (id / 8) % gx, y = id % 8
// + 8 ((id / 8) / gx).
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int id = blockIdx.x + gridDim.x * blockIdx.y;
  const int slot = id >> 3;
  bx = slot % gridDim.x;
  by = (id & 7) + 8 * (slot / gridDim.x);
}

// Partner of this lane at butterfly step STEP (its value of x): lane ^ STEP
// for 32 and 16 (LDS crossbar), the mirror within 16 or 8 lanes for 8 and 4,
// lane ^ 2 and lane ^ 1 for 2 and 1 (DPP).  Each pairs lanes that differ in
// bit log2(STEP) and agree in every higher bit.
template <int STEP>
__device__ __forceinline__ double bfly_partner(double x, int lane) {
  if constexpr (STEP == 32 || STEP == 16) {
    const int a = (lane ^ STEP) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(x));
    return __hiloint2double(hi, lo);
  } else if constexpr (STEP == 8) {
    return dpp_d<0x140>(x);   // row_mirror
  } else if constexpr (STEP == 4) {
    return dpp_d<0x141>(x);   // row_half_mirror
  } else if constexpr (STEP == 2) {
    return dpp_d<0x4E>(x);    // quad_perm [2,3,0,1]
  } else {
    return dpp_d<0xB1>(x);    // quad_perm [1,0,3,2]
  }
}

// One halving step of the transposed wave sum: the lane keeps the half of its
// N values selected by bit log2(STEP) of its id and adds its partner's copy of
// that half (the partner keeps the other half).
template <int N, int STEP>
__device__ __forceinline__ void bfly_halve(double* v, int lane) {
  const bool up = (lane & STEP) != 0;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double send = up ? v[i] : v[i + N / 2];
    const double keep = up ? v[i + N / 2] : v[i];
    v[i] = keep + bfly_partner<STEP>(send, lane);
  }
}

// Sums over the 64 lanes of a wave of each of NV (8, 16 or 32) per-lane
// values, transposed: halving steps with partners inside a 16-lane row (DPP:
// mirrors at 8 and 4, swaps at 2 and 1) leave one value per lane, then lanes
// holding the same column are folded (the steps left of 1, then 16 and 32
// through the LDS crossbar).  Lane l ends with the total of column
// wave_tsum_col<NV>(l); wave_tsum_writer<NV>(l) picks one lane per column.
template <int NV>
__device__ __forceinline__ int wave_tsum_col(int lane) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  if constexpr (NV == 32)
    return 16 * b3 + 8 * b2 + 4 * b1 + 2 * b0 + ((lane >> 4) & 1);
  else if constexpr (NV == 16)
    return 8 * b3 + 4 * b2 + 2 * b1 + b0;
  else
    return 4 * b3 + 2 * b2 + b1;
}

template <int NV>
__device__ __forceinline__ bool wave_tsum_writer(int lane) {
  if constexpr (NV == 32) return lane < 32;
  else if constexpr (NV == 16) return lane < 16;
  else return (lane & 0x31) == 0;
}

template <int NV>
__device__ __forceinline__ double wave_tsum(double (&v)[NV], int lane) {
  static_assert(NV == 8 || NV == 16 || NV == 32, "transposed wave sum of 8, 16 or 32 values");
  double t[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) t[i] = v[i];
  bfly_halve<NV, 8>(t, lane);
  bfly_halve<NV / 2, 4>(t, lane);
  bfly_halve<NV / 4, 2>(t, lane);
  if constexpr (NV >= 16) bfly_halve<NV / 8, 1>(t, lane);
  else t[0] += bfly_partner<1>(t[0], lane);
  if constexpr (NV >= 32) bfly_halve<NV / 16, 16>(t, lane);
  else t[0] += bfly_partner<16>(t[0], lane);
  t[0] += bfly_partner<32>(t[0], lane);
  return t[0];
}

// Sums of NV per-thread values over the workgroup, returned to every thread.
// NV = 1: DPP sum within each wave, one value per wave in red, every thread
// adds the NW of them (one barrier).  NV > 1: the transposed wave sum leaves
// each column's wave total in a few lanes, one of which writes it to red;
// NV threads add the NW rows and every thread reads the NV totals (two
// barriers).  red holds NW NV + NV doubles; callers alternate two such
// buffers.  The barriers order LDS only, so global loads issued before them
// (the next reflector) stay in flight.
template <int NV>
__device__ __forceinline__ void wg_sums(double (&v)[NV], double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if constexpr (NV == 1) {
    v[0] = wave_sum(v[0]);
    if (lane == 0) red[w] = v[0];
    lds_barrier();
    double t = red[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) t += red[q];
    v[0] = t;
  } else {
    const double s = wave_tsum<NV>(v, lane);
    if (wave_tsum_writer<NV>(lane)) red[w * NV + wave_tsum_col<NV>(lane)] = s;
    lds_barrier();
    if (tid < NV) {
      double t = red[tid];
#pragma unroll
      for (int q = 1; q < NW; ++q) t += red[q * NV + tid];
      red[NW * NV + tid] = t;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = red[NW * NV + k];
  }
}

// Householder QR with nonnegative diagonal of the mp x jb panel P0 (ld ld,
// jb <= 32, mp <= 512 U), with the output of wg_geqr2 (R on and above the
// diagonal, reflectors below it with unit leading entry implicit, tau).  The
// columns are held in registers CW at a time (a slab; U CW = 64): thread t
// holds rows t + 512 u of the slab.  A slab first takes the reflectors of the
// columns before it, one at a time (one workgroup sum of CW inner products
// each), then is factorised column by column: one workgroup sum for the
// column's norm below the diagonal, one for its inner products with the
// slab's later columns.  Each reflector follows wg_geqr2 (Parlett's form of
// the leading entry, the scaled path for columns near underflow, the identity
// when the column already lies along e_j), so both give the same factors up to
// the order of summation.  red: 2 x NW x CW doubles of LDS; bc: 1 double.
template <int U, int CW>
__device__ __forceinline__ void wg_panel_qr(double* P0, int mp, int jb, int64_t ld, double* tau, double* red,
                            double* bc, double* red2) {
  static_assert(U * CW == 64, "64 panel values per thread");
  const int tid = threadIdx.x;
  int ph = 0;
  double x[U][CW];
  for (int sb = 0; sb < jb; sb += CW) {
    const int cw = jb - sb < CW ? jb - sb : CW;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = tid + NT * u;
#pragma unroll
      for (int c = 0; c < CW; ++c)
        x[u][c] = (r < mp && c < cw) ? P0[(int64_t)(sb + c) * ld + r] : 0.0;
    }
    // the reflectors of columns 0 .. sb-1, in order (left-looking)
    double vn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = tid + NT * u;
      vn[u] = (sb > 0 && r > 0 && r < mp) ? P0[r] : (r == 0 ? 1.0 : 0.0);
    }
    for (int j = 0; j < sb; ++j) {
      double vj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) vj[u] = vn[u];
      const double tj = tau[j];
      if (j + 1 < sb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = tid + NT * u;
          vn[u] = (r > j + 1 && r < mp) ? P0[(int64_t)(j + 1) * ld + r] : (r == j + 1 ? 1.0 : 0.0);
        }
      }
      if (tj == 0.0) continue;   // uniform: tau is read by every thread
      double d[CW];
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) a += vj[u] * x[u][c];
        d[c] = a;
      }
      wg_sums<CW>(d, red + (ph++ & 1) * (NW + 1) * CW);
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const double f = tj * d[c];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u][c] -= f * vj[u];
      }
    }
    // the slab's own columns
    cfor<0, CW>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (c >= cw) return;
      const int jg = sb + c;
      double s2a[1] = {0.0};
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = tid + NT * u;
        if (r > jg && r < mp) s2a[0] += x[u][c] * x[u][c];
        if (r == jg) *bc = x[u][c];
      }
      wg_sums<1>(s2a, red + (ph++ & 1) * (NW + 1) * CW);
      double s2 = s2a[0];
      double alpha = *bc;
      double scl = 1.0;
      if (s2 > 0.0 && s2 < 0x1p-900 && !(alpha > 0.0 && s2 <= 0x1p-106 * alpha * alpha)) {
        double mx = fabs(alpha);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = tid + NT * u;
          if (r > jg && r < mp) mx = fmax(mx, fabs(x[u][c]));
        }
        mx = block_max(mx, red2);
        if (mx < 0x1p-1000) {
          s2 = 0.0;
        } else {
          const double inv = 1.0 / mx;
          double t2 = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int r = tid + NT * u;
            if (r > jg && r < mp) {
              const double t = x[u][c] * inv;
              t2 += t * t;
            }
          }
          s2 = block_sum(t2, red2);
          alpha *= inv;
          scl = mx;
        }
      }
      double tj, beta, inv_v0;
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
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = tid + NT * u;
        if (r > jg && r < mp) {
          x[u][c] *= inv_v0;
          v[u] = x[u][c];
        } else {
          v[u] = r == jg ? 1.0 : 0.0;
          if (r == jg) x[u][c] = beta;
        }
      }
      if (tid == 0) tau[jg] = tj;
      if constexpr (c + 1 < CW) {
        if (tj != 0.0 && c + 1 < cw) {
          double d[CW];
#pragma unroll
          for (int q = 0; q < CW; ++q) {
            double a = 0.0;
            if (q > c) {
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int r = tid + NT * u;
                // row jg of column q enters with v = 1 (x[u][q] there is its value)
                a += v[u] * x[u][q];
              }
            }
            d[q] = a;
          }
          wg_sums<CW>(d, red + (ph++ & 1) * (NW + 1) * CW);
#pragma unroll
          for (int q = c + 1; q < CW; ++q) {
            const double f = tj * d[q];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u][q] -= f * v[u];
          }
        }
      }
    });
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = tid + NT * u;
      if (r < mp) {
#pragma unroll
        for (int c = 0; c < CW; ++c)
          if (c < cw) P0[(int64_t)(sb + c) * ld + r] = x[u][c];
      }
    }
    __syncthreads();
  }
}

// Whether core i sends its MPO to the wide launches: a panel wider than the
// register path and at least wmin columns, or (only at the default wmin) a
// last-core panel beyond the TSQR leaves.  A last core of at most 256 columns
// does not count: it stays with the rest of its MPO on the one-workgroup path
// (one blocked QR there costs less than taking every core of the MPO through
// the wide launches).  Larger wmin leave more MPOs on the one-workgroup path
// (a choice of the sweep autotuner).
__device__ __forceinline__ bool wide_core(int i, int d, int n, int P, int rnext, int wmin) {
  if (i == 0) return false;
  if (P > kRegCols && P >= wmin && (i < d - 1 || P > 2 * kRegCols)) return true;
  return wmin <= kRegCols + 1 && i == d - 1 && n * rnext > kTsqrLeavesMax * kRegRows;
}

// One workgroup: need[t * kWidePlan + .] = maxima over the wide MPOs of
// (column blocks, P, n rho', rho', n) at step t; wflag[b] = 1 for the MPOs the
// wide launches take.  With a plan, an MPO is taken only if every step fits
// it; without one the caller launches from `need`.
__global__ __launch_bounds__(512) void k_wide_classify(const MpoDesc* mpos,
                                                       const CoreDesc* cores, int batch, int op,
                                                       const int* pr, const int* plan,
                                                       int max_d, int wmin, int* wflag,
                                                       int* need) {
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
      if (wide_core(i, d, n, P, rn, wmin)) wide = true;
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
                                                  const double* L, int batch) {
  __shared__ double lds[GEMM_LDS];
  int bx, b;
  xcd_tile(bx, b);
  if (b >= batch || !wflag[b]) return;
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
    for (int64_t o = (int64_t)bx * NT + threadIdx.x; o < tot; o += (int64_t)gridDim.x * NT)
      Xt[o] = (double)Zc[o];
    return;
  }
  const int rnext = rho[md.r0 + i + 1];
  const int Pn = pr[md.r0 + i + 1];
  const int m = n * rnext;
  int x = bx;
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

// Shapes of core i = d - 1 - t of a wide MPO at step t; false when the MPO
// has no such core with a QR (core 0 is absorbed only).
struct WideCore {
  int i, n, P, m, kmax;
};
__device__ __forceinline__ bool wide_core_at(const MpoDesc& md, const CoreDesc* cores, int op,
                                             const int* pr, const int* rho, int t, CoreDesc& cd,
                                             WideCore& wc) {
  wc.i = md.d - 1 - t;
  if (wc.i < 1) return false;
  cd = cores[md.c0 + wc.i];
  wc.n = op == 0 ? cd.I : cd.J;
  wc.P = pr[md.r0 + wc.i];
  const int rnext = (wc.i == md.d - 1) ? md.K : rho[md.r0 + wc.i + 1];
  wc.m = wc.n * rnext;
  wc.kmax = wc.m < wc.P ? wc.m : wc.P;
  return true;
}

// Step t, column block j of core i = d - 1 - t: strip s (SW columns) of the
// trailing columns takes C <- (I - V T V^T)^T C = C - V (C^T V T)^T with the
// explicit reflectors V of block j (buffer j & 1) and its T.  A small LDS
// footprint keeps two workgroups per compute unit.
__global__ __launch_bounds__(NT, 2) void k_wide_update(const MpoDesc* mpos, const CoreDesc* cores,
                                                    int op, const int* pr, const int* rho,
                                                    const int* wflag, int t, int j, double* Wd,
                                                    const double* WV, int batch) {
  __shared__ double sm[2 * SW * NB + NB * NB];
  const int tid = threadIdx.x;
  int bx, b;
  xcd_tile(bx, b);
  if (b >= batch || !wflag[b]) return;
  const MpoDesc md = mpos[b];
  CoreDesc cd;
  WideCore wc;
  if (!wide_core_at(md, cores, op, pr, rho, t, cd, wc)) return;
  const int j0 = NB * j;
  if (j0 >= wc.kmax) return;
  const int jb = wc.kmax - j0 < NB ? wc.kmax - j0 : NB;
  const int mp = wc.m - j0;
  const int c0 = j0 + jb + SW * bx;
  const int cs = wc.P - c0 < SW ? wc.P - c0 : SW;
  if (cs <= 0) return;
  double* Wt = sm;                  // C^T V, cs x jb (ld NB)
  double* W2t = sm + SW * NB;       // C^T V T
  double* Ts = sm + 2 * SW * NB;    // T, row-major NB x NB
  const double* Vp = WV + md.wv_off + (int64_t)(j & 1) * md.wmcap * NB;
  const double* Tb = Wd + cd.wt_off;
  for (int e = tid; e < NB * NB; e += NT) Ts[e] = Tb[(int64_t)j * NB * NB + e];
  __syncthreads();
  double* C = Wd + cd.w_off + (int64_t)c0 * wc.m + j0;
  // W^T = C^T V (cs x jb), split over K = mp rows on the matrix cores
  wg_atb<SW / 16, NB / 16>(cs, jb, mp, C, wc.m, Vp, mp, Wt);
  // W2^T = W^T T (T upper triangular)
  for (int e = tid; e < cs * jb; e += NT) {
    const int i = e / jb, q = e - i * jb;
    double acc = 0.0;
    for (int r = 0; r <= q; ++r) acc += Wt[i * NB + r] * Ts[r * NB + q];
    W2t[i * NB + q] = acc;
  }
  __syncthreads();
  // C -= V W2 (W2 element (q, i) = W2t[i NB + q]), by 16-row blocks
  wg_ab_rows<SW / 16>(mp, cs, jb, -1.0, Vp, mp, W2t, 1, NB, C, wc.m);
}

// Step t: the Householder QR of column block j of core i = d - 1 - t (rows from
// its diagonal down, in place), then its reflectors written explicitly to
// buffer j & 1 and its T factor.  BIG = false takes panels of at most 4096
// rows (held in registers, small LDS); BIG = true the taller ones (blocked, in
// LDS or global memory).
template <bool BIG>
__global__ __launch_bounds__(NT) void k_wide_panel(const MpoDesc* mpos, const CoreDesc* cores,
                                                   int op, const int* pr, const int* rho,
                                                   const int* wflag, int t, int j, double* Wd,
                                                   double* WV, double* tau) {
  constexpr int AR = BIG ? WARENA : 2 * (NW + 1) * 32 + 64 + 2 * QBMAX * QBMAX;
  __shared__ double arena[AR];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  if (!wflag[b]) return;
  const MpoDesc md = mpos[b];
  CoreDesc cd;
  WideCore wc;
  if (!wide_core_at(md, cores, op, pr, rho, t, cd, wc)) return;
  const int j0 = NB * j;
  if (j0 >= wc.kmax) return;
  const int jb = wc.kmax - j0 < NB ? wc.kmax - j0 : NB;
  const int mp = wc.m - j0;
  if (BIG != (mp > 8 * NT)) return;
  double* Xt = Wd + cd.w_off;
  double* P0 = Xt + (int64_t)j0 * wc.m + j0;
  double* taui = tau + cd.tau_off + j0;
  double* Ts = arena + AR - 32 - 2 * QBMAX * QBMAX;
  double* Gs = Ts + QBMAX * QBMAX;
  double* red = arena + AR - 16;
  if constexpr (BIG) {
    double* qws = WV + md.wv_off + 2 * (int64_t)md.wmcap * NB;   // wmcap * 16 + 1024
    wg_geqrf_impl<true>(P0, mp, jb, taui, arena, red, qws, arena, RCAP, Ts, Gs, wc.m, QBMAX);
  } else {
    double* pred = arena;            // 2 (NW + 1) 32 doubles
    double* pbc = arena + 2 * (NW + 1) * 32;
    if (mp <= 2 * NT)
      wg_panel_qr<2, 32>(P0, mp, jb, wc.m, taui, pred, pbc, red);
    else if (mp <= 4 * NT)
      wg_panel_qr<4, 16>(P0, mp, jb, wc.m, taui, pred, pbc, red);
    else
      wg_panel_qr<8, 8>(P0, mp, jb, wc.m, taui, pred, pbc, red);
  }
  double* Vp = WV + md.wv_off + (int64_t)(j & 1) * md.wmcap * NB;
  for (int64_t e = tid; e < (int64_t)mp * jb; e += NT) {
    const int c = (int)(e / mp), r = (int)(e - (int64_t)c * mp);
    Vp[e] = r > c ? P0[(int64_t)c * wc.m + r] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  wg_build_t_splitk(Vp, mp, jb, taui, Ts, Gs);
  double* Tb = Wd + cd.wt_off;
  for (int e = tid; e < NB * NB; e += NT) Tb[(int64_t)j * NB * NB + e] = Ts[e];
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
                                const int* pr, const int* plan, int max_d, int wmin, int* wflag,
                                int* need, hipStream_t s) {
  k_wide_classify<<<1, 512, 0, s>>>(mpos, cores, batch, op, pr, plan, max_d, wmin, wflag, need);
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
  const int gy = (batch + 7) / 8 * 8;   // whole groups of 8 for the XCD mapping
  by_dtype(dtype, [&](auto* tp) {
    using T = elem_t<decltype(tp)>;
    k_wide_load<T><<<dim3(gx, gy), NT, 0, s>>>(mpos, cores, op, pr, rho, wflag, t, tf_n, tp_n,
                                               (const T*)Z, Wd, L, batch);
  });
  const bool big = mm > 8 * NT;   // some panel taller than the register path
  // update(jj) after the panel of block jj: the columns right of it, which
  // start at NB jj + 1 or later (a last block may be narrower than NB)
  auto update = [&](int jj) {
    const int rest = Pm - NB * jj - 1;
    if (rest > 0)
      k_wide_update<<<dim3((rest + SW - 1) / SW, gy), NT, 0, s>>>(mpos, cores, op, pr, rho,
                                                                  wflag, t, jj, Wd, WV, batch);
  };
  for (int j = 0; j < nb; ++j) {
    if (j > 0) update(j - 1);
    k_wide_panel<false><<<batch, NT, 0, s>>>(mpos, cores, op, pr, rho, wflag, t, j, Wd, WV, tau);
    if (big)
      k_wide_panel<true><<<batch, NT, 0, s>>>(mpos, cores, op, pr, rho, wflag, t, j, Wd, WV, tau);
  }
  if (nb > 0) update(nb - 1);
  k_wide_finish<<<dim3(tp_n, batch), NT, 0, s>>>(mpos, cores, op, pr, rho, ldm, wflag, t, Wd, L);
  return hipGetLastError();
}

}  // namespace tnr
