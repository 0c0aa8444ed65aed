// Host runtime behind include/tnrsvd.h: validation, merge plan, capacity plan,
// device slabs, the call-order state machine of Algorithm 5.4, and launches.
// No step of the method runs on the host: shapes are planned here, all
// arithmetic runs in the kernels of kernels_contract.hip / kernels_sweep.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <chrono>
#include <climits>
#include <vector>

#include "../../include/tnrsvd.h"
#include <array>

#include "tnrsvd_internal.h"


using namespace tnr;

namespace {

thread_local std::string g_err;

tnrsvd_status fail(tnrsvd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

constexpr int64_t kSat = int64_t(1) << 40;   // saturation of mode-size products
constexpr int64_t kHardCap = 4096;           // largest bond rank a plan may reserve

inline int64_t sat_mul(int64_t a, int64_t b) {
  if (a >= kSat || b >= kSat) return kSat;
  const __int128 r = (__int128)a * b;   // exact: |a|, |b| < 2^63
  return r > kSat ? kSat : (r < -kSat ? -kSat : (int64_t)r);
}

enum Space { kNone = 0, kRow = 1, kCol = 2 };

constexpr int kKinds = 7;  // contract, rl, lr, form_u, load_omega, copy_y0, sketch

}  // namespace

struct tnrsvd_s {
  int device = 0;
  int leaf_nc = 0;   // most TSQR leaves of a last-core panel over the batch (grid of k_rl_leaves)
  // TNRSVD_K_FIRST: the caller's MPO b was read reversed (core i of the caller is
  // core d - 1 - i here, rank legs swapped); paper_shape[b] keeps the caller's cores
  int orientation = 0;
  std::vector<std::vector<std::array<int64_t, 4>>> paper_shape;
  hipStream_t stream = nullptr;
  int batch = 0;
  int dtype = 0;         // contraction storage of A, X, Z: kF64, kF32 or kBF16
  int y0_dtype = 0;      // storage of the Y0 slab (the creation precision)
  // BF16 handles keep FP32 copies of A, X and Z for tnrsvd_refine; `refined`
  // says the FP32 set is the active one (swapped into A, X, Z)
  void *A32 = nullptr, *X32 = nullptr, *Z32 = nullptr;
  bool refined = false;
  int64_t x_elems = 0;
  tnrsvd_opts opts{};
  std::vector<MpoDesc> mh;
  std::vector<CoreDesc> ch;
  std::vector<int> core_mpo;
  int ncores = 0, max_d = 0;
  int64_t max_core_out = 1, max_om = 1, max_y0 = 1;
  int vcap = 64, scap = 64;
  int64_t tcap = 1, mcap_s = 1, ucap = 1, qcap = 1;
  // device buffers
  MpoDesc* mpos_d = nullptr;
  CoreDesc* cores_d = nullptr;
  int* core_mpo_d = nullptr;
  int *xr = nullptr, *vr = nullptr, *pr = nullptr, *rho = nullptr, *ldm = nullptr,
      *err = nullptr;
  void *A = nullptr, *X = nullptr, *Z = nullptr, *Y0 = nullptr;
  double *W = nullptr, *L = nullptr, *tau = nullptr, *scratch = nullptr, *outs = nullptr,
         *om = nullptr, *U = nullptr, *V = nullptr;
  std::vector<void*> allocs;
  // state machine
  int space = kNone;     // where the current basis lives
  int pending = -1;      // op of a pending product, -1 none
  bool projected = false;
  bool solved = false;
  bool y0_valid = false;
  bool first_product = true;
  // measurement: event pairs per kernel kind
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[kKinds];
  // captured whole-solve graph (tnrsvd_run_graph): a private default-priority
  // stream that owns the capture and the replays, joined to `stream` by events
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t gev[2] = {nullptr, nullptr};
  // backward: input dtype, original core count and merge count per MPO; the
  // original trailing cores that were merged (FP64, kept for the merge
  // adjoint); gradient buffers planned at the first tnrsvd_backward
  std::vector<int> in_dtype, d_orig, mcount;
  std::vector<std::vector<int64_t>> tail_off;
  std::vector<std::vector<std::array<int, 4>>> tail_shape;
  double* tail = nullptr;
  // sketched product truncation (opts.sketch_rank > 0): per-MPO FP64 workspace
  double* sk = nullptr;
  int64_t* sk_off_d = nullptr;
  int* sk_nm_d = nullptr;
  int prod_t = 0;   // products since the first of the solve (the sketch's stream index)
  bool grad_ready = false;
  GradMpo* gm_d = nullptr;
  int64_t* eoff_d = nullptr;
  double *gws = nullptr, *gG = nullptr, *gw = nullptr, *gchain = nullptr;
  int64_t a_elems = 0, chain_cap = 0;
  // launch shape of the contraction per op (threads per block, blocks per core
  // cap), from tnrsvd_autotune
  int ct_threads[2] = {256, 256}, ct_cap[2] = {256, 256};
  // multi-workgroup right-to-left path (kernels_wide.hip): whether the rank
  // capacities allow a panel beyond the register path; per MPO flag; the
  // device-side needs of the current rounding; the capacity plan; the plan of
  // each rounding of a solve as last measured (used when a solve is captured)
  // MPOs in decreasing order of a sweep-cost estimate (sum over cores of n P^2),
  // the order the one-workgroup-per-MPO sweeps dispatch them in
  int* order_d = nullptr;
  std::vector<int> order;
  // sweep launch choices (tnrsvd_autotune_sweeps / tnrsvd_set_sweep_config):
  // the fewest product columns that send an MPO to the wide launches (above
  // the register path), and whether the sweeps dispatch costliest MPOs first
  int wide_min_p = kRegCols + 1;
  bool lpt = true;
  // ranks kept by each rounding of the current solve (slots of d + 1 per MPO),
  // its product (0: A X, 1: A^T X) and whether it was the solve's SVD, for
  // tnrsvd_backward
  int* rhist_d = nullptr;
  int hist_slots = 0, r_tot = 0;
  std::vector<int> hist_op, hist_svd;
  bool wide_possible = false;
  double* WV = nullptr;
  int *wflag_d = nullptr, *wneed_d = nullptr, *wcap_d = nullptr, *wplan_d = nullptr;
  std::vector<int> wcap;
  std::vector<std::vector<int>> wplan;
  std::vector<int> wscratch;
  int wslots = 0;
  int round_idx = 0;
};

namespace {

template <typename P>
tnrsvd_status dalloc(tnrsvd_s* h, P** out, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TNRSVD_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  h->allocs.push_back(p);
  *out = (P*)p;
  return TNRSVD_OK;
}

void release(tnrsvd_s* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

size_t elem_size(int dt) {
  return dt == kF64 ? sizeof(double) : (dt == kF32 ? sizeof(float) : sizeof(bf16));
}

tnrsvd_status dev_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TNRSVD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }
  return TNRSVD_OK;
}

#define TRY(x)                               \
  do {                                       \
    const tnrsvd_status st_ = (x);           \
    if (st_ != TNRSVD_OK) return st_;        \
  } while (0)

// Validate one MPO and return the merge count m (last m cores become one).
tnrsvd_status plan_mpo(const tnrsvd_mpo& a, int K, int* m_out) {
  if (a.d < 1) return fail(TNRSVD_E_SHAPE, "d must be >= 1");
  if (!a.rank || !a.rows || !a.cols || !a.core)
    return fail(TNRSVD_E_INVALID, "null rank/rows/cols/core array");
  if (a.dtype != TNRSVD_F64 && a.dtype != TNRSVD_F32)
    return fail(TNRSVD_E_INVALID, "core dtype must be TNRSVD_F64 or TNRSVD_F32");
  if (a.rank[0] != 1 || a.rank[a.d] != 1)
    return fail(TNRSVD_E_SHAPE, "rank[0] and rank[d] must be 1");
  for (int i = 0; i < a.d; ++i) {
    if (a.rows[i] < 1 || a.cols[i] < 1 || a.rank[i + 1] < 1)
      return fail(TNRSVD_E_SHAPE, "core %d: non-positive dimension or rank", i);
    if (a.rank[i] > 65536 || a.rows[i] > 65536 || a.cols[i] > 65536)
      return fail(TNRSVD_E_SHAPE, "core %d: dimension too large", i);
    if (!a.core[i]) return fail(TNRSVD_E_INVALID, "core %d: null pointer", i);
  }
  int64_t pi = 1, pj = 1;
  for (int m = 1; m <= a.d; ++m) {
    pi = sat_mul(pi, a.rows[a.d - m]);
    pj = sat_mul(pj, a.cols[a.d - m]);
    if (pi >= K && pj >= K) {
      *m_out = m;
      return TNRSVD_OK;
    }
  }
  return fail(TNRSVD_E_SHAPE, "prod(I) = %lld or prod(J) = %lld is smaller than K = %d",
              (long long)pi, (long long)pj, K);
}

}  // namespace

extern "C" {

const char* tnrsvd_last_error(void) { return g_err.c_str(); }

const char* tnrsvd_version(void) { return "tnrsvd-gfx950 0.1"; }

tnrsvd_status tnrsvd_destroy(tnrsvd_t h) {
  if (!h) return TNRSVD_OK;
  (void)hipStreamSynchronize(h->stream);
  if (h->gstream) (void)hipStreamSynchronize(h->gstream);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (hipEvent_t e : h->gev)
    if (e) (void)hipEventDestroy(e);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  release(h);
  delete h;
  return TNRSVD_OK;
}

// Checks of the scalar options (no device call).
static tnrsvd_status check_opts(const tnrsvd_opts* o) {
  if (o->k < 1 || o->p < 0 || o->q < 0)
    return fail(TNRSVD_E_INVALID, "need k >= 1, p >= 0, q >= 0");
  if (o->k + o->p > kMaxK) return fail(TNRSVD_E_INVALID, "K = k + p must be <= %d", kMaxK);
  if (o->precision != TNRSVD_F64 && o->precision != TNRSVD_F32 && o->precision != TNRSVD_BF16)
    return fail(TNRSVD_E_INVALID, "unknown precision %d", o->precision);
  if (!(o->round_tol >= 0.0) || !std::isfinite(o->round_tol))
    return fail(TNRSVD_E_INVALID, "round_tol must be finite and >= 0");
  if (o->max_rank < 0) return fail(TNRSVD_E_INVALID, "max_rank must be >= 0");
  if (o->sketch_rank < 0 || o->sketch_rank > 256)
    return fail(TNRSVD_E_INVALID, "sketch_rank must be in [0, 256]");
  if (o->orientation != TNRSVD_K_LAST && o->orientation != TNRSVD_K_FIRST)
    return fail(TNRSVD_E_INVALID, "unknown orientation %d", o->orientation);
  return TNRSVD_OK;
}

static tnrsvd_status create_lib(tnrsvd_t* out, int batch, const tnrsvd_mpo* mpos,
                                const tnrsvd_opts* o) {
  g_err.clear();
  if (!out || !mpos || !o) return fail(TNRSVD_E_INVALID, "null argument");
  *out = nullptr;
  if (batch < 1) return fail(TNRSVD_E_INVALID, "batch must be >= 1");
  TRY(check_opts(o));
  const int K = o->k + o->p;

  std::vector<int> merge(batch);
  for (int b = 0; b < batch; ++b) TRY(plan_mpo(mpos[b], K, &merge[b]));
  // original trailing cores kept in FP64 for the merge adjoint of tnrsvd_backward
  std::vector<std::vector<int64_t>> tail_off(batch);
  std::vector<std::vector<std::array<int, 4>>> tail_shape(batch);
  int64_t tail_tot = 0;
  for (int b = 0; b < batch; ++b) {
    const tnrsvd_mpo& a = mpos[b];
    if (merge[b] < 2) continue;
    for (int j = a.d - merge[b]; j < a.d; ++j) {
      tail_off[b].push_back(tail_tot);
      tail_shape[b].push_back({(int)a.rank[j], (int)a.rows[j], (int)a.cols[j], (int)a.rank[j + 1]});
      tail_tot += a.rank[j] * a.rows[j] * a.cols[j] * a.rank[j + 1];
    }
  }

  tnrsvd_s* h = new (std::nothrow) tnrsvd_s();
  if (!h) return fail(TNRSVD_E_NOMEM, "host allocation failed");
  h->batch = batch;
  h->opts = *o;
  h->stream = (hipStream_t)o->stream;
  h->dtype = o->precision == TNRSVD_F64 ? kF64 : (o->precision == TNRSVD_F32 ? kF32 : kBF16);
  for (int b = 0; b < batch; ++b) {
    h->in_dtype.push_back(mpos[b].dtype == TNRSVD_F64 ? kF64 : kF32);
    h->d_orig.push_back(mpos[b].d);
    h->mcount.push_back(merge[b]);
  }
  h->tail_off = tail_off;
  h->tail_shape = tail_shape;
  h->y0_dtype = h->dtype;
  (void)hipGetDevice(&h->device);
  const int64_t rmax = o->max_rank;

  // ---- capacity plan -----------------------------------------------------
  int64_t a_tot = 0, x_tot = 0, z_tot = 0, w_tot = 0, l_tot = 0, t_tot = 0, y_tot = 0,
          u_tot = 0, om_tot = 0, s_tot = 0, out_tot = 0, wv_tot = 0;
  std::vector<int> sk_nm;
  int r_tot = 0;
  int64_t tcap = 1, mcap_s = 1, ucap = 1, qcap = 1;
  int vcap = 64, scap = K;
  for (int b = 0; b < batch; ++b) {
    const tnrsvd_mpo& a = mpos[b];
    const int m = merge[b];
    const int dm = a.d - m + 1;
    std::vector<int64_t> I(dm), J(dm), R(dm + 1);
    for (int i = 0; i < dm - 1; ++i) {
      I[i] = a.rows[i];
      J[i] = a.cols[i];
      R[i] = a.rank[i];
    }
    I[dm - 1] = 1;
    J[dm - 1] = 1;
    for (int i = dm - 1; i < a.d; ++i) {
      I[dm - 1] *= a.rows[i];
      J[dm - 1] *= a.cols[i];
    }
    R[dm - 1] = a.rank[dm - 1];
    R[dm] = 1;
    if (I[dm - 1] > 65536 || J[dm - 1] > 65536) {
      delete h;
      return fail(TNRSVD_E_SHAPE, "merged core too large (%lld x %lld)", (long long)I[dm - 1],
                  (long long)J[dm - 1]);
    }
    // bond capacities of the basis: Theorem 3.2 style bounds, the cap, growth
    std::vector<int64_t> xc(dm + 1);
    xc[0] = 1;
    xc[dm] = K;
    for (int i = 1; i < dm; ++i) {
      int64_t li = 1, lj = 1, ri = K, rj = K;
      for (int j = 0; j < i; ++j) {
        li = sat_mul(li, I[j]);
        lj = sat_mul(lj, J[j]);
      }
      for (int j = i; j < dm; ++j) {
        ri = sat_mul(ri, I[j]);
        rj = sat_mul(rj, J[j]);
      }
      int64_t cap = std::min(std::max(li, lj), std::max(ri, rj));
      if (rmax > 0) cap = std::min<int64_t>(cap, rmax);
      // without a cap, ranks of the rounded products are bounded by R^(2q+2)
      int64_t g = 1;
      // (a BF16 handle plans one more power step for tnrsvd_refine)
      const int qp = o->q + (o->precision == TNRSVD_BF16 ? 1 : 0);
      for (int t = 0; t < 2 * qp + 2; ++t) g = sat_mul(g, R[i]);
      cap = std::min(cap, std::max<int64_t>(g, 1));
      if (cap > kHardCap) {
        delete h;
        return fail(TNRSVD_E_SHAPE,
                    "MPO %d bond %d would need rank capacity %lld > %lld; set max_rank", b, i,
                    (long long)cap, (long long)kHardCap);
      }
      xc[i] = cap;
    }
    MpoDesc md{};
    md.d = dm;
    md.K = K;
    md.c0 = (int)h->ch.size();
    md.r0 = r_tot;
    r_tot += dm + 1;
    md.om_off = om_tot;
    int64_t omn = 0;
    for (int i = 0; i < dm - 1; ++i) omn += J[i];
    omn += J[dm - 1] * K;
    om_tot += omn;
    h->max_om = std::max(h->max_om, omn);
    int64_t mpo_t = 1, mpo_m = 1, mpo_u = 1, mpo_q = 1, mpo_pc = 1, mpo_nm = 1;
    int mpo_v = 64;
    // multi-workgroup path: possible when some core i >= 1 may have more than
    // kRegCols product columns, or a last-core panel beyond the TSQR leaves
    bool mpo_wide = false;
    int64_t mpo_wm = 0;
    {
      int64_t rn = K;
      for (int i = dm - 1; i >= 0; --i) {
        const int64_t nmax = std::max(I[i], J[i]);
        const int64_t P = R[i] * xc[i];
        const int64_t m = nmax * rn;
        if (i >= 1 && (P > kRegCols || (i == dm - 1 && m > (int64_t)kTsqrLeavesMax * kRegRows)))
          mpo_wide = true;
        rn = std::min(m, P);
      }
    }
    for (int i = 0; i < dm; ++i) {
      CoreDesc cd{};
      cd.I = (int)I[i];
      cd.J = (int)J[i];
      cd.RA = (int)R[i];
      cd.RA2 = (int)R[i + 1];
      cd.xcap = (int)xc[i];
      cd.xcap2 = (int)xc[i + 1];
      const int64_t nmax = std::max(I[i], J[i]);
      const int64_t P = R[i] * xc[i], P2 = R[i + 1] * xc[i + 1];
      mpo_pc = std::max(mpo_pc, P);
      mpo_nm = std::max(mpo_nm, nmax);
      // register panels pad each y block of rows to a power of two (>= 16)
      int64_t P2pad = 16;
      while (P2pad < P2) P2pad *= 2;
      cd.a_off = a_tot;
      a_tot += R[i] * I[i] * J[i] * R[i + 1];
      cd.x_off = x_tot;
      cd.u_off = x_tot;
      x_tot += xc[i] * nmax * xc[i + 1];
      cd.z_off = z_tot;
      z_tot += P * nmax * P2;
      cd.w_off = w_tot;
      int64_t wneed = nmax * P2pad * P;
      if (i == dm - 1) {
        // a tall last-core panel may be factorised by TSQR: leaf + merge
        // reflectors (2 nc blocks of 256 x P), two P x P factors, 2 nc taus,
        // and the R factors of leaves 1 .. nc-1 (P x P each)
        // (the rank in force may be below P and the mode below nmax, so the
        // leaf count and width are bounded by the register panel's limits)
        const int64_t nc = (nmax * K + kRegRows - 1) / kRegRows;
        const int64_t ncl = std::min<int64_t>(nc, kTsqrLeavesMax);
        const int64_t Pl = std::min<int64_t>(P, kRegCols);
        wneed = std::max(wneed, (2 * nc * kRegRows + 2 * P) * P + 2 * nc * P +
                                    (ncl > 1 ? (ncl - 1) * Pl * Pl : 0));
        if (ncl > 1) h->leaf_nc = std::max(h->leaf_nc, (int)ncl);
      }
      // the blocked QR of the global path needs m qb + 2 qb P more (qb <= 32)
      wneed += nmax * P2pad * 32 + 2 * 32 * P;
      cd.wt_off = w_tot + wneed;
      if (mpo_wide) {
        wneed += (int64_t)kWideNB * kWideNB * ((P + kWideNB - 1) / kWideNB);
        mpo_wm = std::max(mpo_wm, nmax * P2pad);
      }
      w_tot += wneed;
      cd.l_off = l_tot;
      l_tot += P * P;
      cd.tau_off = t_tot;
      t_tot += P;
      cd.y0_off = y_tot;
      y_tot += R[i] * I[i] * R[i + 1] * (i == dm - 1 ? K : 1);
      h->max_core_out = std::max(h->max_core_out, P * nmax * P2);
      mpo_t = std::max(mpo_t, xc[i] * P);
      mpo_t = std::max(mpo_t, xc[i + 1] * P2);
      mpo_m = std::max(mpo_m, xc[i] * nmax * P2pad);
      mpo_v = (int)std::max<int64_t>(mpo_v, nmax * P2);
      const int64_t nv = xc[i] * nmax;
      // QR-preconditioned Jacobi of the left-to-right pass: blocked QR of the
      // transposed panel (P2 rows, nv columns) and its scalars
      // (and R^T, nv x nv, when it does not fit in LDS)
      mpo_q = std::max(mpo_q, P2 * 16 + 2 * 16 * nv + nv + (i < dm - 1 ? nv * nv : 0));
      if (i < dm - 1) {
        scap = (int)std::max<int64_t>(scap, nv);
        mpo_u = std::max(mpo_u, nv * nv);
      } else {
        mpo_v = (int)std::max<int64_t>(mpo_v, nv);
        mpo_u = std::max(mpo_u, 2 * nv * K + K + (int64_t)K * K);
      }
      h->ch.push_back(cd);
      h->core_mpo.push_back(b);
    }
    md.s_off = s_tot;
    md.s_len = mpo_t + mpo_m + mpo_u + mpo_q;
    s_tot += md.s_len;
    md.out_off = out_tot;
    out_tot += K + 2 * (int64_t)K * K;
    md.mcap = mpo_v;
    md.pcap = (int)mpo_pc;
    md.wv_off = wv_tot;
    md.wmcap = (int)mpo_wm;
    if (mpo_wide) {
      h->wide_possible = true;
      wv_tot += 2 * mpo_wm * kWideNB + mpo_wm * 16 + 1024;
    }
    // capacity plan of the wide launches at each step t (core dm - 1 - t)
    if ((int)h->wcap.size() < kWidePlan * dm) h->wcap.resize(kWidePlan * dm, 0);
    if (mpo_wide) {
      int64_t rn = K;
      for (int i = dm - 1; i >= 0; --i) {
        const int64_t nmax = std::max(I[i], J[i]);
        const int64_t P = R[i] * xc[i];
        const int64_t m = nmax * rn;
        const int64_t k = std::min(m, P);
        const int64_t v[kWidePlan] = {i >= 1 ? (k + kWideNB - 1) / kWideNB : 0, P, m, rn, nmax};
        const int t = dm - 1 - i;
        for (int c = 0; c < kWidePlan; ++c)
          h->wcap[t * kWidePlan + c] = (int)std::max<int64_t>(h->wcap[t * kWidePlan + c], v[c]);
        rn = k;
      }
    }
    sk_nm.push_back((int)mpo_nm);
    tcap = std::max(tcap, mpo_t);
    mcap_s = std::max(mcap_s, mpo_m);
    ucap = std::max(ucap, mpo_u);
    qcap = std::max(qcap, mpo_q);
    vcap = std::max(vcap, mpo_v);
    h->max_d = std::max(h->max_d, dm);
    h->mh.push_back(md);
  }
  // every MPO's scratch uses the global maxima so the kernels share one layout
  s_tot = 0;
  for (auto& md : h->mh) {
    md.s_off = s_tot;
    md.s_len = tcap + mcap_s + ucap + qcap;
    s_tot += md.s_len;
  }
  h->ncores = (int)h->ch.size();
  h->vcap = vcap;
  h->scap = scap;
  h->tcap = tcap;
  h->mcap_s = mcap_s;
  h->ucap = ucap;
  h->qcap = qcap;
  if (vcap > kSweepArena - 64 - 2 * 32 * 32 || scap > kSortCap) {
    delete h;
    return fail(TNRSVD_E_SHAPE,
                "panels too large for one workgroup (rows %d, sorted vectors %d); lower max_rank",
                vcap, scap);
  }
  const size_t esz = elem_size(h->dtype);
  h->x_elems = x_tot;

  // ---- allocation ---------------------------------------------------------
  tnrsvd_status st = TNRSVD_OK;
#define ALLOC(ptr, bytes)                         \
  do {                                            \
    st = dalloc(h, &(ptr), (bytes));              \
    if (st != TNRSVD_OK) {                        \
      release(h);                                 \
      delete h;                                   \
      return st;                                  \
    }                                             \
  } while (0)
  ALLOC(h->mpos_d, sizeof(MpoDesc) * batch);
  ALLOC(h->cores_d, sizeof(CoreDesc) * h->ncores);
  ALLOC(h->core_mpo_d, sizeof(int) * h->ncores);
  ALLOC(h->xr, sizeof(int) * r_tot);
  ALLOC(h->vr, sizeof(int) * r_tot);
  ALLOC(h->pr, sizeof(int) * r_tot);
  ALLOC(h->rho, sizeof(int) * r_tot);
  ALLOC(h->ldm, sizeof(int) * r_tot);
  ALLOC(h->err, sizeof(int) * 4);
  ALLOC(h->A, esz * a_tot);
  ALLOC(h->X, esz * x_tot);
  ALLOC(h->Z, esz * z_tot);
  ALLOC(h->Y0, esz * y_tot);
  if (h->dtype == kBF16) {
    ALLOC(h->A32, sizeof(float) * a_tot);
    ALLOC(h->X32, sizeof(float) * x_tot);
    ALLOC(h->Z32, sizeof(float) * z_tot);
  }
  ALLOC(h->W, sizeof(double) * w_tot);
  ALLOC(h->L, sizeof(double) * l_tot);
  ALLOC(h->tau, sizeof(double) * t_tot);
  ALLOC(h->scratch, sizeof(double) * s_tot);
  ALLOC(h->outs, sizeof(double) * out_tot);
  ALLOC(h->om, sizeof(double) * om_tot);
  ALLOC(h->U, sizeof(double) * x_tot);
  ALLOC(h->V, sizeof(double) * x_tot);
  ALLOC(h->tail, sizeof(double) * tail_tot);
  ALLOC(h->order_d, sizeof(int) * batch);
  h->hist_slots = 2 * o->q + 5;
  h->r_tot = r_tot;
  ALLOC(h->rhist_d, sizeof(int) * r_tot * h->hist_slots);
  if (h->wide_possible) {
    h->wcap.resize((size_t)kWidePlan * h->max_d, 0);
    // one plan slot per rounding of a solve (2q + 2), three more for tnrsvd_refine
    h->wslots = 2 * o->q + 5;
    h->wplan.assign(h->wslots, std::vector<int>());
    ALLOC(h->WV, sizeof(double) * wv_tot);
    ALLOC(h->wflag_d, sizeof(int) * batch);
    ALLOC(h->wneed_d, sizeof(int) * kWidePlan * h->max_d);
    ALLOC(h->wcap_d, sizeof(int) * kWidePlan * h->max_d);
    ALLOC(h->wplan_d, sizeof(int) * kWidePlan * h->max_d * h->wslots);
  }
  std::vector<int64_t> sk_off;
  if (o->sketch_rank > 0) {
    int64_t sk_tot = 0;
    for (int b = 0; b < batch; ++b) {
      sk_off.push_back(sk_tot);
      sk_tot += sketch_ws_doubles(h->mh[b].d, h->mh[b].pcap, sk_nm[b], h->mh[b].K,
                                  o->sketch_rank);
    }
    ALLOC(h->sk, sizeof(double) * sk_tot);
    ALLOC(h->sk_off_d, sizeof(int64_t) * batch);
    ALLOC(h->sk_nm_d, sizeof(int) * batch);
  }
  h->a_elems = a_tot;
#undef ALLOC
  hipStream_t s = h->stream;
  auto fail_dev = [&](hipError_t e, const char* what) {
    const tnrsvd_status r = dev_check(e, what);
    release(h);
    delete h;
    return r;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(h->mpos_d, h->mh.data(), sizeof(MpoDesc) * batch,
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_dev(e, "upload MPO descriptors");
  if (o->sketch_rank > 0) {
    if ((e = hipMemcpyAsync(h->sk_off_d, sk_off.data(), sizeof(int64_t) * batch,
                            hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h->sk_nm_d, sk_nm.data(), sizeof(int) * batch,
                            hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail_dev(e, "upload sketch plan");
  }
  if ((e = hipMemcpyAsync(h->cores_d, h->ch.data(), sizeof(CoreDesc) * h->ncores,
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_dev(e, "upload core descriptors");
  if ((e = hipMemcpyAsync(h->core_mpo_d, h->core_mpo.data(), sizeof(int) * h->ncores,
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_dev(e, "upload core map");
  {
    std::vector<double> cost(batch, 0.0);
    for (int b = 0; b < batch; ++b)
      for (int i = 0; i < h->mh[b].d; ++i) {
        const CoreDesc& cd = h->ch[h->mh[b].c0 + i];
        const double P = (double)cd.RA * cd.xcap;
        cost[b] += (double)std::max(cd.I, cd.J) * P * P;
      }
    h->order.resize(batch);
    for (int b = 0; b < batch; ++b) h->order[b] = b;
    std::stable_sort(h->order.begin(), h->order.end(),
                     [&](int a, int c) { return cost[a] > cost[c]; });
    if ((e = hipMemcpyAsync(h->order_d, h->order.data(), sizeof(int) * batch,
                            hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail_dev(e, "upload MPO order");
  }
  if (h->wide_possible &&
      (e = hipMemcpyAsync(h->wcap_d, h->wcap.data(), sizeof(int) * h->wcap.size(),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_dev(e, "upload wide plan");
  if ((e = hipMemsetAsync(h->err, 0, sizeof(int) * 4, s)) != hipSuccess)
    return fail_dev(e, "clear error flags");

  // ---- stage A: copy/convert leading cores, merge the trailing ones (FP64) --
  int64_t tmp_need = 1;
  for (int b = 0; b < batch; ++b) {
    const tnrsvd_mpo& a = mpos[b];
    const int m = merge[b];
    if (m > 1) {
      int64_t acc = a.rank[a.d - m];
      int64_t in = 1, jn = 1;
      for (int i = a.d - m; i < a.d; ++i) {
        in *= a.rows[i];
        jn *= a.cols[i];
        tmp_need = std::max(tmp_need, a.rank[i] * a.rows[i] * a.cols[i] * a.rank[i + 1]);
        tmp_need = std::max(tmp_need, acc * in * jn * a.rank[i + 1]);
      }
    }
  }
  double *t0 = nullptr, *t1 = nullptr, *t2 = nullptr;
  if ((e = hipMalloc(&t0, sizeof(double) * tmp_need)) != hipSuccess ||
      (e = hipMalloc(&t1, sizeof(double) * tmp_need)) != hipSuccess ||
      (e = hipMalloc(&t2, sizeof(double) * tmp_need)) != hipSuccess) {
    (void)hipGetLastError();
    if (t0) (void)hipFree(t0);
    if (t1) (void)hipFree(t1);
    release(h);
    delete h;
    return fail(TNRSVD_E_NOMEM, "merge staging allocation failed");
  }
  int* fin = h->err + 2;
  for (int b = 0; b < batch && e == hipSuccess; ++b) {
    const tnrsvd_mpo& a = mpos[b];
    const MpoDesc& md = h->mh[b];
    const int m = merge[b];
    const int dm = md.d;
    // BF16 handles stage A in FP32 (kept for tnrsvd_refine) and narrow it below
    const int sdt = h->dtype == kBF16 ? kF32 : h->dtype;
    const size_t sesz = elem_size(sdt);
    char* Abase = (char*)(h->dtype == kBF16 ? h->A32 : h->A);
    if (o->check_finite) {
      for (int i = 0; i < a.d && e == hipSuccess; ++i)
        e = launch_check_finite(a.core[i], a.dtype,
                                a.rank[i] * a.rows[i] * a.cols[i] * a.rank[i + 1], fin, s);
    }
    for (int i = 0; i < dm - 1 && e == hipSuccess; ++i) {
      const CoreDesc& cd = h->ch[md.c0 + i];
      e = launch_convert_core(a.core[i], a.dtype, Abase + sesz * cd.a_off, sdt,
                              a.rank[i] * a.rows[i] * a.cols[i] * a.rank[i + 1], s);
    }
    const CoreDesc& cl = h->ch[md.c0 + dm - 1];
    const int f = a.d - m;
    if (m == 1) {
      if (e == hipSuccess)
        e = launch_convert_core(a.core[f], a.dtype, Abase + sesz * cl.a_off, sdt,
                                a.rank[f] * a.rows[f] * a.cols[f] * a.rank[f + 1], s);
    } else {
      for (int j = f; j < a.d && e == hipSuccess; ++j)
        e = launch_convert_core(a.core[j], a.dtype, h->tail + h->tail_off[b][j - f], kF64,
                                a.rank[j] * a.rows[j] * a.cols[j] * a.rank[j + 1], s);
      // T <- core f (FP64); repeatedly T <- merge(T, core j)
      int64_t ra = a.rank[f], ti = a.rows[f], tj = a.cols[f], tb = a.rank[f + 1];
      if (e == hipSuccess) e = launch_convert_core(a.core[f], a.dtype, t0, 0, ra * ti * tj * tb, s);
      double* cur = t0;
      double* nxt = t1;
      for (int j = f + 1; j < a.d && e == hipSuccess; ++j) {
        e = launch_convert_core(a.core[j], a.dtype, t2, 0,
                                a.rank[j] * a.rows[j] * a.cols[j] * a.rank[j + 1], s);
        if (e != hipSuccess) break;
        e = launch_merge_pair(cur, t2, nxt, (int)ra, (int)ti, (int)tj, (int)tb, (int)a.rows[j],
                              (int)a.cols[j], (int)a.rank[j + 1], s);
        ti *= a.rows[j];
        tj *= a.cols[j];
        tb = a.rank[j + 1];
        std::swap(cur, nxt);
      }
      if (e == hipSuccess)
        e = launch_convert_core(cur, 0, Abase + sesz * cl.a_off, sdt, ra * ti * tj * tb, s);
    }
  }
  if (e == hipSuccess && h->dtype == kBF16)
    e = launch_convert_core(h->A32, kF32, h->A, kBF16, a_tot, s);
  if (e == hipSuccess) e = launch_omega(h->mpos_d, h->cores_d, batch, o->seed, h->om, h->max_om, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(t0);
  (void)hipFree(t1);
  (void)hipFree(t2);
  if (e != hipSuccess) return fail_dev(e, "staging the MPO cores");
  if (o->check_finite) {
    int flag = 0;
    if ((e = hipMemcpy(&flag, fin, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
      return fail_dev(e, "read finite flag");
    if (flag) {
      release(h);
      delete h;
      return fail(TNRSVD_E_NONFINITE, "an input core holds NaN or Inf");
    }
  }
  *out = h;
  return TNRSVD_OK;
}

// TNRSVD_K_FIRST: stage every MPO reversed (core order reversed, rank legs
// swapped) and plan it as usual; results are reversed back on the way out.
tnrsvd_status tnrsvd_create(tnrsvd_t* out, int batch, const tnrsvd_mpo* mpos,
                            const tnrsvd_opts* o) {
  g_err.clear();
  if (!out || !mpos || !o) return fail(TNRSVD_E_INVALID, "null argument");
  TRY(check_opts(o));   // before any staging
  if (o->orientation == TNRSVD_K_LAST) return create_lib(out, batch, mpos, o);
  *out = nullptr;
  if (batch < 1) return fail(TNRSVD_E_INVALID, "batch must be >= 1");
  const hipStream_t s = (hipStream_t)o->stream;
  std::vector<void*> temps;
  std::vector<std::vector<int64_t>> rk(batch), rw(batch), cl(batch);
  std::vector<std::vector<const void*>> cp(batch);
  std::vector<tnrsvd_mpo> rev(batch);
  std::vector<std::vector<std::array<int64_t, 4>>> shapes(batch);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : temps) (void)hipFree(p);
  };
  for (int b = 0; b < batch; ++b) {
    const tnrsvd_mpo& a = mpos[b];
    if (a.d < 1) return cleanup(), fail(TNRSVD_E_SHAPE, "d must be >= 1");
    if (!a.rank || !a.rows || !a.cols || !a.core)
      return cleanup(), fail(TNRSVD_E_INVALID, "null rank/rows/cols/core array");
    if (a.dtype != TNRSVD_F64 && a.dtype != TNRSVD_F32)
      return cleanup(), fail(TNRSVD_E_INVALID, "core dtype must be F64 or F32");
    const int d = a.d;
    if (a.rank[0] != 1 || a.rank[d] != 1)
      return cleanup(), fail(TNRSVD_E_SHAPE, "MPO %d: rank[0] and rank[d] must be 1", b);
    const int dt = a.dtype == TNRSVD_F64 ? kF64 : kF32;
    rk[b].resize(d + 1);
    rw[b].resize(d);
    cl[b].resize(d);
    cp[b].resize(d);
    for (int i = 0; i <= d; ++i) rk[b][i] = a.rank[d - i];
    for (int i = 0; i < d; ++i) {
      const int src = d - 1 - i;
      const int64_t R0 = a.rank[src], I = a.rows[src], J = a.cols[src], R1 = a.rank[src + 1];
      if (R0 < 1 || I < 1 || J < 1 || R1 < 1 || !a.core[src])
        return cleanup(), fail(TNRSVD_E_SHAPE, "MPO %d core %d: bad shape or null core", b, src);
      rw[b][i] = I;
      cl[b][i] = J;
      void* t = nullptr;
      if (hipMalloc(&t, (size_t)(R0 * I * J * R1) * (dt == kF64 ? 8 : 4)) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(), fail(TNRSVD_E_NOMEM, "staging the reversed cores");
      }
      temps.push_back(t);
      const hipError_t e = launch_swap_legs(a.core[src], dt, t, R0, I, J, R1, s);
      if (e != hipSuccess) return cleanup(), dev_check(e, "reverse core");
      cp[b][i] = t;
    }
    for (int i = 0; i < d; ++i)
      shapes[b].push_back({a.rank[i], a.rows[i], a.cols[i], a.rank[i + 1]});
    rev[b] = tnrsvd_mpo{d, rk[b].data(), rw[b].data(), cl[b].data(), cp[b].data(), a.dtype};
  }
  tnrsvd_opts lib = *o;
  lib.orientation = TNRSVD_K_LAST;
  const tnrsvd_status st = create_lib(out, batch, rev.data(), &lib);
  cleanup();
  if (st != TNRSVD_OK) return st;
  (*out)->orientation = TNRSVD_K_FIRST;
  (*out)->paper_shape = shapes;
  return TNRSVD_OK;
}

}  // extern "C"

namespace {

hipEvent_t next_event(tnrsvd_t h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Bracket one launch with events when profiling is enabled.
struct Timed {
  tnrsvd_t h;
  int kind;
  hipEvent_t a = nullptr;
  Timed(tnrsvd_t hh, int k) : h(hh), kind(k) {
    if (h->profiling) {
      a = next_event(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~Timed() {
    if (h->profiling && a) {
      hipEvent_t b = next_event(h);
      if (b) {
        (void)hipEventRecord(b, h->stream);
        h->ev_pairs[kind].push_back({a, b});
      }
    }
  }
};

tnrsvd_status check_handle(tnrsvd_t h) {
  g_err.clear();
  if (!h) return fail(TNRSVD_E_INVALID, "null handle");
  return TNRSVD_OK;
}

void restore_precision(tnrsvd_t h) {
  if (!h->refined) return;
  std::swap(h->A, h->A32);
  std::swap(h->X, h->X32);
  std::swap(h->Z, h->Z32);
  h->dtype = kBF16;
  h->refined = false;
}

tnrsvd_status load_omega(tnrsvd_t h) {
  restore_precision(h);
  Timed tm(h, 4);
  hipError_t e = launch_load_omega(h->mpos_d, h->cores_d, h->batch, h->om, h->xr, h->X, h->dtype,
                                   h->max_d, h->max_om, h->err, h->stream);
  TRY(dev_check(e, "load Omega"));
  h->space = kCol;
  h->first_product = true;
  h->projected = false;
  h->solved = false;
  h->round_idx = 0;
  h->hist_op.clear();
  h->hist_svd.clear();
  return TNRSVD_OK;
}

tnrsvd_status do_mult(tnrsvd_t h, int op) {
  hipError_t e;
  if (h->first_product) h->prod_t = 0;
  {
    Timed tm(h, 0);
    e = launch_contract(h->mpos_d, h->cores_d, h->core_mpo_d, h->ncores, h->xr, h->pr,
                                 h->A, h->X, h->Z, h->dtype, op, h->max_core_out, h->err,
                                 h->ct_threads[op], h->ct_cap[op], h->stream);
  }
  TRY(dev_check(e, "contract"));
  if (op == 0 && h->first_product) {
    Timed tm(h, 5);
    e = launch_copy_y0(h->mpos_d, h->cores_d, h->core_mpo_d, h->ncores, h->pr, h->Z, h->Y0,
                       h->dtype, h->max_core_out, h->stream);
    TRY(dev_check(e, "copy Y0"));
    h->y0_valid = true;
  }
  h->first_product = false;
  if (h->opts.sketch_rank > 0) {
    // stream index t of this product: counters from (t + 1) 2^40 on, past Omega's
    Timed tm(h, 6);
    e = launch_sketch(h->mpos_d, h->cores_d, h->batch, op, h->pr, h->Z, h->dtype,
                      h->opts.sketch_rank, h->opts.seed, (uint64_t)(h->prod_t + 1) << 40,
                      h->sk_nm_d, h->sk_off_d, h->sk, h->err, h->stream);
    TRY(dev_check(e, "sketch the product"));
    ++h->prod_t;
  }
  return TNRSVD_OK;
}

// Right-to-left pass.  When the capacities allow panels beyond the register
// path, k_wide_classify first picks the MPOs whose panels are that wide (from
// the ranks on the device); they take the multi-workgroup launches, the rest
// the one-workgroup kernels.  Run eagerly, the launches follow the device's
// needs (read back once per rounding) and that plan is kept for the rounding's
// index within the solve; under stream capture the kept plan (or, before any
// eager solve, the capacity plan) is used, and MPOs it does not cover stay on
// the one-workgroup path.
tnrsvd_status rl_sweep(tnrsvd_t h, int op) {
  hipError_t e;
  const int* wflag = nullptr;
  const int* plan = nullptr;
  if (h->wide_possible) {
    const int idx = h->round_idx++;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TRY(dev_check(hipStreamIsCapturing(h->stream, &cs), "query capture"));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    const int nplan = kWidePlan * h->max_d;
    const int* plan_d = nullptr;
    if (capturing) {
      if (idx < h->wslots && (int)h->wplan[idx].size() == nplan) {
        plan = h->wplan[idx].data();
        plan_d = h->wplan_d + (int64_t)idx * nplan;
      } else {
        plan = h->wcap.data();
        plan_d = h->wcap_d;
      }
    }
    e = launch_wide_classify(h->mpos_d, h->cores_d, h->batch, op, h->pr, plan_d, h->max_d,
                             h->wide_min_p, h->wflag_d, h->wneed_d, h->stream);
    TRY(dev_check(e, "classify panels"));
    if (!capturing) {
      std::vector<int> need(nplan);
      TRY(dev_check(hipMemcpyAsync(need.data(), h->wneed_d, sizeof(int) * nplan,
                                   hipMemcpyDeviceToHost, h->stream),
                    "read panel sizes"));
      TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
      if (idx < h->wslots) {
        h->wplan[idx] = need;
        TRY(dev_check(hipMemcpyAsync(h->wplan_d + (int64_t)idx * nplan, h->wplan[idx].data(),
                                     sizeof(int) * nplan, hipMemcpyHostToDevice, h->stream),
                      "keep panel plan"));
        plan = h->wplan[idx].data();
      } else {
        h->wscratch = need;
        plan = h->wscratch.data();
      }
    }
    wflag = h->wflag_d;
  }
  {
    Timed tm(h, 1);
    e = launch_rl_pass(h->mpos_d, h->cores_d, h->batch, op, h->pr, h->rho, h->ldm, h->Z, h->dtype,
                       h->W, h->L, h->tau, h->err, h->leaf_nc, wflag,
                       h->lpt ? h->order_d : nullptr, h->stream);
    TRY(dev_check(e, "right-to-left sweep"));
    if (plan) {
      for (int t = 0; t < h->max_d; ++t) {
        e = launch_rl_wide_step(h->mpos_d, h->cores_d, h->batch, op, h->pr, h->rho, h->ldm,
                                h->wflag_d, h->Z, h->dtype, h->W, h->WV, h->L, h->tau, t,
                                plan + kWidePlan * t, h->stream);
        TRY(dev_check(e, "right-to-left sweep (wide panels)"));
      }
    }
  }
  return TNRSVD_OK;
}

tnrsvd_status do_sweep(tnrsvd_t h, int op, int mode) {
  hipError_t e;
  TRY(rl_sweep(h, op));
  Timed tm(h, 2);
  SweepOpts so;
  so.eps = h->opts.round_tol;
  so.rmax = (int)h->opts.max_rank;
  so.mode = mode;
  so.qcap = h->qcap;
  void* out = mode == 0 ? h->X : (void*)h->V;
  const int odt = mode == 0 ? h->dtype : kF64;
  int* rout = mode == 0 ? h->xr : h->vr;
  e = launch_lr_pass(h->mpos_d, h->cores_d, h->batch, op, h->rho, h->ldm, rout, h->W, h->tau,
                     h->scratch, out, odt, h->outs, so, h->tcap, h->mcap_s, h->ucap, h->err,
                     h->wide_possible ? h->wflag_d : nullptr, h->lpt ? h->order_d : nullptr,
                     h->stream);
  TRY(dev_check(e, "left-to-right sweep"));
  // the ranks this rounding kept, for tnrsvd_backward
  const int slot = (int)h->hist_op.size();
  if (slot < h->hist_slots) {
    e = hipMemcpyAsync(h->rhist_d + (int64_t)slot * h->r_tot, rout, sizeof(int) * h->r_tot,
                       hipMemcpyDeviceToDevice, h->stream);
    TRY(dev_check(e, "record ranks"));
  }
  h->hist_op.push_back(op);
  h->hist_svd.push_back(mode);
  return TNRSVD_OK;
}

tnrsvd_status read_sigma(tnrsvd_t h, double* sigma) {
  const int k = h->opts.k;
  std::vector<double> tmp;
  for (int b = 0; b < h->batch; ++b) {
    hipError_t e = hipMemcpyAsync(sigma + (int64_t)b * k, h->outs + h->mh[b].out_off,
                                  sizeof(double) * k, hipMemcpyDeviceToHost, h->stream);
    TRY(dev_check(e, "copy sigma"));
  }
  int flags[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(flags, h->err, sizeof(flags), hipMemcpyDeviceToHost, h->stream);
  TRY(dev_check(e, "copy error flags"));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  if (flags[0] & 2) return fail(TNRSVD_E_SHAPE, "a bond rank exceeded its planned capacity");
  if (flags[0] & 4) return fail(TNRSVD_E_SHAPE, "a kernel met shapes beyond its planned capacity");
  return TNRSVD_OK;
}

}  // namespace

extern "C" {

tnrsvd_status tnrsvd_mult(tnrsvd_t h, int op) {
  TRY(check_handle(h));
  if (op != 0 && op != 1) return fail(TNRSVD_E_INVALID, "op must be 0 (A X) or 1 (A^T X)");
  if (h->pending >= 0 || h->projected)
    return fail(TNRSVD_E_STATE, "a product is pending; call tnrsvd_orthogonalize or tnrsvd_solve");
  if (h->space == kNone || h->solved) {
    if (op != 0) return fail(TNRSVD_E_STATE, "the first product must be Y = A Omega (op 0)");
    TRY(load_omega(h));
  }
  if (op == 0 && h->space != kCol)
    return fail(TNRSVD_E_STATE, "Y = A X needs a column-space basis (Omega or an A^T Q result)");
  if (op == 1 && h->space != kRow)
    return fail(TNRSVD_E_STATE, "Z = A^T Q needs a row-space basis");
  TRY(do_mult(h, op));
  h->pending = op;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_orthogonalize(tnrsvd_t h) {
  TRY(check_handle(h));
  if (h->pending < 0) return fail(TNRSVD_E_STATE, "no pending product to orthogonalize");
  TRY(do_sweep(h, h->pending, 0));
  h->space = h->pending == 0 ? kRow : kCol;
  h->pending = -1;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_project(tnrsvd_t h) {
  TRY(check_handle(h));
  if (h->pending >= 0) return fail(TNRSVD_E_STATE, "a product is pending");
  if (h->space != kRow || h->solved)
    return fail(TNRSVD_E_STATE, "projection needs the row-space basis Q of an orthogonalized A X");
  TRY(do_mult(h, 1));
  h->projected = true;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_solve(tnrsvd_t h, double* sigma) {
  TRY(check_handle(h));
  if (!h->projected) return fail(TNRSVD_E_STATE, "tnrsvd_project has not run");
  TRY(do_sweep(h, 1, 1));
  hipError_t e;
  {
    Timed tm(h, 3);
    e = launch_form_u(h->mpos_d, h->cores_d, h->core_mpo_d, h->ncores, h->xr, h->X,
                               h->dtype, h->outs, h->U, h->max_core_out, h->err, h->stream);
  }
  TRY(dev_check(e, "form U"));
  h->projected = false;
  h->solved = true;
  if (sigma) TRY(read_sigma(h, sigma));
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_run(tnrsvd_t h, double* sigma) {
  TRY(check_handle(h));
  h->pending = -1;
  h->projected = false;
  h->solved = false;
  h->space = kNone;
  TRY(tnrsvd_mult(h, 0));
  TRY(tnrsvd_orthogonalize(h));
  for (int t = 0; t < h->opts.q; ++t) {
    TRY(tnrsvd_mult(h, 1));
    TRY(tnrsvd_orthogonalize(h));
    TRY(tnrsvd_mult(h, 0));
    TRY(tnrsvd_orthogonalize(h));
  }
  TRY(tnrsvd_project(h));
  return tnrsvd_solve(h, sigma);
}

tnrsvd_status tnrsvd_run_graph(tnrsvd_t h, double* sigma) {
  TRY(check_handle(h));
  if (h->profiling)
    return fail(TNRSVD_E_STATE, "profiling events cannot be captured; disable profiling first");
  if (!h->gexec) {
    if (!h->gstream) {
      TRY(dev_check(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking),
                    "create capture stream"));
      for (hipEvent_t& e : h->gev)
        TRY(dev_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "create event"));
    }
    // the multi-workgroup launches of a captured solve follow the plan of an
    // eager solve: run one first if none has been kept
    if (h->wide_possible) {
      bool kept = true;
      for (int r = 0; r < 2 * h->opts.q + 2; ++r)
        kept = kept && (int)h->wplan[r].size() == kWidePlan * h->max_d;
      if (!kept) TRY(tnrsvd_run(h, nullptr));
    }
    // work already queued on the caller's stream (create, set_omega) must not
    // be reordered behind the capture
    TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
    hipStream_t user = h->stream;
    h->stream = h->gstream;
    hipError_t e = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal);
    tnrsvd_status st = e == hipSuccess ? tnrsvd_run(h, nullptr) : dev_check(e, "begin capture");
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->gstream, &g);
    h->stream = user;
    if (st == TNRSVD_OK) st = dev_check(e2, "end capture");
    if (st == TNRSVD_OK)
      st = dev_check(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0), "instantiate graph");
    if (st != TNRSVD_OK) {
      if (g) (void)hipGraphDestroy(g);
      h->gexec = nullptr;
      return st;
    }
    h->graph = g;
  }
  restore_precision(h);
  // caller's stream -> replay on the capture stream -> caller's stream
  TRY(dev_check(hipEventRecord(h->gev[0], h->stream), "record event"));
  TRY(dev_check(hipStreamWaitEvent(h->gstream, h->gev[0], 0), "wait event"));
  TRY(dev_check(hipGraphLaunch(h->gexec, h->gstream), "launch graph"));
  TRY(dev_check(hipEventRecord(h->gev[1], h->gstream), "record event"));
  TRY(dev_check(hipStreamWaitEvent(h->stream, h->gev[1], 0), "wait event"));
  h->pending = -1;
  h->projected = false;
  h->solved = true;
  h->space = kRow;
  h->first_product = false;
  h->y0_valid = true;
  if (sigma) TRY(read_sigma(h, sigma));
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_refine(tnrsvd_t h, double round_tol, double* sigma) {
  TRY(check_handle(h));
  if (!(round_tol >= 0.0) || !std::isfinite(round_tol))
    return fail(TNRSVD_E_INVALID, "round_tol must be finite and >= 0");
  if (h->dtype != kBF16 || h->refined)
    return fail(TNRSVD_E_STATE, "refinement follows a BF16 solve on a BF16 handle");
  if (!h->solved) return fail(TNRSVD_E_STATE, "no BF16 solve to refine");
  // the basis Q of the BF16 solve, widened to FP32, becomes the starting basis
  TRY(dev_check(launch_convert_core(h->X, kBF16, h->X32, kF32, h->x_elems, h->stream),
                "widen the basis"));
  std::swap(h->A, h->A32);
  std::swap(h->X, h->X32);
  std::swap(h->Z, h->Z32);
  h->dtype = kF32;
  h->refined = true;
  h->space = kRow;
  h->pending = -1;
  h->projected = false;
  h->solved = false;
  h->first_product = false;
  const double tol = h->opts.round_tol;
  h->opts.round_tol = round_tol;
  tnrsvd_status st = tnrsvd_mult(h, 1);
  if (st == TNRSVD_OK) st = tnrsvd_orthogonalize(h);
  if (st == TNRSVD_OK) st = tnrsvd_mult(h, 0);
  if (st == TNRSVD_OK) st = tnrsvd_orthogonalize(h);
  if (st == TNRSVD_OK) st = tnrsvd_project(h);
  if (st == TNRSVD_OK) st = tnrsvd_solve(h, sigma);
  h->opts.round_tol = tol;
  return st;
}

}  // extern "C"

namespace {

// Workspace of the backward pass, planned from the rank capacities at its first
// call: per MPO the left environments E_0 .. E_{d'-1} and five temporaries;
// the merged-core gradient slab; the weights; the merge-adjoint chain.
tnrsvd_status plan_grad(tnrsvd_t h) {
  if (h->grad_ready) return TNRSVD_OK;
  std::vector<GradMpo> gm(h->batch);
  std::vector<int64_t> eoff(h->ncores);
  int64_t tot = 0;
  h->chain_cap = 1;
  for (int b = 0; b < h->batch; ++b) {
    const MpoDesc& md = h->mh[b];
    int64_t tmp = 1;
    for (int i = 0; i < md.d; ++i) {
      const CoreDesc& cd = h->ch[md.c0 + i];
      const int64_t l = cd.xcap, r = cd.xcap2, n = std::max(cd.I, cd.J);
      eoff[md.c0 + i] = tot;
      tot += l * cd.RA * l;
      tmp = std::max({tmp, (int64_t)cd.RA * n * l * r, (int64_t)cd.RA2 * n * l * r,
                      l * cd.RA * l, r * cd.RA2 * r});
    }
    gm[b].tmp0 = tot;
    gm[b].tmpcap = tmp;
    tot += 5 * tmp;
    if (h->mcount[b] >= 2) {
      // chain T_1 .. T_{m-2}, two ping-pong gradients and one core gradient
      const auto& sh = h->tail_shape[b];
      int64_t chain = 0, big = 0, cmax = 0, I1 = sh[0][1], J1 = sh[0][2];
      big = (int64_t)sh[0][0] * I1 * J1 * sh[0][3];
      for (size_t j = 1; j < sh.size(); ++j) {
        I1 *= sh[j][1];
        J1 *= sh[j][2];
        const int64_t tj = (int64_t)sh[0][0] * I1 * J1 * sh[j][3];
        if (j + 1 < sh.size()) chain += tj;
        big = std::max(big, tj);
      }
      for (const auto& c : sh) cmax = std::max<int64_t>(cmax, (int64_t)c[0] * c[1] * c[2] * c[3]);
      h->chain_cap = std::max(h->chain_cap, chain + 2 * big + cmax);
    }
  }
  tnrsvd_status st = TNRSVD_OK;
  if ((st = dalloc(h, &h->gm_d, sizeof(GradMpo) * h->batch)) != TNRSVD_OK) return st;
  if ((st = dalloc(h, &h->eoff_d, sizeof(int64_t) * h->ncores)) != TNRSVD_OK) return st;
  if ((st = dalloc(h, &h->gws, sizeof(double) * tot)) != TNRSVD_OK) return st;
  if ((st = dalloc(h, &h->gG, sizeof(double) * h->a_elems)) != TNRSVD_OK) return st;
  if ((st = dalloc(h, &h->gw, sizeof(double) * h->batch * h->opts.k)) != TNRSVD_OK) return st;
  if ((st = dalloc(h, &h->gchain, sizeof(double) * h->chain_cap)) != TNRSVD_OK) return st;
  TRY(dev_check(hipMemcpyAsync(h->gm_d, gm.data(), sizeof(GradMpo) * h->batch,
                               hipMemcpyHostToDevice, h->stream), "copy gradient plan"));
  TRY(dev_check(hipMemcpyAsync(h->eoff_d, eoff.data(), sizeof(int64_t) * h->ncores,
                               hipMemcpyHostToDevice, h->stream), "copy gradient plan"));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  h->grad_ready = true;
  return TNRSVD_OK;
}

}  // namespace

extern "C" {

// After a change of launch choices: drop any captured graph (it holds the
// old launches) and the solve state, so the next call starts afresh.
static void forget_solve(tnrsvd_t h) {
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  h->space = kNone;
  h->pending = -1;
  h->projected = false;
  h->solved = false;
  h->y0_valid = false;
}

tnrsvd_status tnrsvd_autotune(tnrsvd_t h, int reps, int* choice) {
  TRY(check_handle(h));
  if (reps < 1) return fail(TNRSVD_E_INVALID, "reps must be >= 1");
  if (h->profiling) return fail(TNRSVD_E_STATE, "disable profiling before autotuning");
  // one solve leaves a basis of the planned ranks in X; both products are then
  // timed on it (for op 0 with I != J the values are meaningless but every
  // access stays inside the slabs, and the products are recomputed by the next
  // solve, which the state reset below requires)
  TRY(tnrsvd_run(h, nullptr));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TRY(dev_check(hipEventCreate(&e0), "create event"));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TNRSVD_E_DEVICE, "create event");
  }
  const int th[4] = {64, 128, 256, 512};
  const int cp[4] = {64, 256, 1024, 4096};
  tnrsvd_status st = TNRSVD_OK;
  for (int op = 0; op < 2 && st == TNRSVD_OK; ++op) {
    float best = 1e30f;
    int bt = h->ct_threads[op], bc = h->ct_cap[op];
    for (int a = 0; a < 4 && st == TNRSVD_OK; ++a)
      for (int c = 0; c < 4 && st == TNRSVD_OK; ++c) {
        auto go = [&]() {
          return launch_contract(h->mpos_d, h->cores_d, h->core_mpo_d, h->ncores, h->xr, h->pr,
                                 h->A, h->X, h->Z, h->dtype, op, h->max_core_out, h->err, th[a],
                                 cp[c], h->stream);
        };
        hipError_t e = go();   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = go();
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = dev_check(e, "autotune contraction");
          break;
        }
        if (ms < best) {
          best = ms;
          bt = th[a];
          bc = cp[c];
        }
      }
    h->ct_threads[op] = bt;
    h->ct_cap[op] = bc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TRY(st);
  if (choice) {
    choice[0] = h->ct_threads[0];
    choice[1] = h->ct_cap[0];
    choice[2] = h->ct_threads[1];
    choice[3] = h->ct_cap[1];
  }
  forget_solve(h);
  return TNRSVD_OK;
}

// Sweep launch choices, each a pair {wmin, lpt}: wmin = the fewest product
// columns that send an MPO to the wide (multi-workgroup) right-to-left
// launches, 0 for never; lpt = 1 to dispatch the one-workgroup sweeps
// costliest MPO first.
static void apply_sweep_config(tnrsvd_t h, const int* c) {
  h->wide_min_p = c[0] <= 0 ? INT_MAX : std::max(c[0], kRegCols + 1);
  h->lpt = c[1] != 0;
  // the kept panel plans and any captured graph follow the old choice
  for (auto& p : h->wplan) p.clear();
}

tnrsvd_status tnrsvd_set_sweep_config(tnrsvd_t h, const int* choice) {
  TRY(check_handle(h));
  if (!choice) return fail(TNRSVD_E_INVALID, "null sweep configuration");
  if (choice[0] < 0 || (choice[0] > 0 && choice[0] <= kRegCols) || (choice[1] != 0 && choice[1] != 1))
    return fail(TNRSVD_E_INVALID, "sweep configuration {%d, %d}: wmin must be 0 or > %d, lpt 0 or 1",
                choice[0], choice[1], kRegCols);
  apply_sweep_config(h, choice);
  forget_solve(h);
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_autotune_sweeps(tnrsvd_t h, int reps, int* choice) {
  TRY(check_handle(h));
  if (reps < 1) return fail(TNRSVD_E_INVALID, "reps must be >= 1");
  if (h->profiling) return fail(TNRSVD_E_STATE, "disable profiling before autotuning");
  // product-rank capacity over all cores: the one-workgroup path is offered
  // panels up to 4 kRegCols columns only (beyond that it is known to be far
  // slower, and one timed solve there can take minutes)
  int64_t pcap = 0;
  for (const CoreDesc& cd : h->ch) pcap = std::max<int64_t>(pcap, (int64_t)cd.RA * cd.xcap);
  std::vector<std::array<int, 2>> cand;
  const int wm[4] = {kRegCols + 1, 2 * kRegCols + 1, 4 * kRegCols + 1, 0};
  const int lim[4] = {INT_MAX, INT_MAX, 4 * kRegCols, 4 * kRegCols};
  for (int a = 0; a < (h->wide_possible ? 4 : 1); ++a) {
    if (h->wide_possible && pcap > lim[a]) continue;
    for (int l = 1; l >= 0; --l) {
      if (h->batch == 1 && l == 0) continue;   // one MPO: the order does not matter
      cand.push_back({h->wide_possible ? wm[a] : 0, l});
    }
  }
  const int keep[2] = {h->wide_min_p == INT_MAX ? 0 : h->wide_min_p, h->lpt ? 1 : 0};
  double best = 1e300;
  std::array<int, 2> pick = {keep[0], keep[1]};
  for (const auto& c : cand) {
    apply_sweep_config(h, c.data());
    forget_solve(h);
    TRY(tnrsvd_run(h, nullptr));   // warm-up (and the panel plans of this choice)
    TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps; ++r) TRY(tnrsvd_run(h, nullptr));
    TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (dt < best) {
      best = dt;
      pick = c;
    }
  }
  apply_sweep_config(h, pick.data());
  forget_solve(h);
  if (choice) {
    choice[0] = pick[0];
    choice[1] = pick[1];
  }
  return TNRSVD_OK;
}

// The derivative of the whole solve (tnrsvd_backward) into the merged-core
// gradient slab gG, MPO by MPO: the staged cores widened to FP64, the ranks
// of every rounding read back once, then pipeline_adjoint.
static tnrsvd_status pipeline_grad_lib(tnrsvd_t h, const double* dsigma) {
  const int T = 2 * h->opts.q + 2;
  if (h->refined || (int)h->hist_op.size() != T)
    return fail(TNRSVD_E_STATE,
                "the last solve is not a plain Algorithm 5.4 sequence (tnrsvd_run); "
                "refined solves are not differentiated");
  for (int t = 0; t < T; ++t) {
    const int want_op = (t == 0) ? 0 : (t == T - 1 ? 1 : (t % 2 == 1 ? 1 : 0));
    if (h->hist_op[t] != want_op || h->hist_svd[t] != (t == T - 1 ? 1 : 0))
      return fail(TNRSVD_E_STATE, "the last solve is not a plain Algorithm 5.4 sequence");
  }
  std::vector<int> hist((size_t)T * h->r_tot);
  TRY(dev_check(hipMemcpyAsync(hist.data(), h->rhist_d, sizeof(int) * hist.size(),
                               hipMemcpyDeviceToHost, h->stream), "read ranks"));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  const int k = h->opts.k, K = h->opts.k + h->opts.p;
  for (int b = 0; b < h->batch; ++b) {
    const MpoDesc& md = h->mh[b];
    const int d = md.d;
    std::vector<CoreShape> sh(d);
    std::vector<std::vector<int>> ranks(T, std::vector<int>(d + 1));
    std::vector<int> ops(h->hist_op.begin(), h->hist_op.end());
    int64_t a_len = 0;
    for (int i = 0; i < d; ++i) {
      const CoreDesc& cd = h->ch[md.c0 + i];
      sh[i] = {cd.RA, cd.I, cd.J, cd.RA2};
      a_len = std::max<int64_t>(a_len, (int64_t)cd.RA * cd.I * cd.J * cd.RA2);
    }
    for (int t = 0; t < T; ++t)
      for (int i = 0; i <= d; ++i) ranks[t][i] = hist[(size_t)t * h->r_tot + md.r0 + i];
    // panels the adjoint cannot take: a last core with fewer rows than K
    for (int t = 0; t < T; ++t) {
      const CoreDesc& cl = h->ch[md.c0 + d - 1];
      const int n = ops[t] == 0 ? cl.I : cl.J;
      if ((int64_t)ranks[t][d - 1] * n < K || ranks[t][d] != K)
        return fail(TNRSVD_E_SHAPE, "MPO %d: last panel of rounding %d has fewer rows than K",
                    b, t);
    }
    // FP64 copies of the staged (merged) cores
    DevArena arena;
    std::vector<const double*> A(d);
    std::vector<double*> dA(d);
    const size_t esz = elem_size(h->dtype);
    for (int i = 0; i < d; ++i) {
      const CoreDesc& cd = h->ch[md.c0 + i];
      const int64_t len = (int64_t)cd.RA * cd.I * cd.J * cd.RA2;
      double* a64 = arena.get<double>(len);
      if (arena.e != hipSuccess) {
        (void)hipGetLastError();
        return fail(TNRSVD_E_NOMEM, "gradient workspace");
      }
      TRY(dev_check(launch_convert_core((const char*)h->A + esz * cd.a_off, h->dtype, a64, kF64,
                                        len, h->stream), "widen cores"));
      A[i] = a64;
      dA[i] = h->gG + cd.a_off;
    }
    const hipError_t e = pipeline_adjoint(d, sh.data(), A.data(), dA.data(), h->om + md.om_off,
                                          K, k, dsigma ? dsigma + (size_t)b * k : nullptr, ranks,
                                          ops, h->stream);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return fail(TNRSVD_E_NOMEM, "gradient workspace");
    }
    TRY(dev_check(e, "pipeline adjoint"));
  }
  return TNRSVD_OK;
}

static tnrsvd_status backward_lib(tnrsvd_t h, const double* dsigma, void* const* dcores,
                                  bool pipeline) {
  TRY(check_handle(h));
  if (!dcores) return fail(TNRSVD_E_INVALID, "null gradient pointer array");
  if (!h->solved) return fail(TNRSVD_E_STATE, "no solve to differentiate");
  TRY(plan_grad(h));
  const int k = h->opts.k;
  if (pipeline) {
    TRY(pipeline_grad_lib(h, dsigma));
  } else {
    std::vector<double> w((size_t)h->batch * k, 1.0);
    if (dsigma) std::copy(dsigma, dsigma + w.size(), w.begin());
    TRY(dev_check(hipMemcpyAsync(h->gw, w.data(), sizeof(double) * w.size(),
                                 hipMemcpyHostToDevice, h->stream), "copy weights"));
    TRY(dev_check(launch_grad_env(h->mpos_d, h->cores_d, h->gm_d, h->eoff_d, h->batch, h->xr,
                                  h->vr, h->A, h->dtype, h->U, h->V, h->gw, k, h->gws, h->gG,
                                  h->err, h->stream), "environment gradient"));
  }
  int base = 0;
  for (int b = 0; b < h->batch; ++b) {
    const MpoDesc& md = h->mh[b];
    const int odt = h->in_dtype[b];
    for (int i = 0; i + 1 < md.d; ++i) {
      const CoreDesc& cd = h->ch[md.c0 + i];
      TRY(dev_check(launch_convert_core(h->gG + cd.a_off, kF64, dcores[base + i], odt,
                                        (int64_t)cd.RA * cd.I * cd.J * cd.RA2, h->stream),
                    "write gradient"));
    }
    const CoreDesc& cl = h->ch[md.c0 + md.d - 1];
    const int m = h->mcount[b];
    const int f = h->d_orig[b] - m;   // first merged original core
    if (m < 2) {
      TRY(dev_check(launch_convert_core(h->gG + cl.a_off, kF64, dcores[base + f], odt,
                                        (int64_t)cl.RA * cl.I * cl.J * cl.RA2, h->stream),
                    "write gradient"));
    } else {
      // recompute the merge chain T_0 = P_0, T_j = merge(T_{j-1}, P_j), then run it backwards
      const auto& sh = h->tail_shape[b];
      const auto& off = h->tail_off[b];
      std::vector<const double*> T(m);
      std::vector<int64_t> TI(m), TJ(m);
      T[0] = h->tail + off[0];
      TI[0] = sh[0][1];
      TJ[0] = sh[0][2];
      double* cur = h->gchain;
      for (int j = 1; j < m; ++j) {
        TI[j] = TI[j - 1] * sh[j][1];
        TJ[j] = TJ[j - 1] * sh[j][2];
        if (j + 1 < m) {
          TRY(dev_check(launch_merge_pair(T[j - 1], h->tail + off[j], cur, sh[0][0], (int)TI[j - 1],
                                          (int)TJ[j - 1], sh[j][0], sh[j][1], sh[j][2], sh[j][3],
                                          h->stream), "recompute merge"));
          T[j] = cur;
          cur += (int64_t)sh[0][0] * TI[j] * TJ[j] * sh[j][3];
        }
      }
      int64_t big = 0;
      for (int j = 0; j < m; ++j) big = std::max(big, (int64_t)sh[0][0] * TI[j] * TJ[j] * sh[j][3]);
      double* pp[2] = {cur, cur + big};
      double* dC = cur + 2 * big;
      const double* dT = h->gG + cl.a_off;
      for (int j = m - 1; j >= 1; --j) {
        double* out = pp[j & 1];
        TRY(dev_check(launch_merge_pair_bwd(T[j - 1], h->tail + off[j], dT, out, dC, sh[0][0],
                                            (int)TI[j - 1], (int)TJ[j - 1], sh[j][0], sh[j][1],
                                            sh[j][2], sh[j][3], h->stream), "merge adjoint"));
        TRY(dev_check(launch_convert_core(dC, kF64, dcores[base + f + j], odt,
                                          (int64_t)sh[j][0] * sh[j][1] * sh[j][2] * sh[j][3],
                                          h->stream), "write gradient"));
        dT = out;
      }
      TRY(dev_check(launch_convert_core(dT, kF64, dcores[base + f], odt,
                                        (int64_t)sh[0][0] * sh[0][1] * sh[0][2] * sh[0][3],
                                        h->stream), "write gradient"));
    }
    base += h->d_orig[b];
  }
  int flags[4] = {0, 0, 0, 0};
  TRY(dev_check(hipMemcpyAsync(flags, h->err, sizeof(flags), hipMemcpyDeviceToHost, h->stream),
                "copy error flags"));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  if (flags[0] & 4) return fail(TNRSVD_E_SHAPE, "a kernel met shapes beyond its planned capacity");
  return TNRSVD_OK;
}

// TNRSVD_K_FIRST: gradients are formed in the library's layout in staging
// buffers, then written reversed (core order and rank legs) to the caller's.
static tnrsvd_status backward_any(tnrsvd_t h, const double* dsigma, void* const* dcores,
                                  bool pipeline) {
  TRY(check_handle(h));
  if (h->orientation != TNRSVD_K_FIRST) return backward_lib(h, dsigma, dcores, pipeline);
  if (!dcores) return fail(TNRSVD_E_INVALID, "null gradient pointer array");
  std::vector<void*> tmp;
  auto release = [&]() {
    (void)hipStreamSynchronize(h->stream);
    for (void* p : tmp) (void)hipFree(p);
  };
  for (int b = 0; b < h->batch; ++b) {
    const size_t esz = elem_size(h->in_dtype[b]);
    const auto& ps = h->paper_shape[b];
    for (int i = 0; i < (int)ps.size(); ++i) {
      const auto& c = ps[ps.size() - 1 - i];
      void* t = nullptr;
      if (hipMalloc(&t, (size_t)(c[0] * c[1] * c[2] * c[3]) * esz) != hipSuccess) {
        (void)hipGetLastError();
        return release(), fail(TNRSVD_E_NOMEM, "staging the gradient cores");
      }
      tmp.push_back(t);
    }
  }
  tnrsvd_status st = backward_lib(h, dsigma, tmp.data(), pipeline);
  int base = 0;
  for (int b = 0; b < h->batch && st == TNRSVD_OK; ++b) {
    const auto& ps = h->paper_shape[b];
    const int d = (int)ps.size();
    for (int i = 0; i < d && st == TNRSVD_OK; ++i) {
      const auto& c = ps[d - 1 - i];   // library core i is the caller's core d - 1 - i
      st = dev_check(launch_swap_legs(tmp[base + i], h->in_dtype[b], dcores[base + d - 1 - i],
                                      c[3], c[1], c[2], c[0], h->stream),
                     "reverse gradient");
    }
    base += d;
  }
  if (st == TNRSVD_OK) st = dev_check(hipStreamSynchronize(h->stream), "synchronise");
  release();
  return st;
}

tnrsvd_status tnrsvd_backward(tnrsvd_t h, const double* dsigma, void* const* dcores) {
  return backward_any(h, dsigma, dcores, true);
}

tnrsvd_status tnrsvd_backward_frozen(tnrsvd_t h, const double* dsigma, void* const* dcores) {
  return backward_any(h, dsigma, dcores, false);
}

tnrsvd_status tnrsvd_get_ranks(tnrsvd_t h, int b, int64_t* host_out, int* d_merged) {
  TRY(check_handle(h));
  if (b < 0 || b >= h->batch) return fail(TNRSVD_E_INVALID, "MPO index out of range");
  const MpoDesc& md = h->mh[b];
  if (d_merged) *d_merged = md.d;
  if (!host_out) return TNRSVD_OK;
  std::vector<int> tmp(md.d + 1);
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  TRY(dev_check(hipMemcpy(tmp.data(), h->xr + md.r0, sizeof(int) * (md.d + 1),
                          hipMemcpyDeviceToHost),
                "copy ranks"));
  for (int i = 0; i <= md.d; ++i)
    host_out[i] = tmp[h->orientation == TNRSVD_K_FIRST ? md.d - i : i];
  return TNRSVD_OK;
}

}  // extern "C"

static tnrsvd_status get_factor_lib(tnrsvd_t h, int b, int which, int core, const void** dev_ptr,
                                    int64_t shape[4], int* dtype) {
  TRY(check_handle(h));
  if (b < 0 || b >= h->batch) return fail(TNRSVD_E_INVALID, "MPO index out of range");
  const MpoDesc& md = h->mh[b];
  if (core < 0 || core >= md.d) return fail(TNRSVD_E_INVALID, "core index out of range");
  if (which < 0 || which > 3) return fail(TNRSVD_E_INVALID, "which must be 0..3");
  if ((which == 0 || which == 1) && !h->solved)
    return fail(TNRSVD_E_STATE, "U and V are available after tnrsvd_solve");
  if (which == 2 && h->space == kNone) return fail(TNRSVD_E_STATE, "no basis yet");
  if (which == 3 && !h->y0_valid) return fail(TNRSVD_E_STATE, "no first product yet");
  const CoreDesc& cd = h->ch[md.c0 + core];
  std::vector<int> r(md.d + 1);
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  const int* src = which == 3 ? nullptr : (which == 1 ? h->vr : h->xr);
  if (src)
    TRY(dev_check(hipMemcpy(r.data(), src + md.r0, sizeof(int) * (md.d + 1),
                            hipMemcpyDeviceToHost),
                  "copy ranks"));
  const size_t esz = elem_size(h->dtype);
  int64_t n;
  if (which == 0) {
    n = cd.I;
  } else if (which == 1) {
    n = cd.J;
  } else if (which == 2) {
    n = h->space == kRow ? cd.I : cd.J;
  } else {
    n = cd.I;
  }
  if (which == 3) {
    shape[0] = cd.RA;
    shape[1] = cd.I;
    shape[2] = core == md.d - 1 ? md.K : cd.RA2;
    shape[3] = 1;
    *dev_ptr = (const char*)h->Y0 + elem_size(h->y0_dtype) * cd.y0_off;
    *dtype = h->y0_dtype;
    return TNRSVD_OK;
  }
  shape[0] = r[core];
  shape[1] = n;
  shape[2] = r[core + 1];
  shape[3] = 1;
  if (which == 0) {
    *dev_ptr = h->U + cd.u_off;
    *dtype = TNRSVD_F64;
  } else if (which == 1) {
    *dev_ptr = h->V + cd.u_off;
    *dtype = TNRSVD_F64;
  } else {
    *dev_ptr = (const char*)h->X + esz * cd.x_off;
    *dtype = h->dtype;
  }
  return TNRSVD_OK;
}

// core index of the library's layout for the caller's core `core` of MPO b
static int lib_core(tnrsvd_t h, int b, int core) {
  if (h->orientation != TNRSVD_K_FIRST || b < 0 || b >= h->batch) return core;
  return h->mh[b].d - 1 - core;
}

extern "C" {

tnrsvd_status tnrsvd_get_factor(tnrsvd_t h, int b, int which, int core, const void** dev_ptr,
                                int64_t shape[4], int* dtype) {
  TRY(check_handle(h));
  if (!dev_ptr || !shape || !dtype) return fail(TNRSVD_E_INVALID, "null output pointer");
  TRY(get_factor_lib(h, b, which, lib_core(h, b, core), dev_ptr, shape, dtype));
  if (h->orientation == TNRSVD_K_FIRST) {
    std::swap(shape[0], shape[2]);
    *dev_ptr = nullptr;
  }
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_copy_factor(tnrsvd_t h, int b, int which, int core, void* dst) {
  const void* src = nullptr;
  int64_t shape[4];
  int dt = 0;
  TRY(check_handle(h));
  TRY(get_factor_lib(h, b, which, lib_core(h, b, core), &src, shape, &dt));
  if (!dst) return fail(TNRSVD_E_INVALID, "null destination");
  if (h->orientation == TNRSVD_K_FIRST) {
    // the mode index of the merged core lists the caller's digits in reverse
    const MpoDesc& md = h->mh[b];
    const int lc = lib_core(h, b, core), m = lc == md.d - 1 ? h->mcount[b] : 1;
    const bool cols = which == 1 || (which == 2 && h->space != kRow);
    const auto& ps = h->paper_shape[b];
    Radices rad{};
    for (int j = 0; j < m; ++j) {   // library core d - m + j is the caller's core m - 1 - j
      const int64_t r = m == 1 ? shape[1] : ps[m - 1 - j][cols ? 2 : 1];
      if (r > 1) {
        if (rad.nd == Radices::kMax) return fail(TNRSVD_E_SHAPE, "too many merged digits");
        rad.r[rad.nd++] = r;
      }
    }
    for (int k = rad.nd - 1; k >= 0; --k)
      rad.below[k] = k == rad.nd - 1 ? 1 : rad.below[k + 1] * rad.r[k + 1];
    if ((rad.nd ? rad.below[0] * rad.r[0] : 1) != shape[1])
      return fail(TNRSVD_E_SHAPE, "merged digits do not match the core's mode size");
    TRY(dev_check(launch_reverse_core(src, dt, dst, shape[0], shape[1], shape[2], rad, h->stream),
                  "reverse factor"));
  } else {
    const size_t bytes = (size_t)(shape[0] * shape[1] * shape[2]) * elem_size(dt);
    TRY(dev_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, h->stream),
                  "copy factor"));
  }
  return dev_check(hipStreamSynchronize(h->stream), "synchronise");
}

tnrsvd_status tnrsvd_get_omega(tnrsvd_t h, int b, double* host_out, int64_t* n) {
  TRY(check_handle(h));
  if (b < 0 || b >= h->batch) return fail(TNRSVD_E_INVALID, "MPO index out of range");
  const MpoDesc& md = h->mh[b];
  int64_t cnt = 0;
  for (int i = 0; i < md.d - 1; ++i) cnt += h->ch[md.c0 + i].J;
  cnt += (int64_t)h->ch[md.c0 + md.d - 1].J * md.K;
  if (n) *n = cnt;
  if (!host_out) return TNRSVD_OK;
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  return dev_check(hipMemcpy(host_out, h->om + md.om_off, sizeof(double) * cnt,
                             hipMemcpyDeviceToHost),
                   "copy Omega");
}

tnrsvd_status tnrsvd_set_omega(tnrsvd_t h, int b, const double* host_in) {
  TRY(check_handle(h));
  if (b < 0 || b >= h->batch) return fail(TNRSVD_E_INVALID, "MPO index out of range");
  if (!host_in) return fail(TNRSVD_E_INVALID, "null Omega");
  const MpoDesc& md = h->mh[b];
  int64_t cnt = 0;
  for (int i = 0; i < md.d - 1; ++i) cnt += h->ch[md.c0 + i].J;
  cnt += (int64_t)h->ch[md.c0 + md.d - 1].J * md.K;
  TRY(dev_check(hipMemcpyAsync(h->om + md.om_off, host_in, sizeof(double) * cnt,
                               hipMemcpyHostToDevice, h->stream),
                "copy Omega"));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  h->space = kNone;
  h->pending = -1;
  h->projected = false;
  h->solved = false;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_profile(tnrsvd_t h, int enable) {
  TRY(check_handle(h));
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  for (auto& v : h->ev_pairs) v.clear();
  h->ev_used = 0;
  h->profiling = enable != 0;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_profile_read(tnrsvd_t h, int kernel, double* total_ms, int64_t* launches) {
  TRY(check_handle(h));
  if (kernel < 0 || kernel >= kKinds) return fail(TNRSVD_E_INVALID, "kernel kind out of range");
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  double tot = 0.0;
  for (auto& pr : h->ev_pairs[kernel]) {
    float ms = 0.f;
    TRY(dev_check(hipEventElapsedTime(&ms, pr.first, pr.second), "event time"));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)h->ev_pairs[kernel].size();
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_get_product_ranks(tnrsvd_t h, int b, int64_t* P_out, int64_t* rho_out) {
  TRY(check_handle(h));
  if (b < 0 || b >= h->batch) return fail(TNRSVD_E_INVALID, "MPO index out of range");
  const MpoDesc& md = h->mh[b];
  std::vector<int> tmp(md.d + 1);
  TRY(dev_check(hipStreamSynchronize(h->stream), "synchronise"));
  if (P_out) {
    TRY(dev_check(hipMemcpy(tmp.data(), h->pr + md.r0, sizeof(int) * (md.d + 1),
                            hipMemcpyDeviceToHost),
                  "copy ranks"));
    for (int i = 0; i <= md.d; ++i) P_out[i] = tmp[i];
  }
  if (rho_out) {
    TRY(dev_check(hipMemcpy(tmp.data(), h->rho + md.r0, sizeof(int) * (md.d + 1),
                            hipMemcpyDeviceToHost),
                  "copy ranks"));
    for (int i = 0; i <= md.d; ++i) rho_out[i] = tmp[i];
  }
  return TNRSVD_OK;
}

}  // extern "C"

namespace {

// Checks shared by the sparse entry points; M and Nc receive the matrix size.
tnrsvd_status check_coo(int d, const int64_t* rows, const int64_t* cols, int64_t nnz,
                        const int64_t* coo_row, const int64_t* coo_col, const double* coo_val,
                        int64_t* M_out, int64_t* Nc_out) {
  if (d < 1) return fail(TNRSVD_E_SHAPE, "d must be >= 1");
  if (!rows || !cols) return fail(TNRSVD_E_INVALID, "null rows/cols");
  if (nnz < 0 || nnz > INT32_MAX) return fail(TNRSVD_E_SHAPE, "nnz must be in [0, 2^31)");
  if (nnz > 0 && (!coo_row || !coo_col || !coo_val))
    return fail(TNRSVD_E_INVALID, "null COO array");
  constexpr int64_t kIdxCap = int64_t(1) << 62;
  int64_t M = 1, Nc = 1;
  for (int k = 0; k < d; ++k) {
    if (rows[k] < 1 || cols[k] < 1) return fail(TNRSVD_E_SHAPE, "mode %d size < 1", k);
    if (M > kIdxCap / rows[k] || Nc > kIdxCap / cols[k])
      return fail(TNRSVD_E_SHAPE, "matrix dimensions exceed 2^62");
    M *= rows[k];
    Nc *= cols[k];
  }
  if ((M / rows[0]) > kIdxCap / (Nc / cols[0]))
    return fail(TNRSVD_E_SHAPE, "number of block positions exceeds 2^62");
  *M_out = M;
  *Nc_out = Nc;
  return TNRSVD_OK;
}

}  // namespace

// The rounded MPO of tnrsvd_sparse_round.
struct tnrsvd_rounded_s {
  int d = 0;
  std::vector<int64_t> rows, cols, ranks;
  std::vector<double*> cores;
  hipStream_t stream = nullptr;
};

extern "C" {

tnrsvd_status tnrsvd_sparse_to_mpo(int d, const int64_t* rows, const int64_t* cols, int64_t nnz,
                                   const int64_t* coo_row, const int64_t* coo_col,
                                   const double* coo_val, int64_t* nblocks, double* const* cores,
                                   void* stream) {
  int64_t M = 0, Nc = 0;
  TRY(check_coo(d, rows, cols, nnz, coo_row, coo_col, coo_val, &M, &Nc));
  if (!nblocks) return fail(TNRSVD_E_INVALID, "null nblocks");
  const int64_t expect = cores ? *nblocks : -1;
  if (cores) {
    if (expect < 1) return fail(TNRSVD_E_INVALID, "*nblocks must hold the rank of the cores");
    if (expect > (nnz > 0 ? nnz : 1))
      return fail(TNRSVD_E_SHAPE, "rank %lld exceeds the number of entries", (long long)expect);
    for (int k = 0; k < d; ++k) {
      const int64_t len = sat_mul(sat_mul(k == 0 ? 1 : expect, rows[k]),
                                  sat_mul(cols[k], k == d - 1 ? 1 : expect));
      if (len >= kSat) return fail(TNRSVD_E_SHAPE, "core %d would exceed 2^40 entries", k);
    }
    for (int k = 0; k < d; ++k)
      if (!cores[k]) return fail(TNRSVD_E_INVALID, "null core %d", k);
  }
  int bad = 0;
  int64_t nb = 0;
  TRY(dev_check(sparse_to_mpo(d, rows, cols, nnz, coo_row, coo_col, coo_val, expect, &nb, cores,
                              &bad, (hipStream_t)stream),
                "sparse to MPO"));
  if (bad) return fail(TNRSVD_E_SHAPE, "COO index outside the %lld x %lld matrix", (long long)M,
                       (long long)Nc);
  *nblocks = nb;
  if (cores && nb != expect)
    return fail(TNRSVD_E_SHAPE, "the matrix has %lld nonzero blocks, cores sized for %lld",
                (long long)nb, (long long)expect);
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_sparse_to_mpo_noalloc(int d, const int64_t* rows, const int64_t* cols,
                                           int64_t nnz, const int64_t* coo_row,
                                           const int64_t* coo_col, const double* coo_val,
                                           int64_t* nblocks, double* const* cores, void* stream) {
  int64_t M = 0, Nc = 0;
  TRY(check_coo(d, rows, cols, nnz, coo_row, coo_col, coo_val, &M, &Nc));
  if (!nblocks) return fail(TNRSVD_E_INVALID, "null nblocks");
  if (d > kNoAllocMaxD)
    return fail(TNRSVD_E_SHAPE, "d = %d exceeds the %d cores the no-allocation call takes", d,
                kNoAllocMaxD);
  const int64_t expect = cores ? *nblocks : -1;
  if (cores) {
    if (expect < 1) return fail(TNRSVD_E_INVALID, "*nblocks must hold the rank of the cores");
    if (expect > (nnz > 0 ? nnz : 1))
      return fail(TNRSVD_E_SHAPE, "rank %lld exceeds the number of entries", (long long)expect);
    for (int k = 0; k < d; ++k) {
      const int64_t len = sat_mul(sat_mul(k == 0 ? 1 : expect, rows[k]),
                                  sat_mul(cols[k], k == d - 1 ? 1 : expect));
      if (len >= kSat) return fail(TNRSVD_E_SHAPE, "core %d would exceed 2^40 entries", k);
    }
    for (int k = 0; k < d; ++k)
      if (!cores[k]) return fail(TNRSVD_E_INVALID, "null core %d", k);
  }
  int bad = 0;
  int64_t nb = 0;
  size_t need = 0;
  TRY(dev_check(sparse_to_mpo_noalloc(d, rows, cols, nnz, coo_row, coo_col, coo_val, expect, &nb,
                                      cores, &bad, &need, (hipStream_t)stream),
                "sparse to MPO (no allocation)"));
  if (need > kNoAllocScratchBytes)
    return fail(TNRSVD_E_SHAPE,
                "the input needs %zu bytes of scratch; the no-allocation call has %zu", need,
                kNoAllocScratchBytes);
  if (bad) return fail(TNRSVD_E_SHAPE, "COO index outside the %lld x %lld matrix", (long long)M,
                       (long long)Nc);
  *nblocks = nb;
  if (cores && nb != expect)
    return fail(TNRSVD_E_SHAPE, "the matrix has %lld nonzero blocks, cores sized for %lld",
                (long long)nb, (long long)expect);
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_sparse_round(int d, const int64_t* rows, const int64_t* cols, int64_t nnz,
                                  const int64_t* coo_row, const int64_t* coo_col,
                                  const double* coo_val, double round_tol, int max_rank,
                                  void* stream, tnrsvd_rounded_t* out) {
  if (!out) return fail(TNRSVD_E_INVALID, "null out");
  *out = nullptr;
  int64_t M = 0, Nc = 0;
  TRY(check_coo(d, rows, cols, nnz, coo_row, coo_col, coo_val, &M, &Nc));
  if (!(round_tol >= 0.0) || std::isinf(round_tol))
    return fail(TNRSVD_E_INVALID, "round_tol must be finite and >= 0");
  if (max_rank < 0) return fail(TNRSVD_E_INVALID, "max_rank must be >= 0");
  if (sat_mul(rows[0], cols[0]) > INT32_MAX)
    return fail(TNRSVD_E_SHAPE, "first core has more than 2^31 rows I_1 J_1");
  RoundedMpo res;
  int why = 0;
  TRY(dev_check(sparse_round(d, rows, cols, nnz, coo_row, coo_col, coo_val, round_tol, max_rank,
                             &res, &why, (hipStream_t)stream),
                "sparse rounding"));
  if (why == 1)
    return fail(TNRSVD_E_SHAPE, "COO index outside the %lld x %lld matrix", (long long)M,
                (long long)Nc);
  if (why == 2)
    return fail(TNRSVD_E_SHAPE, "more than 2^28 block positions (I / I_1) x (J / J_1)");
  if (why == 3) return fail(TNRSVD_E_SHAPE, "more than 16384 nonzero blocks");
  auto* r = new (std::nothrow) tnrsvd_rounded_s;
  if (!r) {
    for (double* p : res.cores) (void)hipFree(p);
    return fail(TNRSVD_E_NOMEM, "host allocation");
  }
  r->d = d;
  r->rows.assign(rows, rows + d);
  r->cols.assign(cols, cols + d);
  r->ranks = res.ranks;
  r->cores = res.cores;
  r->stream = (hipStream_t)stream;
  *out = r;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_round_mpo(const tnrsvd_mpo* a, double round_tol, int max_rank, void* stream,
                               tnrsvd_rounded_t* out) {
  g_err.clear();
  if (!out) return fail(TNRSVD_E_INVALID, "null out");
  *out = nullptr;
  if (!a) return fail(TNRSVD_E_INVALID, "null MPO");
  if (a->d < 1) return fail(TNRSVD_E_SHAPE, "d must be >= 1");
  if (!a->rank || !a->rows || !a->cols || !a->core)
    return fail(TNRSVD_E_INVALID, "null rank/rows/cols/core array");
  if (a->dtype != TNRSVD_F64 && a->dtype != TNRSVD_F32)
    return fail(TNRSVD_E_INVALID, "core dtype must be F64 or F32");
  if (!(round_tol >= 0.0) || std::isinf(round_tol))
    return fail(TNRSVD_E_INVALID, "round_tol must be finite and >= 0");
  if (max_rank < 0) return fail(TNRSVD_E_INVALID, "max_rank must be >= 0");
  const int d = a->d;
  if (a->rank[0] != 1 || a->rank[d] != 1) return fail(TNRSVD_E_SHAPE, "rank[0] and rank[d] must be 1");
  for (int k = 0; k < d; ++k) {
    const int64_t r0 = a->rank[k], n = sat_mul(a->rows[k], a->cols[k]), r1 = a->rank[k + 1];
    if (r0 < 1 || r1 < 1 || a->rows[k] < 1 || a->cols[k] < 1 || !a->core[k])
      return fail(TNRSVD_E_SHAPE, "core %d: bad shape or null pointer", k);
    if (r0 > kRoundRankMax || r1 > kRoundRankMax || a->rows[k] > INT32_MAX ||
        a->cols[k] > INT32_MAX || sat_mul(n, r1) > INT32_MAX || sat_mul(r0, n) > INT32_MAX)
      return fail(TNRSVD_E_SHAPE, "core %d: ranks above %d or a panel above 2^31 entries", k,
                  kRoundRankMax);
  }
  const hipStream_t s = (hipStream_t)stream;
  std::vector<const double*> c64(d);
  std::vector<void*> conv;
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : conv) (void)hipFree(p);
  };
  for (int k = 0; k < d; ++k) {
    if (a->dtype == TNRSVD_F64) {
      c64[k] = (const double*)a->core[k];
      continue;
    }
    const int64_t len = a->rank[k] * a->rows[k] * a->cols[k] * a->rank[k + 1];
    void* t = nullptr;
    if (hipMalloc(&t, sizeof(double) * (size_t)len) != hipSuccess) {
      (void)hipGetLastError();
      return release(), fail(TNRSVD_E_NOMEM, "FP64 copy of core %d", k);
    }
    conv.push_back(t);
    const hipError_t e = launch_convert_core(a->core[k], kF32, t, kF64, len, s);
    if (e != hipSuccess) return release(), dev_check(e, "widen core");
    c64[k] = (const double*)t;
  }
  RoundedMpo res;
  const hipError_t e =
      round_mpo(d, a->rank, a->rows, a->cols, c64.data(), round_tol, max_rank, &res, s);
  release();
  TRY(dev_check(e, "rounding"));
  auto* r = new (std::nothrow) tnrsvd_rounded_s;
  if (!r) {
    for (double* p : res.cores) (void)hipFree(p);
    return fail(TNRSVD_E_NOMEM, "host allocation");
  }
  r->d = d;
  r->rows.assign(a->rows, a->rows + d);
  r->cols.assign(a->cols, a->cols + d);
  r->ranks = res.ranks;
  r->cores = res.cores;
  r->stream = s;
  *out = r;
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_complex_embed(const tnrsvd_mpo* a, void* const* out, void* stream) {
  g_err.clear();
  if (!a || !out) return fail(TNRSVD_E_INVALID, "null argument");
  if (a->d < 1) return fail(TNRSVD_E_SHAPE, "d must be >= 1");
  if (!a->rank || !a->rows || !a->cols || !a->core)
    return fail(TNRSVD_E_INVALID, "null rank/rows/cols/core array");
  if (a->dtype != TNRSVD_F64 && a->dtype != TNRSVD_F32)
    return fail(TNRSVD_E_INVALID, "core dtype must be F64 or F32 (interleaved complex)");
  const int d = a->d;
  if (a->rank[0] != 1 || a->rank[d] != 1) return fail(TNRSVD_E_SHAPE, "rank[0] and rank[d] must be 1");
  for (int k = 0; k < d; ++k) {
    if (a->rank[k] < 1 || a->rank[k + 1] < 1 || a->rows[k] < 1 || a->cols[k] < 1 || !a->core[k] ||
        !out[k])
      return fail(TNRSVD_E_SHAPE, "core %d: bad shape or null pointer", k);
    if (sat_mul(sat_mul(sat_mul(a->rank[k], a->rows[k]), a->cols[k]), a->rank[k + 1]) >= kSat)
      return fail(TNRSVD_E_SHAPE, "core %d too large", k);
  }
  const hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < d; ++k)
    TRY(dev_check(launch_complex_embed(a->core[k], a->dtype == TNRSVD_F64 ? kF64 : kF32, out[k],
                                       a->rank[k], a->rows[k], a->cols[k], a->rank[k + 1], k == 0,
                                       k == d - 1, s),
                  "complex embedding"));
  return dev_check(hipStreamSynchronize(s), "synchronise");
}

tnrsvd_status tnrsvd_solve_complex(const tnrsvd_mpo* a, const tnrsvd_opts* opts, double* sigma) {
  g_err.clear();
  if (!a || !opts || !sigma) return fail(TNRSVD_E_INVALID, "null argument");
  if (opts->k < 1 || opts->p < 0) return fail(TNRSVD_E_INVALID, "k must be >= 1 and p >= 0");
  if (a->d < 1 || !a->rank || !a->rows || !a->cols)
    return fail(TNRSVD_E_INVALID, "null rank/rows/cols array or d < 1");
  if (a->dtype != TNRSVD_F64 && a->dtype != TNRSVD_F32)
    return fail(TNRSVD_E_INVALID, "core dtype must be F64 or F32 (interleaved complex)");
  const int d = a->d;
  if (!a->core) return fail(TNRSVD_E_INVALID, "null core array");
  if (a->rank[0] != 1 || a->rank[d] != 1) return fail(TNRSVD_E_SHAPE, "rank[0] and rank[d] must be 1");
  for (int k = 0; k < d; ++k)
    if (a->rank[k + 1] < 1 || a->rows[k] < 1 || a->cols[k] < 1 || !a->core[k])
      return fail(TNRSVD_E_SHAPE, "core %d: bad shape or null pointer", k);
  // shapes of the real form: inner ranks doubled, 2 I on the first core, 2 J
  // on the last
  std::vector<int64_t> rank(d + 1), rows(d), cols(d);
  for (int k = 0; k <= d; ++k) rank[k] = (k == 0 || k == d) ? 1 : 2 * a->rank[k];
  for (int k = 0; k < d; ++k) {
    rows[k] = (k == 0 ? 2 : 1) * a->rows[k];
    cols[k] = (k == d - 1 ? 2 : 1) * a->cols[k];
  }
  const size_t esz = a->dtype == TNRSVD_F64 ? sizeof(double) : sizeof(float);
  std::vector<void*> buf(d, nullptr);
  auto release_all = [&]() {
    (void)hipStreamSynchronize((hipStream_t)opts->stream);
    for (void* q : buf) (void)hipFree(q);
  };
  for (int k = 0; k < d; ++k) {
    const int64_t n = sat_mul(sat_mul(sat_mul(rank[k], rows[k]), cols[k]), rank[k + 1]);
    if (n >= kSat || n < 1) {
      release_all();
      return fail(TNRSVD_E_SHAPE, "core %d of the real form too large", k);
    }
    if (hipMalloc(&buf[k], esz * (size_t)n) != hipSuccess) {
      (void)hipGetLastError();
      release_all();
      return fail(TNRSVD_E_NOMEM, "real form of core %d", k);
    }
  }
  tnrsvd_status st = tnrsvd_complex_embed(a, buf.data(), opts->stream);
  if (st != TNRSVD_OK) {
    release_all();
    return st;
  }
  tnrsvd_mpo real;
  real.d = d;
  real.rank = rank.data();
  real.rows = rows.data();
  real.cols = cols.data();
  real.core = (const void* const*)buf.data();
  real.dtype = a->dtype;
  tnrsvd_opts o = *opts;
  o.k = 2 * opts->k;
  o.p = 2 * opts->p;
  tnrsvd_t h = nullptr;
  st = tnrsvd_create(&h, 1, &real, &o);
  std::vector<double> s2((size_t)o.k);
  if (st == TNRSVD_OK) st = tnrsvd_run(h, s2.data());
  if (h) {
    const std::string keep = g_err;   // destroy must not hide the first error
    (void)tnrsvd_destroy(h);
    g_err = keep;
  }
  release_all();
  if (st != TNRSVD_OK) return st;
  for (int j = 0; j < opts->k; ++j) sigma[j] = s2[(size_t)2 * j];
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_mpo_add(const tnrsvd_mpo* a, const tnrsvd_mpo* b, void* const* out,
                             void* stream) {
  g_err.clear();
  if (!a || !b || !out) return fail(TNRSVD_E_INVALID, "null argument");
  if (a->d < 1 || b->d != a->d) return fail(TNRSVD_E_SHAPE, "d must be >= 1 and equal");
  for (const tnrsvd_mpo* m : {a, b})
    if (!m->rank || !m->rows || !m->cols || !m->core)
      return fail(TNRSVD_E_INVALID, "null rank/rows/cols/core array");
  if ((a->dtype != TNRSVD_F64 && a->dtype != TNRSVD_F32) || b->dtype != a->dtype)
    return fail(TNRSVD_E_INVALID, "both MPOs must be F64 or both F32");
  const int d = a->d;
  for (const tnrsvd_mpo* m : {a, b})
    if (m->rank[0] != 1 || m->rank[d] != 1)
      return fail(TNRSVD_E_SHAPE, "rank[0] and rank[d] must be 1");
  for (int k = 0; k < d; ++k) {
    if (a->rows[k] < 1 || a->cols[k] < 1 || b->rows[k] != a->rows[k] ||
        b->cols[k] != a->cols[k] || a->rank[k + 1] < 1 || b->rank[k + 1] < 1 || !a->core[k] ||
        !b->core[k] || !out[k])
      return fail(TNRSVD_E_SHAPE, "core %d: modes differ, bad rank or null pointer", k);
    const int64_t L = k == 0 ? 1 : a->rank[k] + b->rank[k];
    const int64_t R = k == d - 1 ? 1 : a->rank[k + 1] + b->rank[k + 1];
    if (L > ((int64_t)1 << 20) || R > ((int64_t)1 << 20) ||
        sat_mul(sat_mul(sat_mul(L, a->rows[k]), a->cols[k]), R) >= kSat)
      return fail(TNRSVD_E_SHAPE, "core %d of the sum too large", k);
  }
  const hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < d; ++k)
    TRY(dev_check(launch_mpo_add(a->core[k], b->core[k], out[k],
                                 a->dtype == TNRSVD_F64 ? kF64 : kF32, a->rank[k], b->rank[k],
                                 a->rows[k], a->cols[k], a->rank[k + 1], b->rank[k + 1], k == 0,
                                 k == d - 1, s),
                  "MPO addition"));
  return dev_check(hipStreamSynchronize(s), "synchronise");
}

tnrsvd_status tnrsvd_rounded_ranks(tnrsvd_rounded_t r, int64_t* ranks) {
  if (!r || !ranks) return fail(TNRSVD_E_INVALID, "null argument");
  for (int k = 0; k <= r->d; ++k) ranks[k] = r->ranks[k];
  return TNRSVD_OK;
}

tnrsvd_status tnrsvd_rounded_copy(tnrsvd_rounded_t r, int k, double* dst) {
  if (!r || !dst) return fail(TNRSVD_E_INVALID, "null argument");
  if (k < 0 || k >= r->d) return fail(TNRSVD_E_INVALID, "core index out of range");
  const int64_t n = r->ranks[k] * r->rows[k] * r->cols[k] * r->ranks[k + 1];
  TRY(dev_check(hipMemcpyAsync(dst, r->cores[k], sizeof(double) * (size_t)n,
                               hipMemcpyDeviceToDevice, r->stream),
                "copy core"));
  return dev_check(hipStreamSynchronize(r->stream), "synchronise");
}

tnrsvd_status tnrsvd_rounded_destroy(tnrsvd_rounded_t r) {
  if (!r) return TNRSVD_OK;
  for (double* p : r->cores)
    if (p) (void)hipFree(p);
  delete r;
  return TNRSVD_OK;
}

}  // extern "C"
