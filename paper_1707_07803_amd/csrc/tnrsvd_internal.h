// Internal declarations shared by the TNrSVD HIP sources (gfx950 only).
//
// Data model (all device resident, one slab per kind, offsets in elements):
//   A slab    (T)      merged MPO cores of every MPO, (R, I, J, R')
//   X slab    (T)      current basis cores (r, n, r'), last core (r, n, K)
//   Z slab    (T)      product cores (P, n, P'), P = R * r, last core (P, n, K)
//   W slab    (double) per core: the absorbed panel Zt = Z x_3 L, stored as
//                      Zt^T in column-major (m x P, m = n * rho'), overwritten
//                      in place by its Householder QR (R above, vectors below)
//   L slab    (double) per core: the rho x P upper-trapezoidal R of that QR,
//                      i.e. L^T of the LQ Zt = L Qt
//   TAU slab  (double) per core: Householder scalars
//   scratch   (double) per MPO: carried factor T, panel M, Jacobi vectors
// Dynamic ranks live in device int arrays indexed by MpoDesc::r0 + bond, so a
// whole solve is enqueued without reading anything back to the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

namespace tnr {

// Per (MPO, merged core) static plan.
struct CoreDesc {
  int I, J;          // row / column mode sizes of the (merged) core
  int RA, RA2;       // A ranks left / right (RA2 = 1 on the last core)
  int xcap, xcap2;   // capacity of basis ranks left / right (xcap2 = K last)
  int64_t a_off;     // A slab
  int64_t x_off;     // X slab, capacity xcap * max(I,J) * xcap2
  int64_t z_off;     // Z slab, capacity (RA*xcap) * max(I,J) * (RA2*xcap2)
  int64_t w_off;     // W slab, capacity max(I,J) * (RA2*xcap2) * (RA*xcap)
  int64_t l_off;     // L slab, capacity (RA*xcap)^2 (rho <= P)
  int64_t tau_off;   // TAU slab, capacity RA*xcap
  int64_t y0_off;    // Y0 slab (first product), capacity RA * I * RA2 * (xcap2 == K ? K : 1)
  int64_t u_off;     // U / V output slab (double), capacity xcap * max(I,J) * xcap2
  int64_t wt_off;    // W slab: compact-WY factor T of every 32-column block of
                     // the multi-workgroup QR, ceil(RA * xcap / 32) x 32 x 32
};

// Per MPO static plan.
struct MpoDesc {
  int d;             // merged core count
  int K;             // k + p
  int c0;            // first CoreDesc of this MPO
  int r0;            // first bond slot of this MPO in the rank arrays (d + 1 slots)
  int64_t om_off;    // Omega (double): sum_{i<d-1} J_i + J_{d-1} * K values
  int64_t s_off;     // scratch (double) of this MPO
  int64_t s_len;     // scratch length (doubles)
  int64_t out_off;   // small outputs (double): sigma[K], W[K*K], R_K[K*K]
  int mcap;          // max panel rows of this MPO (n * rho' over cores)
  int pcap;          // max product rank of this MPO
  // multi-workgroup right-to-left path (WV slab): two explicit reflector
  // blocks of wmcap x 32 (double-buffered) and the nested-QR workspace
  // (wmcap * 16 + 1024); wmcap bounds the panel rows n * rho' of every core
  int64_t wv_off;
  int wmcap;
};

// Rank arrays (device, int): one slot per bond, MpoDesc::r0 + i, i = 0..d.
//   xr  : current basis ranks (xr[0] = 1, xr[d] = K)
//   pr  : product ranks P_i = R_i * xr_i of the pending product (pr[d] = K)
//   rho : ranks after the right-to-left LQ sweep (rho[d] = K)

// Sweep options passed by value.
struct SweepOpts {
  double eps;        // rounding tolerance
  int rmax;          // rank cap (0 = none)
  int mode;          // 0: orthogonalise (QR of the last core), 1: solve (SVD)
  int64_t qcap;      // scratch doubles per MPO for the QR-preconditioned Jacobi
};

// BF16 storage: the upper 16 bits of an FP32 (1 sign, 8 exponent, 7 fraction
// bits).  FP32 -> BF16 rounds to nearest, ties to even; NaN stays a quiet NaN.
// FP64 values are narrowed through FP32.  Arithmetic on it is always done in
// FP32 or wider after an explicit conversion.
struct bf16 {
  unsigned short u;
  bf16() = default;
  __host__ __device__ explicit bf16(float f) : u(from_f32(f)) {}
  __host__ __device__ explicit bf16(double d) : u(from_f32((float)d)) {}
  __host__ __device__ explicit operator float() const {
    return __builtin_bit_cast(float, (unsigned)u << 16);
  }
  __host__ __device__ explicit operator double() const { return (double)(float)(*this); }
  __host__ __device__ static unsigned short from_f32(float f) {
    unsigned x = __builtin_bit_cast(unsigned, f);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((x >> 16) | 0x40u);
    x += 0x7fffu + ((x >> 16) & 1u);
    return (unsigned short)(x >> 16);
  }
};

// Storage codes of the contraction slabs (A, X, Z, Y0).
constexpr int kF64 = 0, kF32 = 1, kBF16 = 2;

// Host-side dispatch on a storage code: f receives a null pointer of the type.
template <typename F>
inline void by_dtype(int dt, F&& f) {
  if (dt == kF64) f((double*)nullptr);
  else if (dt == kF32) f((float*)nullptr);
  else f((bf16*)nullptr);
}
template <typename P>
using elem_t = std::remove_const_t<std::remove_pointer_t<P>>;

constexpr int kSweepThreads = 512;
constexpr int kMaxK = 256;
constexpr int kRoundRankMax = 4096;  // bond ranks taken by the rounding of a general MPO
constexpr int kSweepArena = 19456;   // doubles of static LDS per sweep workgroup
// register panels of the sweeps: at most 256 rows x 128 columns; a last-core
// panel of up to 16 such row blocks is factorised by TSQR
constexpr int kRegRows = 256, kRegCols = 128, kTsqrLeavesMax = 16;
constexpr int kSortCap = 990;        // largest panel row count the sweep sorts

}  // namespace tnr

// Gradient workspace of one MPO: five temporaries of tmpcap doubles from tmp0.
struct GradMpo {
  int64_t tmp0;
  int64_t tmpcap;
};

// Launchers implemented in the .hip sources, called from the ABI layer.
namespace tnr {

// Counter-based Gaussian stream shared by Omega and the product sketches.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
  // SplitMix64 (Steele, Lea, Flood 2014) in counter form: state seed + (n+1) * golden gamma.
  uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double gaussian_at(uint64_t seed, uint64_t n) {
  // Box-Muller on the pair (2k, 2k+1): u1 in (0,1], u2 in [0,1).
  const uint64_t k = n >> 1;
  const double u1 = (double)((splitmix64_at(seed, 2 * k) >> 11) + 1ull) * 0x1.0p-53;
  const double u2 = (double)(splitmix64_at(seed, 2 * k + 1) >> 11) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * 3.14159265358979311600 * u2;
  return (n & 1ull) ? rad * sin(ang) : rad * cos(ang);
}

hipError_t launch_merge_pair(const double* Tin, const double* C, double* out, int a, int I1, int J1,
                             int b, int I2, int J2, int b2, hipStream_t s);
hipError_t launch_convert_core(const void* in, int in_dtype, void* out, int out_dtype, int64_t n,
                               hipStream_t s);
hipError_t launch_check_finite(const void* in, int dtype, int64_t n, int* flag, hipStream_t s);
// digits of a merged mode index, least significant first; below[k] is the
// product of r[k+1..nd-1] (the digit's weight once the order is reversed)
struct Radices {
  static constexpr int kMax = 32;
  int64_t r[kMax];
  int64_t below[kMax];
  int nd;
};
hipError_t launch_reverse_core(const void* in, int dtype, void* out, int64_t R0, int64_t n,
                               int64_t R1, const Radices& rad, hipStream_t s);
// Sketched product truncation (opt-in): per-MPO FP64 workspace and launch.
__host__ __device__ inline int64_t sketch_ws_doubles(int d, int64_t pc, int64_t nm, int64_t K,
                                                     int64_t ell) {
  const int64_t m = ell * nm;
  return (int64_t)(d - 1) * pc * ell        // W at bonds 1 .. d-1
         + ell * nm * (ell > K ? ell : K)   // one sketch core
         + nm * pc * ell                    // U2
         + ell * nm * (pc > K ? pc : K)     // Zt
         + 2 * m * ell                      // M and Q
         + ell + 2 * ell * pc               // tau, C, C2
         + m * 33 + 64 * ell;               // QR workspace (block width <= 32)
}
constexpr int kSketchMaxD = 256;
hipError_t launch_sketch(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op, int* pr,
                         void* Z, int dtype, int ell, uint64_t seed, uint64_t cbase,
                         const int* nm, const int64_t* off, double* ws, int* err, hipStream_t s);
hipError_t launch_mpo_add(const void* A, const void* B, void* C, int dtype, int64_t ra0,
                          int64_t rb0, int64_t I, int64_t J, int64_t ra1, int64_t rb1, int first,
                          int last, hipStream_t s);
hipError_t launch_complex_embed(const void* in, int dtype, void* out, int64_t R0, int64_t I,
                                int64_t J, int64_t R1, int first, int last, hipStream_t s);
hipError_t launch_swap_legs(const void* in, int dtype, void* out, int64_t R0, int64_t I, int64_t J,
                            int64_t R1, hipStream_t s);
hipError_t launch_omega(const MpoDesc* mpos, const CoreDesc* cores, int batch, uint64_t seed,
                        double* om, int64_t max_len, hipStream_t s);
hipError_t launch_load_omega(const MpoDesc* mpos, const CoreDesc* cores, int batch,
                             const double* om, int* xr, void* X, int dtype, int max_d,
                             int64_t max_len, int* err, hipStream_t s);
hipError_t launch_contract(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                           int ncores, const int* xr, int* pr, const void* A, const void* X,
                           void* Z, int dtype, int op, int64_t max_out, int* err, int threads,
                           int gcap, hipStream_t s);
hipError_t launch_copy_y0(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                          int ncores, const int* pr, const void* Z, void* Y0, int dtype,
                          int64_t max_out, hipStream_t s);
hipError_t launch_rl_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* pr, int* rho, int* ldm, const void* Z, int dtype, double* Wd,
                          double* L, double* tau, int* err, int leaf_nc, const int* wflag,
                          const int* order, hipStream_t s);
// Wide right-to-left pass (kernels_wide.hip).  Per step t (core d-1-t of every
// MPO) the plan holds kWidePlan ints: column blocks of the QR, and bounds on
// P, panel rows m, rho' and the mode size n (grid sizes of the launches).
constexpr int kWidePlan = 5;
constexpr int kWideNB = 32;   // column block of the multi-workgroup QR
hipError_t launch_wide_classify(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                                const int* pr, const int* plan, int max_d, int wmin, int* wflag,
                                int* need, hipStream_t s);
hipError_t launch_rl_wide_step(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                               const int* pr, int* rho, int* ldm, const int* wflag, const void* Z,
                               int dtype, double* Wd, double* WV, double* L, double* tau, int t,
                               const int* plan_t, hipStream_t s);
hipError_t launch_lr_pass(const MpoDesc* mpos, const CoreDesc* cores, int batch, int op,
                          const int* rho, const int* ldm, int* xr, const double* Wd,
                          const double* tau, double* scratch, void* Xout, int out_dtype,
                          double* outs, SweepOpts o, int64_t tcap, int64_t mcap_s, int64_t ucap,
                          int* err, const int* wflag, const int* order, hipStream_t s);
hipError_t launch_form_u(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                         int ncores, const int* xr, const void* X, int dtype, const double* outs,
                         double* U, int64_t max_out, int* err, hipStream_t s);
hipError_t launch_grad_env(const MpoDesc* mpos, const CoreDesc* cores, const GradMpo* gm,
                           const int64_t* eoff, int batch, const int* xr, const int* vr,
                           const void* A, int dtype, const double* U, const double* V,
                           const double* w, int k, double* ws, double* G, int* err,
                           hipStream_t s);
hipError_t sparse_to_mpo(int d, const int64_t* I, const int64_t* J, int64_t nnz,
                         const int64_t* row, const int64_t* col, const double* val,
                         int64_t expect, int64_t* nblocks, double* const* cores, int* bad_index,
                         hipStream_t s);
// The same conversion on the library's static device scratch (no allocation):
// *need receives the scratch bytes the input takes; when that exceeds
// kNoAllocScratchBytes nothing runs and hipSuccess is returned.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int kNoAllocDevices = 64;   // device ordinals served
constexpr int kNoAllocMaxD = 64;      // cores of the converted MPO
hipError_t sparse_to_mpo_noalloc(int d, const int64_t* I, const int64_t* J, int64_t nnz,
                                 const int64_t* row, const int64_t* col, const double* val,
                                 int64_t expect, int64_t* nblocks, double* const* cores,
                                 int* bad_index, size_t* need, hipStream_t s);
// Rounding of Algorithm 4.1's MPO (kernels_round.hip; orchestrated in kernels_sparse.hip).
int64_t qr_ws_doubles(int64_t m, int64_t n);
int64_t colsign_chunks(int64_t n1);
hipError_t launch_tsqr_leaf(double* Pw, int h, int N, int L, double* tau, double* ws, int64_t wss,
                            double* up, hipStream_t s);
hipError_t launch_tsqr_node(double* S, int N, int cnt, double* tau, double* ws, int64_t wss,
                            double* up, hipStream_t s);
hipError_t launch_root_svd(const double* Rf, int N, int64_t n1, double eps, int dm1, int rmax,
                           double* B, double* U, double* nrm, double* sig, int* perm, int* flag,
                           double* Y0, double* T, int* rho_out, double* delta_out, hipStream_t s);
hipError_t launch_tsqr_apply_node(const double* S, const double* tau, int N, int rho, int cnt,
                                  const double* Yup, int root, double* Yl, hipStream_t s);
hipError_t launch_tsqr_apply_leaf(const double* Pw, const double* tau, int h, int N, int rho,
                                  int64_t n1, int L, const double* Yup, double* core1,
                                  hipStream_t s);
hipError_t launch_colsign(double* X, int64_t n1, int rho, double* T, int N, double* pv,
                          int64_t* pi, double* sgn, hipStream_t s);
hipError_t launch_round_level(const double* T, int rp, int cp, const int* pm, const int* nx, int n,
                              int q, const double* delta_p, int rmax, double* M, double* ws,
                              double* tau, double* B, double* U, double* nrm, double* sig,
                              int* perm, double* sgn, int* flag, double* Y, double* core,
                              double* Tn, int* rho_out, hipStream_t s);
hipError_t launch_round_last(const double* T, int rp, int cp, const int* pm, int n, double* core,
                             hipStream_t s);

// Result of sparse_round: ranks (d + 1) and d device cores (C order (r, I, J, r')),
// owned by the caller of sparse_round (hipFree each).
// Device allocations of one call, freed together except those released.
struct DevArena {
  std::vector<void*> ptrs;
  hipError_t e = hipSuccess;
  template <typename P>
  P* get(int64_t count) {
    if (e != hipSuccess) return nullptr;
    void* p = nullptr;
    e = hipMalloc(&p, sizeof(P) * (size_t)(count > 0 ? count : 1));
    if (e != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (P*)p;
  }
  void release(const void* p) {
    for (auto& q : ptrs)
      if (q == p) q = nullptr;
  }
  ~DevArena() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
};

struct RoundedMpo {
  std::vector<int64_t> ranks;
  std::vector<double*> cores;
};
// Status beyond hipError_t: 1 = an index outside the matrix, 2 = more block
// positions than the bitmap path takes, 3 = more blocks than the rounding takes.
hipError_t sparse_round(int d, const int64_t* I, const int64_t* J, int64_t nnz, const int64_t* row,
                        const int64_t* col, const double* val, double eps, int rmax,
                        RoundedMpo* out, int* why, hipStream_t s);
// SVD-based rounding (Sec. 3) of a general MPO with FP64 device cores
// (r_k, I_k, J_k, r_{k+1}); the input cores are not modified.
hipError_t round_mpo(int d, const int64_t* rank, const int64_t* I, const int64_t* J,
                     const double* const* cores, double eps, int rmax, RoundedMpo* out,
                     hipStream_t s);
// Reverse-mode derivative of the whole solve for one MPO (kernels_adjoint.hip).
struct CoreShape {
  int Ra, I, J, Rb;
};
hipError_t pipeline_adjoint(int d, const CoreShape* shapes, const double* const* A,
                            double* const* dA, const double* omega, int K, int k,
                            const double* dsigma_host,
                            const std::vector<std::vector<int>>& ranks,
                            const std::vector<int>& ops, hipStream_t s);
hipError_t launch_merge_pair_bwd(const double* T, const double* C, const double* dN, double* dT,
                                 double* dC, int a, int I1, int J1, int r, int I2, int J2, int b,
                                 hipStream_t s);
}  // namespace tnr
