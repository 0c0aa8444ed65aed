// Core-local kernels of the TNrSVD hot path on gfx950:
//   * merging of the trailing MPO cores (the K-core enlargement of Sec. 6.3),
//   * the counter-based random MPO (lemma of Sec. 5.1),
//   * the MPO x MPS products of Sec. 5.2 (Y = A X and Z = A^T X), and
//   * forming U = Q W on the last core (Sec. 5.4).
// Every kernel reads its shapes from device descriptors, so the host never
// waits on the device between launches.
#include "tnrsvd_internal.h"

namespace tnr {

namespace {

template <typename T>
struct Acc { using type = float; };
template <>
struct Acc<double> { using type = double; };

__global__ void k_merge_pair(const double* __restrict__ T, const double* __restrict__ C,
                             double* __restrict__ out, int a, int I1, int J1, int b, int I2,
                             int J2, int b2) {
  // out[a, x + I1 x', y + J1 y', e] = sum_beta T[a, x, y, beta] C[beta, x', y', e]
  const int64_t I = (int64_t)I1 * I2, J = (int64_t)J1 * J2;
  const int64_t total = (int64_t)a * I * J * b2;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(o % b2);
    int64_t t = o / b2;
    const int64_t Y = t % J;
    t /= J;
    const int64_t X = t % I;
    const int aa = (int)(t / I);
    const int x = (int)(X % I1), xp = (int)(X / I1);
    const int y = (int)(Y % J1), yp = (int)(Y / J1);
    double acc = 0.0;
    for (int beta = 0; beta < b; ++beta)
      acc += T[(((int64_t)aa * I1 + x) * J1 + y) * b + beta] *
             C[(((int64_t)beta * I2 + xp) * J2 + yp) * b2 + e];
    out[o] = acc;
  }
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (TO)in[i];
}

template <typename TI>
__global__ void k_check_finite(const TI* __restrict__ in, int64_t n, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)in[i];
    if (!isfinite(v)) atomicOr(flag, 1);
  }
}

__device__ inline int64_t omega_len(const MpoDesc& md, const CoreDesc* cores) {
  int64_t n = 0;
  for (int i = 0; i < md.d - 1; ++i) n += cores[md.c0 + i].J;
  n += (int64_t)cores[md.c0 + md.d - 1].J * md.K;
  return n;
}

__global__ void k_omega(const MpoDesc* mpos, const CoreDesc* cores, uint64_t seed, double* om) {
  const MpoDesc md = mpos[blockIdx.y];
  const int64_t n = omega_len(md, cores);
  const uint64_t s = seed + (uint64_t)blockIdx.y;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    om[md.om_off + t] = gaussian_at(s, (uint64_t)t);
}

template <typename T>
__global__ void k_load_omega(const MpoDesc* mpos, const CoreDesc* cores, const double* om,
                             int* xr, T* X, int* err) {
  // Basis := Omega as rank-1 cores (1, J_i, 1) and (1, J_{d-1}, K).  A new
  // solve starts here, so the first block also clears the capacity flags
  // (a kernel store, so the whole solve stays capturable in a graph).
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) err[0] = 0;
  const MpoDesc md = mpos[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= md.d) return;
  int64_t off = 0;
  for (int j = 0; j < i; ++j) off += cores[md.c0 + j].J;
  const CoreDesc cd = cores[md.c0 + i];
  const int64_t n = (i == md.d - 1) ? (int64_t)cd.J * md.K : cd.J;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x)
    X[cd.x_off + t] = (T)om[md.om_off + off + t];
  if (threadIdx.x == 0) {
    xr[md.r0 + i] = 1;
    if (i == md.d - 1) xr[md.r0 + md.d] = md.K;
  }
}

// Z_i[(a,c), n, (b,e)] = sum_s A_i[a, x|s, s|y, b] X_i[c, s, e]   (Sec. 5.2)
//   OP 0 (Y = A X):   output mode x in I_i, shared mode y in J_i
//   OP 1 (Z = A^T X): output mode y in J_i, shared mode x in I_i
// Output element o = ((p * n_out + x) * P' + q), p = a * r + c, q = b * r' + e.
template <typename T, int OP>
__global__ void k_contract(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                           const int* xr, int* pr, const T* __restrict__ A,
                           const T* __restrict__ X, T* __restrict__ Z, int* err) {
  using ACC = typename Acc<T>::type;
  const int g = blockIdx.y;
  const int b = core_mpo[g];
  const MpoDesc md = mpos[b];
  const int i = g - md.c0;
  const CoreDesc cd = cores[g];
  const int r = xr[md.r0 + i], r2 = xr[md.r0 + i + 1];
  if (r < 1 || r > cd.xcap || r2 < 1 || r2 > cd.xcap2) {  // capacity guard (block uniform)
    if (threadIdx.x == 0) atomicOr(err, 4);
    return;
  }
  const int P = cd.RA * r, P2 = cd.RA2 * r2;
  const int nout = OP == 0 ? cd.I : cd.J;
  const int nsh = OP == 0 ? cd.J : cd.I;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    pr[md.r0 + i] = P;
    if (i == md.d - 1) pr[md.r0 + md.d] = P2;
  }
  const int64_t total = (int64_t)P * nout * P2;
  const T* Ac = A + cd.a_off;
  const T* Xc = X + cd.x_off;
  T* Zc = Z + cd.z_off;
  const int64_t sa_x = (int64_t)cd.J * cd.RA2;  // stride of x in A
  const int64_t sa_y = cd.RA2;                   // stride of y in A
  const int64_t sa_s = OP == 0 ? sa_y : sa_x;
  const int64_t sa_o = OP == 0 ? sa_x : sa_y;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(o % P2);
    const int64_t t = o / P2;
    const int xo = (int)(t % nout);
    const int p = (int)(t / nout);
    const int a = p / r, c = p % r;
    const int bb = q / r2, e = q % r2;
    const T* ap = Ac + (int64_t)a * cd.I * sa_x + xo * sa_o + bb;
    const T* xp = Xc + (int64_t)c * nsh * r2 + e;
    ACC acc = 0;
    for (int s = 0; s < nsh; ++s) acc += (ACC)ap[s * sa_s] * (ACC)xp[(int64_t)s * r2];
    Zc[o] = (T)acc;
  }
}

template <typename T>
__global__ void k_copy_y0(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                          const int* pr, const T* __restrict__ Z, T* __restrict__ Y0) {
  const int g = blockIdx.y;
  const MpoDesc md = mpos[core_mpo[g]];
  const int i = g - md.c0;
  const CoreDesc cd = cores[g];
  const int64_t total = (int64_t)pr[md.r0 + i] * cd.I * pr[md.r0 + i + 1];
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x)
    Y0[cd.y0_off + o] = Z[cd.z_off + o];
}

// U cores: copies of the basis Q in FP64; on the last core U = Q W (Sec. 5.4).
template <typename T>
__global__ void k_form_u(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                         const int* xr, const T* __restrict__ X, const double* outs,
                         double* __restrict__ U, int* err) {
  const int g = blockIdx.y;
  const MpoDesc md = mpos[core_mpo[g]];
  const int i = g - md.c0;
  const CoreDesc cd = cores[g];
  const int r = xr[md.r0 + i], r2 = xr[md.r0 + i + 1];
  if (r < 1 || r > cd.xcap || r2 < 1 || r2 > cd.xcap2) {
    if (threadIdx.x == 0) atomicOr(err, 4);
    return;
  }
  const int64_t total = (int64_t)r * cd.I * r2;
  const T* Xc = X + cd.x_off;
  double* Uc = U + cd.u_off;
  if (i < md.d - 1) {
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * blockDim.x)
      Uc[o] = (double)Xc[o];
    return;
  }
  const int K = md.K;
  const double* W = outs + md.out_off + K;  // W (K x K, row-major: W[kappa, j])
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(o % K);
    const int64_t row = o / K;
    double acc = 0.0;
    for (int kk = 0; kk < K; ++kk) acc += (double)Xc[row * K + kk] * W[kk * K + j];
    Uc[o] = acc;
  }
}

inline int grid_for(int64_t n, int threads, int cap) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_merge_pair(const double* Tin, const double* C, double* out, int a, int I1,
                             int J1, int b, int I2, int J2, int b2, hipStream_t s) {
  const int64_t total = (int64_t)a * I1 * I2 * J1 * J2 * b2;
  k_merge_pair<<<grid_for(total, 256, 65535), 256, 0, s>>>(Tin, C, out, a, I1, J1, b, I2, J2, b2);
  return hipGetLastError();
}

hipError_t launch_convert_core(const void* in, int in_dtype, void* out, int out_dtype, int64_t n,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = grid_for(n, 256, 4096);
  auto go = [&](auto* ti, auto* to) {
    using TI = std::remove_pointer_t<decltype(ti)>;
    using TO = std::remove_pointer_t<decltype(to)>;
    k_convert<TI, TO><<<g, 256, 0, s>>>((const TI*)in, (TO*)out, n);
  };
  auto out_as = [&](auto* ti) {
    if (out_dtype == kF64) go(ti, (double*)nullptr);
    else if (out_dtype == kF32) go(ti, (float*)nullptr);
    else go(ti, (bf16*)nullptr);
  };
  if (in_dtype == kF64) out_as((double*)nullptr);
  else if (in_dtype == kF32) out_as((float*)nullptr);
  else out_as((bf16*)nullptr);
  return hipGetLastError();
}

// out (R1, I, J, R0) = in (R0, I, J, R1) with the two rank legs swapped: one
// core of an MPO (J = 1: of an MPS) read in the reversed core order.
template <typename T>
__global__ void k_swap_legs(const T* __restrict__ in, T* __restrict__ out, int64_t R0, int64_t I,
                            int64_t J, int64_t R1) {
  const int64_t n = R0 * I * J * R1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % R1, ij = (e / R1) % (I * J), a = e / (R1 * I * J);
    out[(b * I * J + ij) * R0 + a] = in[e];
  }
}

hipError_t launch_swap_legs(const void* in, int dtype, void* out, int64_t R0, int64_t I, int64_t J,
                            int64_t R1, hipStream_t s) {
  const int64_t n = R0 * I * J * R1;
  if (n <= 0) return hipSuccess;
  const int g = grid_for(n, 256, 4096);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_swap_legs<T><<<g, 256, 0, s>>>((const T*)in, (T*)out, R0, I, J, R1);
  });
  return hipGetLastError();
}

// out (R1, n, R0) = in (R0, n, R1) with the rank legs swapped and the mode
// index n, little-endian in the digits of radices rad[0..nd-1] (eq. (1)),
// rewritten little-endian in the reversed digit order: one core of an MPS whose
// cores, some of them merged, are read in the reversed order.
template <typename T>
__global__ void k_reverse_core(const T* __restrict__ in, T* __restrict__ out, int64_t R0, int64_t n,
                               int64_t R1, Radices rad) {
  const int64_t total = R0 * n * R1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % R1, a = e / (R1 * n);
    int64_t idx = (e / R1) % n, rev = 0;
    for (int k = 0; k < rad.nd; ++k) {   // digit k weighs the radices after it
      rev += (idx % rad.r[k]) * rad.below[k];
      idx /= rad.r[k];
    }
    out[(b * n + rev) * R0 + a] = in[e];
  }
}

hipError_t launch_reverse_core(const void* in, int dtype, void* out, int64_t R0, int64_t n,
                               int64_t R1, const Radices& rad, hipStream_t s) {
  const int64_t total = R0 * n * R1;
  if (total <= 0) return hipSuccess;
  const int g = grid_for(total, 256, 4096);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_reverse_core<T><<<g, 256, 0, s>>>((const T*)in, (T*)out, R0, n, R1, rad);
  });
  return hipGetLastError();
}

// Real form of one core of a complex MPO (interleaved re/im of T, shape
// (R0, I, J, R1)): every bond entry z becomes phi(z) = [[Re z, -Im z],
// [Im z, Re z]], bond index (a, s) -> 2 a + s.  On the first core (first != 0)
// the left component s instead becomes the most significant digit of the row
// mode (i' = s I + i, left rank 1); on the last core the right component t
// becomes the most significant digit of the column mode (j' = t J + j).
template <typename T>
__global__ void k_complex_embed(const T* __restrict__ in, T* __restrict__ out, int64_t R0,
                                int64_t I, int64_t J, int64_t R1, int first, int last) {
  const int64_t Io = first ? 2 * I : I, Jo = last ? 2 * J : J, R1o = last ? 1 : 2 * R1;
  const int64_t n = R0 * I * J * R1 * 4;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int st = (int)(e & 3), s = st >> 1, t = st & 1;
    const int64_t src = e >> 2;
    const int64_t b = src % R1, j = (src / R1) % J, i = (src / (R1 * J)) % I, a = src / (R1 * J * I);
    const T re = in[2 * src], im = in[2 * src + 1];
    const T v = s == t ? re : (s == 0 ? T(-(double)im) : im);
    const int64_t ao = first ? 0 : 2 * a + s, io = first ? s * I + i : i;
    const int64_t jo = last ? t * J + j : j, bo = last ? 0 : 2 * b + t;
    out[((ao * Io + io) * Jo + jo) * R1o + bo] = v;
  }
}

hipError_t launch_complex_embed(const void* in, int dtype, void* out, int64_t R0, int64_t I,
                                int64_t J, int64_t R1, int first, int last, hipStream_t s) {
  const int64_t n = R0 * I * J * R1 * 4;
  if (n <= 0) return hipSuccess;
  const int g = grid_for(n, 256, 4096);
  if (dtype == kF64)
    k_complex_embed<double><<<g, 256, 0, s>>>((const double*)in, (double*)out, R0, I, J, R1,
                                              first, last);
  else
    k_complex_embed<float><<<g, 256, 0, s>>>((const float*)in, (float*)out, R0, I, J, R1, first,
                                             last);
  return hipGetLastError();
}

// MPO addition (Sec. 3), one core of the sum C = A + B per launch: ranks add,
// so an inner core is block diagonal, diag(A_k, B_k); the first core stacks A's
// and B's right rank legs, the last core their left rank legs, and for d = 1 the
// single core is A_1 + B_1.  Output (a, i, j, b) in C order over
// (ra0 + rb0 or 1) x I x J x (ra1 + rb1 or 1); a left (right) index belongs to
// A below ra0 (ra1), to B from there on, and to both on the first (last) core.
template <typename T>
__global__ void k_mpo_add(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
                          int64_t ra0, int64_t rb0, int64_t I, int64_t J, int64_t ra1,
                          int64_t rb1, int first, int last) {
  const int64_t L = first ? 1 : ra0 + rb0, Rr = last ? 1 : ra1 + rb1;
  const int64_t n = L * I * J * Rr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % Rr, ij = (e / Rr) % (I * J), a = e / (Rr * I * J);
    const bool la = first || a < ra0, lb = first || a >= ra0;
    const bool ka = last || b < ra1, kb = last || b >= ra1;
    double v = 0.0;
    if (la && ka) {
      const int64_t aa = first ? 0 : a, ba = last ? 0 : b;
      v += (double)A[(aa * I * J + ij) * (last ? 1 : ra1) + ba];
    }
    if (lb && kb) {
      const int64_t ab = first ? 0 : a - ra0, bb = last ? 0 : b - ra1;
      v += (double)B[(ab * I * J + ij) * (last ? 1 : rb1) + bb];
    }
    C[e] = T(v);
  }
}

hipError_t launch_mpo_add(const void* A, const void* B, void* C, int dtype, int64_t ra0,
                          int64_t rb0, int64_t I, int64_t J, int64_t ra1, int64_t rb1, int first,
                          int last, hipStream_t s) {
  const int64_t n = (first ? 1 : ra0 + rb0) * I * J * (last ? 1 : ra1 + rb1);
  if (n <= 0) return hipSuccess;
  const int g = grid_for(n, 256, 8192);
  if (dtype == kF64)
    k_mpo_add<double><<<g, 256, 0, s>>>((const double*)A, (const double*)B, (double*)C, ra0, rb0,
                                        I, J, ra1, rb1, first, last);
  else
    k_mpo_add<float><<<g, 256, 0, s>>>((const float*)A, (const float*)B, (float*)C, ra0, rb0, I, J,
                                       ra1, rb1, first, last);
  return hipGetLastError();
}

hipError_t launch_check_finite(const void* in, int dtype, int64_t n, int* flag, hipStream_t s) {
  const int g = grid_for(n, 256, 4096);
  if (dtype == 0)
    k_check_finite<double><<<g, 256, 0, s>>>((const double*)in, n, flag);
  else
    k_check_finite<float><<<g, 256, 0, s>>>((const float*)in, n, flag);
  return hipGetLastError();
}

hipError_t launch_omega(const MpoDesc* mpos, const CoreDesc* cores, int batch, uint64_t seed,
                        double* om, int64_t max_len, hipStream_t s) {
  dim3 grid(grid_for(max_len, 256, 1024), batch);
  k_omega<<<grid, 256, 0, s>>>(mpos, cores, seed, om);
  return hipGetLastError();
}

hipError_t launch_load_omega(const MpoDesc* mpos, const CoreDesc* cores, int batch,
                             const double* om, int* xr, void* X, int dtype, int max_d,
                             int64_t max_len, int* err, hipStream_t s) {
  dim3 grid(max_d, batch);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_load_omega<T><<<grid, 256, 0, s>>>(mpos, cores, om, xr, (T*)X, err);
  });
  return hipGetLastError();
}

hipError_t launch_contract(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                           int ncores, const int* xr, int* pr, const void* A, const void* X,
                           void* Z, int dtype, int op, int64_t max_out, int* err, int threads,
                           int gcap, hipStream_t s) {
  // threads per block and the cap on blocks per core come from the plan or the
  // autotuner; the grid-stride loop makes every shape cover all outputs
  dim3 grid(grid_for(max_out, threads, gcap), ncores);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    if (op == 0)
      k_contract<T, 0><<<grid, threads, 0, s>>>(mpos, cores, core_mpo, xr, pr, (const T*)A,
                                                 (const T*)X, (T*)Z, err);
    else
      k_contract<T, 1><<<grid, threads, 0, s>>>(mpos, cores, core_mpo, xr, pr, (const T*)A,
                                                 (const T*)X, (T*)Z, err);
  });
  return hipGetLastError();
}

hipError_t launch_copy_y0(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                          int ncores, const int* pr, const void* Z, void* Y0, int dtype,
                          int64_t max_out, hipStream_t s) {
  dim3 grid(grid_for(max_out, 256, 256), ncores);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_copy_y0<T><<<grid, 256, 0, s>>>(mpos, cores, core_mpo, pr, (const T*)Z, (T*)Y0);
  });
  return hipGetLastError();
}

hipError_t launch_form_u(const MpoDesc* mpos, const CoreDesc* cores, const int* core_mpo,
                         int ncores, const int* xr, const void* X, int dtype, const double* outs,
                         double* U, int64_t max_out, int* err, hipStream_t s) {
  dim3 grid(grid_for(max_out, 256, 256), ncores);
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_form_u<T><<<grid, 256, 0, s>>>(mpos, cores, core_mpo, xr, (const T*)X, outs, U, err);
  });
  return hipGetLastError();
}

}  // namespace tnr
