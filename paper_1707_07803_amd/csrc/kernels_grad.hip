// Gradient of L = sum_{j<k} w_j u_j^T A v_j with respect to A's cores, with
// the computed singular triplets (u_j, v_j) held fixed (not part of the
// paper; at fixed U and V this is the derivative of the output singular
// values, sum_j w_j u_j v_j^T, written into MPO form).
//
// k_grad_env: one workgroup per MPO.  Left environments
//   E_0 = 1,  E_{i+1}[r', a', s'] = sum E_i[r,a,s] U_i[r,x,r'] A_i[a,x,y,a'] V_i[s,y,s']
// are formed left to right and kept; the right environment starts on the K
// legs as F[j, 0, j] = w_j (j < k) and moves right to left, and at core i
//   dL/dA_i[a,x,y,a'] = sum E_i[r,a,s] U_i[r,x,r'] V_i[s,y,s'] F_{i+1}[r',a',s'].
// Every contraction runs as three two-operand steps through workspace, one
// thread per output element.  U, V, E, F are FP64; A is read in its storage
// type and widened.
//
// k_merge_pair_dT / k_merge_pair_dC: adjoint of merging two cores
//   N[a, X I1 + x, Y J1 + y, b] = sum_r T[a,x,y,r] C[r,X,Y,b]
// (the merged mode index is little-endian, as in eq. (1)).
#include "tnrsvd_internal.h"

namespace tnr {

namespace {

constexpr int GT = 512;

template <typename TA>
__global__ __launch_bounds__(GT) void k_grad_env(const MpoDesc* mpos, const CoreDesc* cores,
                                                  const GradMpo* gm, const int64_t* eoff,
                                                  const int* xr, const int* vr,
                                                  const TA* __restrict__ A,
                                                  const double* __restrict__ U,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ w, int k,
                                                  double* __restrict__ ws,
                                                  double* __restrict__ G, int* err) {
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const MpoDesc md = mpos[b];
  const GradMpo g = gm[b];
  const int d = md.d, K = md.K;
  const double* wb = w + (int64_t)b * k;
  double* T1 = ws + g.tmp0;
  double* T2 = T1 + g.tmpcap;
  double* S2 = T2 + g.tmpcap;
  double* Fa = S2 + g.tmpcap;
  double* Fb = Fa + g.tmpcap;
  // ranks of U (xr) and V (vr) at bond i; the K legs of the last cores are cut to k
  auto ru = [&](int i) { return i == d ? k : xr[md.r0 + i]; };
  auto rv = [&](int i) { return i == d ? k : vr[md.r0 + i]; };
  for (int i = 0; i <= d; ++i) {   // capacity guard (block uniform)
    const int cap = i == d ? K : (i == 0 ? 1 : cores[md.c0 + i].xcap);
    if (ru(i) < 1 || ru(i) > cap || rv(i) < 1 || rv(i) > cap) {
      if (tid == 0) atomicOr(err, 4);
      return;
    }
  }
  // ---- left environments ------------------------------------------------
  if (tid == 0) ws[eoff[md.c0]] = 1.0;
  __syncthreads();
  for (int i = 0; i + 1 < d; ++i) {
    const CoreDesc cd = cores[md.c0 + i];
    const int I = cd.I, J = cd.J, R = cd.RA, R2 = cd.RA2;
    const int r = ru(i), r2 = ru(i + 1), s = rv(i), s2 = rv(i + 1);
    const double* E = ws + eoff[md.c0 + i];
    const double* Ui = U + cd.u_off;
    const double* Vi = V + cd.u_off;
    const TA* Ai = A + cd.a_off;
    double* En = ws + eoff[md.c0 + i + 1];
    // T1[a,x,s,r'] = sum_r E[r,a,s] U[r,x,r']
    const int n1 = R * I * s * r2;
    for (int o = tid; o < n1; o += GT) {
      const int rp = o % r2, si = (o / r2) % s, x = (o / (r2 * s)) % I, a = o / (r2 * s * I);
      double acc = 0.0;
      for (int ri = 0; ri < r; ++ri)
        acc += E[(ri * R + a) * s + si] * Ui[(ri * I + x) * r2 + rp];
      T1[o] = acc;
    }
    __syncthreads();
    // T2[a',y,s,r'] = sum_{a,x} T1[a,x,s,r'] A[a,x,y,a']
    const int n2 = R2 * J * s * r2;
    for (int o = tid; o < n2; o += GT) {
      const int rp = o % r2, si = (o / r2) % s, y = (o / (r2 * s)) % J, ap = o / (r2 * s * J);
      double acc = 0.0;
      for (int a = 0; a < R; ++a)
        for (int x = 0; x < I; ++x)
          acc += T1[((a * I + x) * s + si) * r2 + rp] *
                 (double)Ai[((a * I + x) * J + y) * R2 + ap];
      T2[o] = acc;
    }
    __syncthreads();
    // E'[r',a',s'] = sum_{s,y} T2[a',y,s,r'] V[s,y,s']
    const int n3 = r2 * R2 * s2;
    for (int o = tid; o < n3; o += GT) {
      const int sp = o % s2, ap = (o / s2) % R2, rp = o / (s2 * R2);
      double acc = 0.0;
      for (int si = 0; si < s; ++si)
        for (int y = 0; y < J; ++y)
          acc += T2[((ap * J + y) * s + si) * r2 + rp] * Vi[(si * J + y) * s2 + sp];
      En[o] = acc;
    }
    __syncthreads();
  }
  // ---- right environments and the core gradients --------------------------
  {
    const int n0 = k * k;
    for (int o = tid; o < n0; o += GT) Fa[o] = (o / k == o % k) ? wb[o % k] : 0.0;
  }
  __syncthreads();
  double* F = Fa;
  double* Fn = Fb;
  for (int i = d - 1; i >= 0; --i) {
    const CoreDesc cd = cores[md.c0 + i];
    const int I = cd.I, J = cd.J, R = cd.RA, R2 = cd.RA2;
    const int r = ru(i), r2 = ru(i + 1), s = rv(i), s2 = rv(i + 1);
    const int su = i == d - 1 ? K : r2;   // stored right extent of U_i / V_i
    const int sv = i == d - 1 ? K : s2;
    const double* E = ws + eoff[md.c0 + i];
    const double* Ui = U + cd.u_off;
    const double* Vi = V + cd.u_off;
    const TA* Ai = A + cd.a_off;
    double* Gi = G + cd.a_off;
    // S1[r',a',s,y] = sum_{s'} V[s,y,s'] F[r',a',s']          (in T2)
    double* S1 = T2;
    const int n1 = r2 * R2 * s * J;
    for (int o = tid; o < n1; o += GT) {
      const int y = o % J, si = (o / J) % s, ap = (o / (J * s)) % R2, rp = o / (J * s * R2);
      double acc = 0.0;
      for (int sp = 0; sp < s2; ++sp)
        acc += Vi[(si * J + y) * sv + sp] * F[(rp * R2 + ap) * s2 + sp];
      S1[o] = acc;
    }
    // T1[a,x,s,r'] = sum_r E[r,a,s] U[r,x,r']
    const int n2 = R * I * s * r2;
    for (int o = tid; o < n2; o += GT) {
      const int rp = o % r2, si = (o / r2) % s, x = (o / (r2 * s)) % I, a = o / (r2 * s * I);
      double acc = 0.0;
      for (int ri = 0; ri < r; ++ri)
        acc += E[(ri * R + a) * s + si] * Ui[(ri * I + x) * su + rp];
      T1[o] = acc;
    }
    __syncthreads();
    // dA_i[a,x,y,a'] = sum_{s,r'} T1[a,x,s,r'] S1[r',a',s,y]
    const int n3 = R * I * J * R2;
    for (int o = tid; o < n3; o += GT) {
      const int ap = o % R2, y = (o / R2) % J, x = (o / (R2 * J)) % I, a = o / (R2 * J * I);
      double acc = 0.0;
      for (int si = 0; si < s; ++si)
        for (int rp = 0; rp < r2; ++rp)
          acc += T1[((a * I + x) * s + si) * r2 + rp] * S1[((rp * R2 + ap) * s + si) * J + y];
      Gi[o] = acc;
    }
    if (i == 0) break;
    // S2[r',a,x,s] = sum_{a',y} A[a,x,y,a'] S1[r',a',s,y]
    const int n4 = r2 * R * I * s;
    for (int o = tid; o < n4; o += GT) {
      const int si = o % s, x = (o / s) % I, a = (o / (s * I)) % R, rp = o / (s * I * R);
      double acc = 0.0;
      for (int ap = 0; ap < R2; ++ap)
        for (int y = 0; y < J; ++y)
          acc += (double)Ai[((a * I + x) * J + y) * R2 + ap] *
                 S1[((rp * R2 + ap) * s + si) * J + y];
      S2[o] = acc;
    }
    __syncthreads();
    // F_i[r,a,s] = sum_{r',x} U[r,x,r'] S2[r',a,x,s]
    const int n5 = r * R * s;
    for (int o = tid; o < n5; o += GT) {
      const int si = o % s, a = (o / s) % R, ri = o / (s * R);
      double acc = 0.0;
      for (int rp = 0; rp < r2; ++rp)
        for (int x = 0; x < I; ++x)
          acc += Ui[(ri * I + x) * su + rp] * S2[((rp * R + a) * I + x) * s + si];
      Fn[o] = acc;
    }
    __syncthreads();
    double* t = F;
    F = Fn;
    Fn = t;
  }
}

// dT[a,x,y,r] = sum_{X,Y,b} dN[a, X I1 + x, Y J1 + y, b] C[r,X,Y,b]
__global__ void k_merge_pair_dT(const double* __restrict__ dN, const double* __restrict__ C,
                                double* __restrict__ dT, int a_, int I1, int J1, int r_, int I2,
                                int J2, int b_) {
  const int64_t n = (int64_t)a_ * I1 * J1 * r_;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(o % r_), y = (int)((o / r_) % J1), x = (int)((o / ((int64_t)r_ * J1)) % I1);
    const int a = (int)(o / ((int64_t)r_ * J1 * I1));
    double acc = 0.0;
    for (int X = 0; X < I2; ++X)
      for (int Y = 0; Y < J2; ++Y)
        for (int b = 0; b < b_; ++b)
          acc += dN[(((int64_t)a * I2 * I1 + X * I1 + x) * (J2 * J1) + Y * J1 + y) * b_ + b] *
                 C[(((int64_t)r * I2 + X) * J2 + Y) * b_ + b];
    dT[o] = acc;
  }
}

// dC[r,X,Y,b] = sum_{a,x,y} dN[a, X I1 + x, Y J1 + y, b] T[a,x,y,r]
__global__ void k_merge_pair_dC(const double* __restrict__ dN, const double* __restrict__ T,
                                double* __restrict__ dC, int a_, int I1, int J1, int r_, int I2,
                                int J2, int b_) {
  const int64_t n = (int64_t)r_ * I2 * J2 * b_;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(o % b_), Y = (int)((o / b_) % J2), X = (int)((o / ((int64_t)b_ * J2)) % I2);
    const int r = (int)(o / ((int64_t)b_ * J2 * I2));
    double acc = 0.0;
    for (int a = 0; a < a_; ++a)
      for (int x = 0; x < I1; ++x)
        for (int y = 0; y < J1; ++y)
          acc += dN[(((int64_t)a * I2 * I1 + X * I1 + x) * (J2 * J1) + Y * J1 + y) * b_ + b] *
                 T[(((int64_t)a * I1 + x) * J1 + y) * r_ + r];
    dC[o] = acc;
  }
}

int grid_of(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t launch_grad_env(const MpoDesc* mpos, const CoreDesc* cores, const GradMpo* gm,
                           const int64_t* eoff, int batch, const int* xr, const int* vr,
                           const void* A, int dtype, const double* U, const double* V,
                           const double* w, int k, double* ws, double* G, int* err,
                           hipStream_t s) {
  by_dtype(dtype, [&](auto* t) {
    using T = elem_t<decltype(t)>;
    k_grad_env<T><<<batch, GT, 0, s>>>(mpos, cores, gm, eoff, xr, vr, (const T*)A, U, V, w, k,
                                       ws, G, err);
  });
  return hipGetLastError();
}

hipError_t launch_merge_pair_bwd(const double* T, const double* C, const double* dN, double* dT,
                                 double* dC, int a, int I1, int J1, int r, int I2, int J2, int b,
                                 hipStream_t s) {
  k_merge_pair_dT<<<grid_of((int64_t)a * I1 * J1 * r), 256, 0, s>>>(dN, C, dT, a, I1, J1, r, I2,
                                                                    J2, b);
  k_merge_pair_dC<<<grid_of((int64_t)r * I2 * J2 * b), 256, 0, s>>>(dN, T, dC, a, I1, J1, r, I2,
                                                                    J2, b);
  return hipGetLastError();
}

}  // namespace tnr
