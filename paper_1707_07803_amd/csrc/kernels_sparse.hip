// Sparse matrix to MPO (Algorithm 4.1, Sec. 4.1) on the GPU.
//
// The matrix is given by its nonzero entries (COO, device).  Its partition
// into I_1 x J_1 blocks follows the Kronecker ordering of eq. (1): entry
// (i, j) lies in block (i / I_1, j / J_1), whose position at level k >= 2 is
// the k-th mixed-radix digit of the block index.  Every nonzero block X is the
// rank-1 MPO (X, E^(2), ..., E^(d)) and the sum of these terms is one MPO of
// rank N = number of nonzero blocks (the rank lemma of Sec. 4.2):
//   core 1   (1, I_1, J_1, N):   [0, x, y, t] = X_t[x, y]
//   core k   (N, I_k, J_k, N):   [t, i_k(t), j_k(t), t] = 1       (1 < k < d)
//   core d   (N, I_d, J_d, 1):   [t, i_d(t), j_d(t), 0] = 1
// Blocks are numbered in increasing order of key = block_row * (J / J_1) +
// block_col: keys are radix-sorted, block heads flagged and numbered by a
// prefix sum, and every entry and every unit entry is then scattered in
// parallel into the zero-filled cores.  Duplicate entries add (FP64 global
// atomics, so the order of their sum is not fixed).
#include <hipcub/hipcub.hpp>

#include "tnrsvd_internal.h"

namespace tnr {

namespace {

// Sort key of entry e, or the sentinel `none` (the number of block positions)
// for an explicit zero, which sorts after every block and forms none; the
// entry's position goes to idx.  An index outside the matrix raises bad[0].
__global__ void k_block_keys(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                             const double* __restrict__ val, int64_t nnz, int64_t M, int64_t Nc,
                             int64_t I1, int64_t J1, int64_t nbc, uint64_t none,
                             uint64_t* __restrict__ key, int64_t* __restrict__ idx,
                             int* __restrict__ bad) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = row[e], j = col[e];
    const bool in = i >= 0 && i < M && j >= 0 && j < Nc;
    if (!in) bad[0] = 1;
    key[e] = (in && val[e] != 0.0) ? (uint64_t)((i / I1) * nbc + j / J1) : none;
    idx[e] = e;
  }
}

// flag[e] = 1 where a new block starts in the sorted keys
__global__ void k_heads(const uint64_t* __restrict__ key, int64_t nnz, uint64_t none,
                        int* __restrict__ flag) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    flag[e] = (key[e] != none && (e == 0 || key[e] != key[e - 1])) ? 1 : 0;
}

// key of every block (scan = inclusive prefix sum of the heads) and the block
// count
__global__ void k_block_ids(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                            const int* __restrict__ scan, int64_t nnz, uint64_t* __restrict__ bkey,
                            int* __restrict__ nblk) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (flag[e]) bkey[scan[e] - 1] = key[e];
    if (e == nnz - 1) nblk[0] = scan[e];
  }
}

// X_t[x, y] += value for every nonzero entry, into core 1 (1, I1, J1, N)
__global__ void k_scatter_blocks(const uint64_t* __restrict__ key, const int64_t* __restrict__ idx,
                                 const int* __restrict__ scan, const int64_t* __restrict__ row,
                                 const int64_t* __restrict__ col, const double* __restrict__ val,
                                 int64_t nnz, uint64_t none, int64_t I1, int64_t J1, int64_t N,
                                 double* __restrict__ core1) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (key[e] == none) continue;
    const int64_t src = idx[e];
    const int64_t t = scan[e] - 1;
    const int64_t x = row[src] % I1, y = col[src] % J1;
    atomicAdd(core1 + (x * J1 + y) * N + t, val[src]);
  }
}

// unit entry of core k >= 2 for every block t: digit k of its row and column
// block index, digit = (index / div) mod dim
__global__ void k_unit_entries(const uint64_t* __restrict__ bkey, int64_t N, int64_t nbc,
                               int64_t rdiv, int64_t cdiv, int64_t Ik, int64_t Jk, int last,
                               double* __restrict__ core) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t br = (int64_t)(bkey[t] / (uint64_t)nbc), bc = (int64_t)(bkey[t] % (uint64_t)nbc);
    const int64_t ik = (br / rdiv) % Ik, jk = (bc / cdiv) % Jk;
    if (last)
      core[(t * Ik + ik) * Jk + jk] = 1.0;
    else
      core[((t * Ik + ik) * Jk + jk) * N + t] = 1.0;
  }
}

// p[0..n) = 0, 16-byte stores over the aligned body
__global__ void k_zero(double* __restrict__ p, int64_t n) {
  const int64_t head = (int64_t)(((16 - ((uintptr_t)p & 15)) & 15) / sizeof(double));
  const int64_t h = head < n ? head : n;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid < h) p[tid] = 0.0;
  double2* q = reinterpret_cast<double2*>(p + h);
  const int64_t n2 = (n - h) / 2;
  for (int64_t e = tid; e < n2; e += stride) q[e] = double2{0.0, 0.0};
  if ((n - h) & 1) {
    if (tid == 0) p[n - 1] = 0.0;
  }
}

int grid_n(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Counts the nonzero blocks (*nblocks) and, when cores is not null and the
// count equals `expect` (the rank the cores were sized for), fills the d
// caller-allocated FP64 cores.  Shapes are validated by the caller; indices
// outside the matrix are reported through *bad_index and then no core is
// written.  One scratch allocation per call; the stream is synchronised to
// read the block count back.
hipError_t sparse_to_mpo(int d, const int64_t* I, const int64_t* J, int64_t nnz,
                         const int64_t* row, const int64_t* col, const double* val,
                         int64_t expect, int64_t* nblocks, double* const* cores, int* bad_index,
                         hipStream_t s) {
  int64_t M = 1, Nc = 1, nbc = 1;
  for (int k = 0; k < d; ++k) {
    M *= I[k];
    Nc *= J[k];
  }
  nbc = Nc / J[0];
  const uint64_t none = (uint64_t)(M / I[0]) * (uint64_t)nbc;   // number of block positions
  int end_bit = 1;
  while (end_bit < 64 && (none >> end_bit) != 0) ++end_bit;
  const int n = (int)(nnz > 0 ? nnz : 1);

  size_t tmp_sort = 0, tmp_scan = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_sort, (uint64_t*)nullptr,
                                                    (uint64_t*)nullptr, (int64_t*)nullptr,
                                                    (int64_t*)nullptr, n, 0, end_bit, s);
  if (e == hipSuccess)
    e = hipcub::DeviceScan::InclusiveSum(nullptr, tmp_scan, (int*)nullptr, (int*)nullptr, n, s);
  if (e != hipSuccess) return e;
  // scratch: key, skey, bkey (u64), idx, sidx (i64), flag, scan (int), nblk+bad (int), tmp
  const size_t o_key = 0, o_skey = o_key + align_up(8 * (size_t)n),
               o_bkey = o_skey + align_up(8 * (size_t)n), o_idx = o_bkey + align_up(8 * (size_t)n),
               o_sidx = o_idx + align_up(8 * (size_t)n), o_flag = o_sidx + align_up(8 * (size_t)n),
               o_scan = o_flag + align_up(4 * (size_t)n), o_cnt = o_scan + align_up(4 * (size_t)n),
               o_tmp = o_cnt + 256,
               total = o_tmp + align_up(tmp_sort > tmp_scan ? tmp_sort : tmp_scan);
  char* base = nullptr;
  e = hipMalloc((void**)&base, total);
  if (e != hipSuccess) return e;
  uint64_t* key = (uint64_t*)(base + o_key);
  uint64_t* skey = (uint64_t*)(base + o_skey);
  uint64_t* bkey = (uint64_t*)(base + o_bkey);
  int64_t* idx = (int64_t*)(base + o_idx);
  int64_t* sidx = (int64_t*)(base + o_sidx);
  int* flag = (int*)(base + o_flag);
  int* scan = (int*)(base + o_scan);
  int* cnt = (int*)(base + o_cnt);   // cnt[0] blocks, cnt[1] bad index
  void* tmp = base + o_tmp;
  size_t tmp_bytes = total - o_tmp;

  int hc[2] = {0, 0};
  e = hipMemsetAsync(cnt, 0, 2 * sizeof(int), s);
  if (e == hipSuccess && nnz > 0) {
    k_block_keys<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, M, Nc, I[0], J[0], nbc, none, key,
                                             idx, cnt + 1);
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, skey, idx, sidx, (int)nnz, 0,
                                           end_bit, s);
    if (e == hipSuccess) {
      k_heads<<<grid_n(nnz), 256, 0, s>>>(skey, nnz, none, flag);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, flag, scan, (int)nnz, s);
    if (e == hipSuccess) {
      k_block_ids<<<grid_n(nnz), 256, 0, s>>>(skey, flag, scan, nnz, bkey, cnt);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hc, cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const int N = hc[0];
  *bad_index = hc[1];
  // the zero matrix is one zero rank-1 term
  const int64_t Nr = N > 0 ? N : 1;
  if (e == hipSuccess) *nblocks = Nr;
  if (e == hipSuccess && cores && !hc[1] && Nr == expect) {
    for (int k = 0; k < d && e == hipSuccess; ++k) {
      const int64_t a = k == 0 ? 1 : Nr, b = (k == d - 1) ? 1 : Nr;
      const int64_t len = a * I[k] * J[k] * b;
      k_zero<<<grid_n(len / 2 + 1), 256, 0, s>>>(cores[k], len);
      e = hipGetLastError();
    }
    if (e == hipSuccess && N > 0) {
      k_scatter_blocks<<<grid_n(nnz), 256, 0, s>>>(skey, sidx, scan, row, col, val, nnz, none,
                                                   I[0], J[0], Nr, cores[0]);
      e = hipGetLastError();
      int64_t rdiv = 1, cdiv = 1;
      for (int k = 1; k < d && e == hipSuccess; ++k) {
        k_unit_entries<<<grid_n(N), 256, 0, s>>>(bkey, N, nbc, rdiv, cdiv, I[k], J[k],
                                                 k == d - 1, cores[k]);
        e = hipGetLastError();
        rdiv *= I[k];
        cdiv *= J[k];
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  const hipError_t ef = hipFree(base);
  return e != hipSuccess ? e : ef;
}

}  // namespace tnr
