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
// block_col.  Two ways to number them:
//   bitmap path (at most 2^28 block positions): one bit per position is set
//     for every nonzero entry, and a block's number is the count of set bits
//     before its own (word popcounts + a prefix sum), so no sort is needed;
//   sort path (larger position spaces): the keys are radix-sorted, block
//     heads flagged and numbered by a prefix sum.
// The cores are then zero-filled and every entry and every unit entry is
// scattered into them in parallel.  Duplicate entries add (FP64 global
// atomics, so the order of their sum is not fixed).  The filling kernels
// check on the device that the block count equals the rank the caller sized
// the cores for and that no index was out of range, and write nothing
// otherwise, so one call needs a single host synchronisation.
#include <hipcub/hipcub.hpp>

#include <mutex>
#include <vector>

#include "tnrsvd_internal.h"

namespace tnr {

namespace {

constexpr uint64_t kBitmapMax = uint64_t(1) << 28;   // largest position count of the bitmap path
constexpr size_t kCacheMax = size_t(256) << 20;      // largest scratch kept between calls

// One core k >= 2 (0-based k >= 1) as the unit-entry kernels see it.
struct UnitCore {
  double* p;
  int64_t Ik, Jk;
  int64_t rdiv, cdiv;   // digit k of a block row / column index = (index / div) mod dim
  int64_t last;         // core (N, Ik, Jk, 1) instead of (N, Ik, Jk, N)
};

// The filling kernels run only when the count (cnt[0], at least 1) equals the
// rank the caller sized the cores for and no index was out of range (cnt[1]).
__device__ inline bool fill_ok(const int* cnt, int64_t expect) {
  const int64_t n = cnt[0] > 0 ? cnt[0] : 1;
  return cnt[1] == 0 && n == expect;
}

__device__ inline bool in_matrix(int64_t i, int64_t j, int64_t M, int64_t Nc) {
  return i >= 0 && i < M && j >= 0 && j < Nc;
}

// the unit entry of every core k >= 2 for block t with the given key
__device__ inline void write_units(uint64_t key, int64_t t, int64_t nbc, const UnitCore* uc,
                                   int nk, int64_t N) {
  const int64_t br = (int64_t)(key / (uint64_t)nbc), bc = (int64_t)(key % (uint64_t)nbc);
  for (int k = 0; k < nk; ++k) {
    const UnitCore c = uc[k];
    const int64_t ik = (br / c.rdiv) % c.Ik, jk = (bc / c.cdiv) % c.Jk;
    const int64_t at = (t * c.Ik + ik) * c.Jk + jk;
    c.p[c.last ? at : at * N + t] = 1.0;
  }
}

// ---------------------------------------------------------------- bitmap path

// Set the bit of every nonzero entry's block; an index outside the matrix
// raises bad[0].  Neighbouring entries mostly share a block, so a wave first
// ORs the bits of lanes with the same bitmap word together and one lane sets
// them, only if they are not already set (read at device scope, past the CU's
// cache): the atomics stay few even when every entry hits a handful of words.
__global__ void k_mark(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                       const double* __restrict__ val, int64_t nnz, int64_t M, int64_t Nc,
                       int64_t I1, int64_t J1, int64_t nbc, unsigned* __restrict__ bm,
                       int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the loop bound is uniform over a wave, so every lane takes part in the shuffles
  for (int64_t wb = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); wb < nnz;
       wb += stride) {
    const int64_t e = wb + lane;
    bool has = false;
    unsigned w = 0, bit = 0;
    if (e < nnz) {
      const int64_t i = row[e], j = col[e];
      if (!in_matrix(i, j, M, Nc)) {
        bad[0] = 1;
      } else if (val[e] != 0.0) {
        const uint64_t key = (uint64_t)((i / I1) * nbc + j / J1);
        has = true;
        w = (unsigned)(key >> 5);
        bit = 1u << (key & 31);
      }
    }
    uint64_t pending = __ballot(has);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const unsigned lw = __shfl(w, leader);
      const bool mine = has && w == lw;
      unsigned b = mine ? bit : 0u;
      for (int off = 32; off > 0; off >>= 1) b |= __shfl_xor(b, off);
      if (lane == leader) {
        const unsigned cur = __hip_atomic_load(bm + lw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((cur & b) != b) atomicOr(bm + lw, b);
      }
      pending &= ~__ballot(mine);
    }
  }
}

__global__ void k_popc(const unsigned* __restrict__ bm, int64_t nw, int* __restrict__ pc) {
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw;
       w += (int64_t)gridDim.x * blockDim.x)
    pc[w] = __popc(bm[w]);
}

// cnt[0] = number of blocks (ws = inclusive prefix sum of the word popcounts)
__global__ void k_total(const int* __restrict__ ws, int64_t nw, int* __restrict__ cnt) {
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[0] = ws[nw - 1];
}

// block number of a marked key: set bits before it
__device__ inline int64_t block_of(const unsigned* bm, const int* ws, uint64_t key) {
  const unsigned word = bm[key >> 5];
  return ws[key >> 5] - __popc(word) + __popc(word & ((1u << (key & 31)) - 1u));
}

// X_t[x, y] += value for every nonzero entry, into core 1 (1, I1, J1, N)
__global__ void k_scatter_bm(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                             const double* __restrict__ val, int64_t nnz, int64_t I1, int64_t J1,
                             int64_t nbc, const unsigned* __restrict__ bm,
                             const int* __restrict__ ws, const int* __restrict__ cnt,
                             int64_t expect, double* __restrict__ core1) {
  if (!fill_ok(cnt, expect)) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = val[e];
    if (v == 0.0) continue;
    const int64_t i = row[e], j = col[e];
    const int64_t t = block_of(bm, ws, (uint64_t)((i / I1) * nbc + j / J1));
    atomicAdd(core1 + ((i % I1) * J1 + j % J1) * expect + t, v);
  }
}

// unit entries of cores k >= 2: one thread per block position, working where its bit is set
__global__ void k_units_bm(const unsigned* __restrict__ bm, const int* __restrict__ ws,
                           int64_t nw, int64_t nbc, const UnitCore* __restrict__ uc, int nk,
                           const int* __restrict__ cnt, int64_t expect) {
  if (!fill_ok(cnt, expect)) return;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nw * 32;
       g += (int64_t)gridDim.x * blockDim.x) {
    const unsigned word = bm[g >> 5];
    const unsigned b = (unsigned)(g & 31);
    if (!((word >> b) & 1u)) continue;
    const int64_t t = ws[g >> 5] - __popc(word) + __popc(word & ((1u << b) - 1u));
    write_units((uint64_t)g, t, nbc, uc, nk, expect);
  }
}

// ------------------------------------------------------------------ sort path

// Sort key of entry e, or the sentinel `none` (the number of block positions)
// for an explicit zero or an index outside the matrix (which raises bad[0]);
// either sorts after every block and forms none.  The entry's position goes to
// idx.
__global__ void k_block_keys(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                             const double* __restrict__ val, int64_t nnz, int64_t M, int64_t Nc,
                             int64_t I1, int64_t J1, int64_t nbc, uint64_t none,
                             uint64_t* __restrict__ key, int64_t* __restrict__ idx,
                             int* __restrict__ bad) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = row[e], j = col[e];
    const bool in = in_matrix(i, j, M, Nc);
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

// key of every block (scan = inclusive prefix sum of the heads) and the count
__global__ void k_block_ids(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                            const int* __restrict__ scan, int64_t nnz, uint64_t* __restrict__ bkey,
                            int* __restrict__ cnt) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (flag[e]) bkey[scan[e] - 1] = key[e];
    if (e == nnz - 1) cnt[0] = scan[e];
  }
}

__global__ void k_scatter_sorted(const uint64_t* __restrict__ key, const int64_t* __restrict__ idx,
                                 const int* __restrict__ scan, const int64_t* __restrict__ row,
                                 const int64_t* __restrict__ col, const double* __restrict__ val,
                                 int64_t nnz, uint64_t none, int64_t I1, int64_t J1,
                                 const int* __restrict__ cnt, int64_t expect,
                                 double* __restrict__ core1) {
  if (!fill_ok(cnt, expect)) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (key[e] == none) continue;
    const int64_t src = idx[e];
    const int64_t t = scan[e] - 1;
    const int64_t x = row[src] % I1, y = col[src] % J1;
    atomicAdd(core1 + (x * J1 + y) * expect + t, val[src]);
  }
}

__global__ void k_units_sorted(const uint64_t* __restrict__ bkey, int64_t nbc,
                               const UnitCore* __restrict__ uc, int nk, const int* __restrict__ cnt,
                               int64_t expect) {
  if (!fill_ok(cnt, expect)) return;
  const int64_t N = cnt[0];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x)
    write_units(bkey[t], t, nbc, uc, nk, expect);
}

// ------------------------------------------------------------------- filling

// p[0..n) = 0 with 16-byte stores over the aligned body (when the fill is allowed)
__global__ void k_zero(double* __restrict__ p, int64_t n, const int* __restrict__ cnt,
                       int64_t expect) {
  if (!fill_ok(cnt, expect)) return;
  const int64_t head = (int64_t)(((16 - ((uintptr_t)p & 15)) & 15) / sizeof(double));
  const int64_t h = head < n ? head : n;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid < h) p[tid] = 0.0;
  double2* q = reinterpret_cast<double2*>(p + h);
  const int64_t n2 = (n - h) / 2;
  for (int64_t e = tid; e < n2; e += stride) q[e] = double2{0.0, 0.0};
  if (((n - h) & 1) && tid == 0) p[n - 1] = 0.0;
}

int grid_n(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------- rounding: block structure

// key of every block t (t = rank of its bit)
__global__ void k_block_list(const unsigned* __restrict__ bm, const int* __restrict__ ws,
                             int64_t nw, uint64_t* __restrict__ bkey) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nw * 32;
       g += (int64_t)gridDim.x * blockDim.x) {
    const unsigned word = bm[g >> 5];
    const unsigned b = (unsigned)(g & 31);
    if ((word >> b) & 1u) bkey[ws[g >> 5] - __popc(word) + __popc(word & ((1u << b) - 1u))] = g;
  }
}

// Suffix of block t from level k on: its block row and column divided by the
// products of the mode sizes of levels 2..k-1 (rdiv, cdiv), as one key over
// (rows / rdiv) x (nsc = nbc / cdiv) positions.
__device__ inline uint64_t suffix_key(uint64_t key, int64_t nbc, int64_t rdiv, int64_t cdiv,
                                      int64_t nsc) {
  const uint64_t br = key / (uint64_t)nbc, bc = key % (uint64_t)nbc;
  return (br / (uint64_t)rdiv) * (uint64_t)nsc + bc / (uint64_t)cdiv;
}

__global__ void k_suffix_mark(const uint64_t* __restrict__ bkey, int64_t N, int64_t nbc,
                              int64_t rdiv, int64_t cdiv, int64_t nsc, unsigned* __restrict__ bm) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t sk = suffix_key(bkey[t], nbc, rdiv, cdiv, nsc);
    atomicOr(bm + (sk >> 5), 1u << (sk & 31));
  }
}

// class of block t at one level = rank of its suffix's bit
__global__ void k_suffix_class(const uint64_t* __restrict__ bkey, int64_t N, int64_t nbc,
                               int64_t rdiv, int64_t cdiv, int64_t nsc,
                               const unsigned* __restrict__ bm, const int* __restrict__ ws,
                               int* __restrict__ cls) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x)
    cls[t] = (int)block_of(bm, ws, suffix_key(bkey[t], nbc, rdiv, cdiv, nsc));
}

// For class c of level k: the mode index of its unit entry in the
// orthogonalised selection core (digit k of row and column) and its class at
// level k + 1 (0 on the last level).  Every block of a class writes the same
// values.
__global__ void k_class_info(const uint64_t* __restrict__ bkey, int64_t N, int64_t nbc,
                             int64_t rdiv, int64_t cdiv, int64_t Ik, int64_t Jk,
                             const int* __restrict__ cls, const int* __restrict__ cls_next,
                             int* __restrict__ pm, int* __restrict__ nx) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t br = (int64_t)(bkey[t] / (uint64_t)nbc), bc = (int64_t)(bkey[t] % (uint64_t)nbc);
    const int c = cls ? cls[t] : (int)t;
    pm[c] = (int)(((br / rdiv) % Ik) * Jk + (bc / cdiv) % Jk);
    nx[c] = cls_next ? cls_next[t] : 0;
  }
}

// Rows of core 1 (m = (i mod I1) J1 + (j mod J1)) that hold a nonzero entry.
__global__ void k_mark_rows(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                            const double* __restrict__ val, int64_t nnz, int64_t I1, int64_t J1,
                            unsigned* __restrict__ rbm) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (val[e] == 0.0) continue;
    const uint64_t m = (uint64_t)((row[e] % I1) * J1 + col[e] % J1);
    const unsigned bit = 1u << (m & 31);
    if (!(rbm[m >> 5] & bit)) atomicOr(rbm + (m >> 5), bit);
  }
}

// row of core 1 held by each compact row (rank of its bit)
__global__ void k_row_list(const unsigned* __restrict__ rbm, const int* __restrict__ rws,
                           int64_t nw, int64_t* __restrict__ rlist) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nw * 32;
       g += (int64_t)gridDim.x * blockDim.x) {
    const unsigned word = rbm[g >> 5];
    const unsigned b = (unsigned)(g & 31);
    if ((word >> b) & 1u) rlist[rws[g >> 5] - __popc(word) + __popc(word & ((1u << b) - 1u))] = g;
  }
}

// Core 1 as row tiles for TSQR: entry (i, j) of block t adds into tile
// l = m / h, element (m mod h, t) of the h x N column-major tile, where m is
// its row of core 1, or that row's rank among the nonzero rows when rbm is
// given.
__global__ void k_scatter_tiles(const int64_t* __restrict__ row, const int64_t* __restrict__ col,
                                const double* __restrict__ val, int64_t nnz, int64_t I1, int64_t J1,
                                int64_t nbc, const unsigned* __restrict__ bm,
                                const int* __restrict__ ws, const unsigned* __restrict__ rbm,
                                const int* __restrict__ rws, int64_t h, int64_t N,
                                double* __restrict__ Pw) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = val[e];
    if (v == 0.0) continue;
    const int64_t i = row[e], j = col[e];
    const int64_t t = block_of(bm, ws, (uint64_t)((i / I1) * nbc + j / J1));
    int64_t m = (i % I1) * J1 + j % J1;
    if (rbm) m = block_of(rbm, rws, (uint64_t)m);
    atomicAdd(Pw + (m / h) * h * N + t * h + m % h, v);
  }
}

// core1[rlist[r], :] = Uc[r, :] (row-major, rho columns); other rows stay zero
__global__ void k_expand_rows(const double* __restrict__ Uc, const int64_t* __restrict__ rlist,
                              int64_t nc, int64_t rho, double* __restrict__ core1) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nc * rho;
       e += (int64_t)gridDim.x * blockDim.x)
    core1[rlist[e / rho] * rho + e % rho] = Uc[e];
}

// Scratch kept per device between calls (up to kCacheMax bytes); the mutex is
// held for a whole call, which ends with a stream synchronisation.
std::mutex g_scratch_mu;
std::vector<std::pair<char*, size_t>> g_scratch;

}  // namespace

namespace {

// Byte layout of one call's scratch (bitmap or sort path), from the shapes
// alone; the hipcub calls below only report their temporary sizes.
struct S2MLayout {
  bool bitmap;
  int64_t nw;
  int end_bit;
  size_t tmp_bytes, o_a, o_b, o_c, o_d, o_e, o_f, o_cnt, o_uc, o_tmp, total;
};

hipError_t s2m_layout(int64_t nnz, uint64_t none, int nk, S2MLayout* L, hipStream_t s) {
  L->bitmap = none <= kBitmapMax;
  const int n = (int)(nnz > 0 ? nnz : 1);
  L->nw = (int64_t)((none + 31) / 32);
  L->end_bit = 1;
  while (L->end_bit < 64 && (none >> L->end_bit) != 0) ++L->end_bit;
  const size_t uc_bytes = align_up(sizeof(UnitCore) * (size_t)(nk + 1));
  hipError_t e = hipSuccess;
  L->tmp_bytes = 0;
  if (L->bitmap) {
    // a: bitmap, b: word popcounts, c: their inclusive prefix sum
    e = hipcub::DeviceScan::InclusiveSum(nullptr, L->tmp_bytes, (int*)nullptr, (int*)nullptr,
                                         (int)L->nw, s);
    L->o_a = 0;
    L->o_b = L->o_a + align_up(4 * (size_t)L->nw);
    L->o_c = L->o_b + align_up(4 * (size_t)L->nw);
    L->o_d = L->o_e = L->o_f = L->o_c + align_up(4 * (size_t)L->nw);
  } else {
    // a: keys, b: sorted keys, c: block keys, d: positions, e: sorted positions, f: heads + scan
    size_t t_sort = 0, t_scan = 0;
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, t_sort, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (int64_t*)nullptr, (int64_t*)nullptr, n, 0, L->end_bit,
                                           s);
    if (e == hipSuccess)
      e = hipcub::DeviceScan::InclusiveSum(nullptr, t_scan, (int*)nullptr, (int*)nullptr, n, s);
    L->tmp_bytes = t_sort > t_scan ? t_sort : t_scan;
    L->o_a = 0;
    L->o_b = L->o_a + align_up(8 * (size_t)n);
    L->o_c = L->o_b + align_up(8 * (size_t)n);
    L->o_d = L->o_c + align_up(8 * (size_t)n);
    L->o_e = L->o_d + align_up(8 * (size_t)n);
    L->o_f = L->o_e + align_up(8 * (size_t)n);
  }
  L->o_cnt = (L->bitmap ? L->o_d : L->o_f + 2 * align_up(4 * (size_t)n));
  L->o_uc = L->o_cnt + 256;
  L->o_tmp = L->o_uc + uc_bytes;
  L->total = L->o_tmp + align_up(L->tmp_bytes > 0 ? L->tmp_bytes : 1);
  return e;
}

// p[0..n) = 0 (a kernel rather than a memset, so a captured stream records no
// memset node)
__global__ void k_clear_u32(unsigned* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

// The conversion proper on a scratch buffer `base` laid out by L: counts the
// blocks, fills the cores when asked, and synchronises the stream.
hipError_t s2m_run(char* base, const S2MLayout& L, int d, const int64_t* I, const int64_t* J,
                   int64_t nnz, const int64_t* row, const int64_t* col, const double* val,
                   int64_t expect, int64_t* nblocks, double* const* cores, const UnitCore* uc,
                   int nk, int* bad_index, hipStream_t s) {
  int64_t M = 1, Nc = 1;
  for (int k = 0; k < d; ++k) {
    M *= I[k];
    Nc *= J[k];
  }
  const int64_t nbc = Nc / J[0];
  const uint64_t none = (uint64_t)(M / I[0]) * (uint64_t)nbc;
  const int64_t nw = L.nw;
  const size_t tmp_bytes = L.tmp_bytes;
  int* cnt = (int*)(base + L.o_cnt);   // cnt[0] blocks, cnt[1] index outside the matrix
  UnitCore* duc = (UnitCore*)(base + L.o_uc);
  void* tmp = base + L.o_tmp;

  k_clear_u32<<<1, 64, 0, s>>>((unsigned*)cnt, 2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && nk > 0)
    e = hipMemcpyAsync(duc, uc, sizeof(UnitCore) * nk, hipMemcpyHostToDevice, s);
  if (L.bitmap) {
    unsigned* bm = (unsigned*)(base + L.o_a);
    int* pc = (int*)(base + L.o_b);
    int* ws = (int*)(base + L.o_c);
    if (e == hipSuccess) {
      k_clear_u32<<<grid_n(nw), 256, 0, s>>>(bm, nw);
      e = hipGetLastError();
    }
    if (e == hipSuccess && nnz > 0) {
      k_mark<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, M, Nc, I[0], J[0], nbc, bm, cnt + 1);
      k_popc<<<grid_n(nw), 256, 0, s>>>(bm, nw, pc);
      e = hipGetLastError();
      size_t tb = tmp_bytes;
      if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(tmp, tb, pc, ws, (int)nw, s);
      if (e == hipSuccess) {
        k_total<<<1, 64, 0, s>>>(ws, nw, cnt);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess && cores) {
      for (int k = 0; k < d && e == hipSuccess; ++k) {
        const int64_t len = (k == 0 ? 1 : expect) * I[k] * J[k] * (k == d - 1 ? 1 : expect);
        k_zero<<<grid_n(len / 2 + 1), 256, 0, s>>>(cores[k], len, cnt, expect);
        e = hipGetLastError();
      }
      if (e == hipSuccess && nnz > 0) {
        k_scatter_bm<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, I[0], J[0], nbc, bm, ws, cnt,
                                                 expect, cores[0]);
        if (nk > 0) k_units_bm<<<grid_n(nw * 32), 256, 0, s>>>(bm, ws, nw, nbc, duc, nk, cnt, expect);
        e = hipGetLastError();
      }
    }
  } else {
    const int n = (int)(nnz > 0 ? nnz : 1);
    uint64_t* key = (uint64_t*)(base + L.o_a);
    uint64_t* skey = (uint64_t*)(base + L.o_b);
    uint64_t* bkey = (uint64_t*)(base + L.o_c);
    int64_t* idx = (int64_t*)(base + L.o_d);
    int64_t* sidx = (int64_t*)(base + L.o_e);
    int* flag = (int*)(base + L.o_f);
    int* scan = (int*)(base + L.o_f + align_up(4 * (size_t)n));
    if (e == hipSuccess && nnz > 0) {
      k_block_keys<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, M, Nc, I[0], J[0], nbc, none,
                                               key, idx, cnt + 1);
      e = hipGetLastError();
      size_t tb = tmp_bytes;
      if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, skey, idx, sidx, (int)nnz, 0,
                                               L.end_bit, s);
      if (e == hipSuccess) {
        k_heads<<<grid_n(nnz), 256, 0, s>>>(skey, nnz, none, flag);
        e = hipGetLastError();
      }
      tb = tmp_bytes;
      if (e == hipSuccess)
        e = hipcub::DeviceScan::InclusiveSum(tmp, tb, flag, scan, (int)nnz, s);
      if (e == hipSuccess) {
        k_block_ids<<<grid_n(nnz), 256, 0, s>>>(skey, flag, scan, nnz, bkey, cnt);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess && cores) {
      for (int k = 0; k < d && e == hipSuccess; ++k) {
        const int64_t len = (k == 0 ? 1 : expect) * I[k] * J[k] * (k == d - 1 ? 1 : expect);
        k_zero<<<grid_n(len / 2 + 1), 256, 0, s>>>(cores[k], len, cnt, expect);
        e = hipGetLastError();
      }
      if (e == hipSuccess && nnz > 0) {
        k_scatter_sorted<<<grid_n(nnz), 256, 0, s>>>(skey, sidx, scan, row, col, val, nnz, none,
                                                     I[0], J[0], cnt, expect, cores[0]);
        if (nk > 0) k_units_sorted<<<grid_n(nnz), 256, 0, s>>>(bkey, nbc, duc, nk, cnt, expect);
        e = hipGetLastError();
      }
    }
  }
  int hc[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hc, cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    *bad_index = hc[1];
    *nblocks = hc[0] > 0 ? hc[0] : 1;   // the zero matrix is one zero rank-1 term
  }
  return e;
}

// Unit-entry table of cores 2..d (nk = d - 1 entries, or 0 without cores).
int s2m_units(int d, const int64_t* I, const int64_t* J, double* const* cores, UnitCore* uc) {
  if (!cores) return 0;
  int64_t rdiv = 1, cdiv = 1;
  for (int k = 1; k < d; ++k) {
    uc[k - 1] = UnitCore{cores[k], I[k], J[k], rdiv, cdiv, k == d - 1 ? 1 : 0};
    rdiv *= I[k];
    cdiv *= J[k];
  }
  return d - 1;
}

std::mutex g_noalloc_mu;   // held for a whole call (which ends synchronised)
char* g_noalloc_ptr[kNoAllocDevices] = {};

}  // namespace

// Scratch of sparse_to_mpo_noalloc: file-scope device memory (each GPU the
// library runs on holds its own copy until the process ends).  Host code uses
// it only through the per-device address from hipGetSymbolAddress, never by
// this name.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// Counts the nonzero blocks (*nblocks) and, when cores is not null, fills the
// d caller-allocated FP64 cores if the count equals `expect` (the rank they
// were sized for).  Shapes are validated by the caller; an index outside the
// matrix is reported through *bad_index and then no core is written.
hipError_t sparse_to_mpo(int d, const int64_t* I, const int64_t* J, int64_t nnz,
                         const int64_t* row, const int64_t* col, const double* val,
                         int64_t expect, int64_t* nblocks, double* const* cores, int* bad_index,
                         hipStream_t s) {
  int64_t M = 1, Nc = 1;
  for (int k = 0; k < d; ++k) {
    M *= I[k];
    Nc *= J[k];
  }
  const uint64_t none = (uint64_t)(M / I[0]) * (uint64_t)(Nc / J[0]);
  std::vector<UnitCore> uc(d > 1 ? d - 1 : 1);
  const int nk = s2m_units(d, I, J, cores, uc.data());
  S2MLayout L;
  hipError_t e = s2m_layout(nnz, none, nk, &L, s);
  if (e != hipSuccess) return e;

  std::lock_guard<std::mutex> lock(g_scratch_mu);
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, {nullptr, 0});
  char* base = nullptr;
  bool owned = false;
  if (L.total <= kCacheMax) {
    auto& sc = g_scratch[dev];
    if (sc.second < L.total) {
      if (sc.first) (void)hipFree(sc.first);
      sc = {nullptr, 0};
      e = hipMalloc((void**)&sc.first, L.total);
      if (e != hipSuccess) {
        sc.first = nullptr;
        return e;
      }
      sc.second = L.total;
    }
    base = sc.first;
  } else {
    e = hipMalloc((void**)&base, L.total);
    if (e != hipSuccess) return e;
    owned = true;
  }
  e = s2m_run(base, L, d, I, J, nnz, row, col, val, expect, nblocks, cores, uc.data(), nk,
              bad_index, s);
  if (owned) {
    const hipError_t ef = hipFree(base);
    if (e == hipSuccess) e = ef;
  }
  return e;
}

hipError_t sparse_to_mpo_noalloc(int d, const int64_t* I, const int64_t* J, int64_t nnz,
                                 const int64_t* row, const int64_t* col, const double* val,
                                 int64_t expect, int64_t* nblocks, double* const* cores,
                                 int* bad_index, size_t* need, hipStream_t s) {
  int64_t M = 1, Nc = 1;
  for (int k = 0; k < d; ++k) {
    M *= I[k];
    Nc *= J[k];
  }
  const uint64_t none = (uint64_t)(M / I[0]) * (uint64_t)(Nc / J[0]);
  UnitCore uc[kNoAllocMaxD];
  const int nk = s2m_units(d, I, J, cores, uc);
  S2MLayout L;
  hipError_t e = s2m_layout(nnz, none, nk, &L, s);
  if (e != hipSuccess) return e;
  *need = L.total;
  if (L.total > kNoAllocScratchBytes) return hipSuccess;   // the caller reports the limit
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocDevices) return hipErrorInvalidDevice;
  if (!g_noalloc_ptr[dev]) {
    // once per device, with that device current: its copy's address
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[dev] = (char*)p;
  }
  return s2m_run(g_noalloc_ptr[dev], L, d, I, J, nnz, row, col, val, expect, nblocks, cores, uc,
                 nk, bad_index, s);
}


namespace {


// Prefix sums of the popcounts of the nw bitmap words into ws; *count = total.
hipError_t scan_words(DevArena& A, const unsigned* bm, int* ws, int64_t nw, int* count,
                      hipStream_t s) {
  int* pc = A.get<int>(nw);
  size_t tb = 0;
  hipError_t e = A.e;
  if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(nullptr, tb, pc, ws, (int)nw, s);
  char* tmp = e == hipSuccess ? A.get<char>((int64_t)tb) : nullptr;
  if (e == hipSuccess) e = A.e;
  if (e != hipSuccess) return e;
  k_popc<<<grid_n(nw), 256, 0, s>>>(bm, nw, pc);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(tmp, tb, pc, ws, (int)nw, s);
  if (e == hipSuccess) {
    k_total<<<1, 64, 0, s>>>(ws, nw, count);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

// SVD-based rounding (Sec. 3: right-to-left orthogonalisation, then
// left-to-right truncated SVDs with delta = eps |A|_F / sqrt(d - 1), ranks
// capped at rmax when rmax > 0) of the MPO that Algorithm 4.1 builds from the
// COO matrix, without forming that MPO.  Its cores 2..d are 0/1 selection
// tensors, so their right-to-left orthogonalisation is exact relabelling: at
// level k the blocks fall into classes of equal digits k..d (suffixes), the
// orthogonalised core k has one unit entry per class (at the class's digit k
// and its class at level k + 1), and the carried factors are selections, so
// core 1 stays the matrix P of vectorised blocks.  What remains is the
// truncated SVD of P (TSQR, multi-workgroup) and of one small panel per core.
hipError_t sparse_round(int d, const int64_t* I, const int64_t* J, int64_t nnz, const int64_t* row,
                        const int64_t* col, const double* val, double eps, int rmax,
                        RoundedMpo* out, int* why, hipStream_t s) {
  *why = 0;
  int64_t M = 1, Nc = 1;
  for (int k = 0; k < d; ++k) {
    M *= I[k];
    Nc *= J[k];
  }
  const int64_t nbc = Nc / J[0], nbr = M / I[0];
  const uint64_t none = (uint64_t)nbr * (uint64_t)nbc;
  if (none > kBitmapMax) {
    *why = 2;
    return hipSuccess;
  }
  const int64_t n1 = I[0] * J[0];
  DevArena A;
  hipError_t e = hipSuccess;
  auto read_back = [&](void* host, const void* dev, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  };
  auto zero = [&](void* p, int64_t bytes) {
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, (size_t)bytes, s);
  };

  // 1. block numbering; cnt[0] blocks, cnt[1] bad index, cnt[k] classes at level k >= 2
  int* cnt = A.get<int>(d + 2);
  const int64_t nw = (int64_t)((none + 31) / 32);
  unsigned* bm = A.get<unsigned>(nw);
  int* wsb = A.get<int>(nw);
  if ((e = A.e) != hipSuccess) return e;
  zero(cnt, sizeof(int) * (d + 2));
  zero(bm, 4 * nw);
  if (e == hipSuccess && nnz > 0) {
    k_mark<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, M, Nc, I[0], J[0], nbc, bm, cnt + 1);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_words(A, bm, wsb, nw, cnt, s);
  }
  int hc[2] = {0, 0};
  read_back(hc, cnt, 2 * sizeof(int));
  if (e != hipSuccess) return e;
  if (hc[1]) {
    *why = 1;
    return hipSuccess;
  }
  const int64_t N = hc[0];
  if (N > 16384) {
    *why = 3;
    return hipSuccess;
  }
  out->ranks.assign(d + 1, 1);
  out->cores.assign(d, nullptr);
  std::vector<double*> cores(d, nullptr);
  auto finish = [&]() {
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int k = 0; k < d; ++k) {
      A.release(cores[k]);
      out->cores[k] = cores[k];
    }
    return hipSuccess;
  };
  if (N == 0 || d == 1) {
    // the zero matrix: rank-1 zero cores; a single core: the matrix itself
    for (int k = 0; k < d && e == hipSuccess; ++k) {
      cores[k] = A.get<double>(I[k] * J[k]);
      if ((e = A.e) == hipSuccess) zero(cores[k], 8 * I[k] * J[k]);
    }
    if (e == hipSuccess && N > 0) {
      k_scatter_tiles<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, I[0], J[0], nbc, bm, wsb,
                                                   nullptr, nullptr, n1, 1, cores[0]);
      e = hipGetLastError();
    }
    return finish();
  }

  // 2. block keys; classes of the suffixes at levels 2..d-1 (level 1: the blocks)
  uint64_t* bkey = A.get<uint64_t>(N);
  if ((e = A.e) != hipSuccess) return e;
  k_block_list<<<grid_n(nw * 32), 256, 0, s>>>(bm, wsb, nw, bkey);
  e = hipGetLastError();
  std::vector<int*> cls(d, nullptr), pm(d, nullptr), nx(d, nullptr);
  std::vector<int64_t> rdiv(d, 1), cdiv(d, 1);
  for (int k = 2; k < d; ++k) {
    rdiv[k] = rdiv[k - 1] * I[k - 1];
    cdiv[k] = cdiv[k - 1] * J[k - 1];
  }
  for (int k = 2; k < d && e == hipSuccess; ++k) {
    const int64_t nsc = nbc / cdiv[k], space = (nbr / rdiv[k]) * nsc;
    const int64_t snw = (space + 31) / 32;
    unsigned* sbm = A.get<unsigned>(snw);
    int* sws = A.get<int>(snw);
    cls[k] = A.get<int>(N);
    if ((e = A.e) != hipSuccess) break;
    zero(sbm, 4 * snw);
    if (e != hipSuccess) break;
    k_suffix_mark<<<grid_n(N), 256, 0, s>>>(bkey, N, nbc, rdiv[k], cdiv[k], nsc, sbm);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_words(A, sbm, sws, snw, cnt + k, s);
    if (e == hipSuccess) {
      k_suffix_class<<<grid_n(N), 256, 0, s>>>(bkey, N, nbc, rdiv[k], cdiv[k], nsc, sbm, sws,
                                               cls[k]);
      e = hipGetLastError();
    }
  }
  for (int k = 1; k < d && e == hipSuccess; ++k) {
    pm[k] = A.get<int>(N);
    nx[k] = A.get<int>(N);
    if ((e = A.e) != hipSuccess) break;
    k_class_info<<<grid_n(N), 256, 0, s>>>(bkey, N, nbc, rdiv[k], cdiv[k], I[k], J[k],
                                           k == 1 ? nullptr : cls[k],
                                           k + 1 < d ? cls[k + 1] : nullptr, pm[k], nx[k]);
    e = hipGetLastError();
  }
  // nonzero rows of core 1 (cnt[d]): the TSQR runs over those alone, since
  // zero rows add nothing to R and the left singular vectors vanish on them
  const int64_t nwr = (n1 + 31) / 32;
  unsigned* rbm = A.get<unsigned>(nwr);
  int* rws = A.get<int>(nwr);
  if (e == hipSuccess) e = A.e;
  zero(rbm, 4 * nwr);
  if (e == hipSuccess) {
    k_mark_rows<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, I[0], J[0], rbm);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = scan_words(A, rbm, rws, nwr, cnt + d, s);
  std::vector<int> hcnt(d + 2, 0);
  read_back(hcnt.data(), cnt, sizeof(int) * (d + 2));
  if (e != hipSuccess) return e;
  std::vector<int64_t> r(d, 1);   // r[k]: classes at level k (columns of the factor entering core k)
  r[1] = N;
  for (int k = 2; k < d; ++k) r[k] = hcnt[k];
  const int64_t n1c = hcnt[d];
  int64_t* rlist = A.get<int64_t>(n1c);
  if ((e = A.e) != hipSuccess) return e;
  k_row_list<<<grid_n(nwr * 32), 256, 0, s>>>(rbm, rws, nwr, rlist);
  e = hipGetLastError();

  // 3. core 1: TSQR of P (its n1c nonzero rows) in row tiles of h rows (h >= N)
  const int64_t h = N <= 960 ? 960 : (N + 63) / 64 * 64;
  const int64_t L = (n1c + h - 1) / h;
  double* Pw = A.get<double>(L * h * N);
  double* tauL = A.get<double>(L * N);
  const int64_t wssL = qr_ws_doubles(h, N);
  double* wsL = A.get<double>(L * wssL);
  std::vector<int64_t> lv;   // node counts of the tree levels above the leaves
  for (int64_t c = L; c > 1;) {
    c = (c + 1) / 2;
    lv.push_back(c);
  }
  const int64_t wssN = qr_ws_doubles(2 * N, N);
  std::vector<double*> S(lv.size()), tauS(lv.size()), wsS(lv.size());
  for (size_t j = 0; j < lv.size(); ++j) {
    S[j] = A.get<double>(lv[j] * 2 * N * N);
    tauS[j] = A.get<double>(lv[j] * N);
    wsS[j] = A.get<double>(lv[j] * wssN);
    if (A.e == hipSuccess) zero(S[j], 8 * lv[j] * 2 * N * N);
  }
  double* Rf = A.get<double>(N * N);
  if (e == hipSuccess) e = A.e;
  zero(Pw, 8 * L * h * N);
  if (e != hipSuccess) return e;
  k_scatter_tiles<<<grid_n(nnz), 256, 0, s>>>(row, col, val, nnz, I[0], J[0], nbc, bm, wsb, rbm,
                                               rws, h, N, Pw);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = launch_tsqr_leaf(Pw, (int)h, (int)N, (int)L, tauL, wsL, wssL, L == 1 ? Rf : S[0], s);
  for (size_t j = 0; j < lv.size() && e == hipSuccess; ++j)
    e = launch_tsqr_node(S[j], (int)N, (int)lv[j], tauS[j], wsS[j], wssN,
                         j + 1 < lv.size() ? S[j + 1] : Rf, s);

  // 4. SVD of the root R, rank of core 1
  double* B = A.get<double>(N * N);
  double* U = A.get<double>(N * N);
  double* nrm = A.get<double>(N);
  double* sig = A.get<double>(N);
  int* perm = A.get<int>(N);
  int* flag = A.get<int>(4);
  double* Y0 = A.get<double>(N * N);
  double* T = A.get<double>(N * N);
  int* rho_d = A.get<int>(d + 1);
  double* delta_d = A.get<double>(1);
  if (e == hipSuccess) e = A.e;
  if (e == hipSuccess)
    e = launch_root_svd(Rf, (int)N, n1c, eps, d - 1, rmax, B, U, nrm, sig, perm, flag, Y0, T,
                        rho_d + 1, delta_d, s);
  int rho1 = 0;
  read_back(&rho1, rho_d + 1, sizeof(int));
  if (e != hipSuccess) return e;
  out->ranks[1] = rho1;

  // 5. left vectors of P: the tree's reflectors top-down, then the leaves'
  // (compact rows), signs, and the rows put back in place
  cores[0] = A.get<double>(n1 * rho1);
  double* Uc = A.get<double>(n1c * rho1);
  std::vector<double*> Yl(lv.size());
  for (size_t j = 0; j < lv.size(); ++j) Yl[j] = A.get<double>(lv[j] * 2 * N * rho1);
  const int64_t nch = colsign_chunks(n1c);
  double* pv = A.get<double>(nch * rho1);
  int64_t* pi = A.get<int64_t>(nch * rho1);
  double* sgn = A.get<double>(rho1);
  if ((e = A.e) != hipSuccess) return e;
  for (int j = (int)lv.size() - 1; j >= 0 && e == hipSuccess; --j) {
    const bool top = j == (int)lv.size() - 1;
    e = launch_tsqr_apply_node(S[j], tauS[j], (int)N, rho1, (int)lv[j], top ? Y0 : Yl[j + 1],
                               top, Yl[j], s);
  }
  if (e == hipSuccess)
    e = launch_tsqr_apply_leaf(Pw, tauL, (int)h, (int)N, rho1, n1c, (int)L,
                               L == 1 ? Y0 : Yl[0], Uc, s);
  if (e == hipSuccess) e = launch_colsign(Uc, n1c, rho1, T, (int)N, pv, pi, sgn, s);
  zero(cores[0], 8 * n1 * rho1);
  if (e == hipSuccess) {
    k_expand_rows<<<grid_n(n1c * rho1), 256, 0, s>>>(Uc, rlist, n1c, rho1, cores[0]);
    e = hipGetLastError();
  }

  // 6. cores 2..d-1: one truncated SVD per core
  int64_t rp = rho1, cp = N;
  for (int k = 1; k < d - 1 && e == hipSuccess; ++k) {
    const int64_t n = I[k] * J[k], q = r[k + 1], nv = rp * n;
    const int64_t mn = nv < q ? nv : q;
    const int64_t cap = (rmax > 0 && rmax < mn) ? rmax : mn;
    double* Mw = A.get<double>(nv * q);
    double* wsk = A.get<double>(qr_ws_doubles(nv, q));
    double* tauk = A.get<double>(q);
    double* Bk = A.get<double>(nv * q);
    double* Uk = A.get<double>(mn * mn);
    double* nrmk = A.get<double>(mn);
    double* sigk = A.get<double>(mn);
    int* permk = A.get<int>(mn);
    double* sgnk = A.get<double>(cap);
    double* Yk = A.get<double>(nv * cap);
    cores[k] = A.get<double>(nv * cap);
    double* Tn = A.get<double>(cap * q);
    if ((e = A.e) != hipSuccess) break;
    e = launch_round_level(T, (int)rp, (int)cp, pm[k], nx[k], (int)n, (int)q, delta_d, rmax, Mw,
                           wsk, tauk, Bk, Uk, nrmk, sigk, permk, sgnk, flag, Yk, cores[k], Tn,
                           rho_d + k + 1, s);
    int rk = 0;
    read_back(&rk, rho_d + k + 1, sizeof(int));
    if (e != hipSuccess) break;
    out->ranks[k + 1] = rk;
    T = Tn;
    rp = rk;
    cp = q;
  }
  // 7. the last core: the carried factor placed at each class's unit entry
  if (e == hipSuccess) {
    const int64_t n = I[d - 1] * J[d - 1];
    cores[d - 1] = A.get<double>(rp * n);
    if ((e = A.e) == hipSuccess)
      e = launch_round_last(T, (int)rp, (int)cp, pm[d - 1], (int)n, cores[d - 1], s);
  }
  return finish();
}

}  // namespace tnr
