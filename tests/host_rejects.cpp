// Host-only checks of the C ABI's argument validation, built against the
// library compiled with AddressSanitizer and UndefinedBehaviorSanitizer on its
// host code: every call below must be refused before any device call, with
// the status the header documents, and without a sanitizer report.
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "tnrsvd.h"

static int fails = 0;

#define EXPECT(call, want)                                                          \
  do {                                                                              \
    const int got_ = (int)(call);                                                   \
    if (got_ != (want)) {                                                           \
      std::printf("FAIL line %d: %s = %d, want %d (%s)\n", __LINE__, #call, got_, \
                  (int)(want), tnrsvd_last_error());                                \
      ++fails;                                                                      \
    }                                                                               \
  } while (0)

struct Mpo {
  int64_t rank[8], rows[8], cols[8];
  const void* core[8];
  tnrsvd_mpo m;
  Mpo(int d, const int64_t* r, const int64_t* I, const int64_t* J, int dtype = TNRSVD_F64) {
    for (int k = 0; k <= d; ++k) rank[k] = r[k];
    for (int k = 0; k < d; ++k) {
      rows[k] = I[k];
      cols[k] = J[k];
      core[k] = (const void*)8;   // never dereferenced: every case fails first
    }
    m.d = d;
    m.rank = rank;
    m.rows = rows;
    m.cols = cols;
    m.core = core;
    m.dtype = dtype;
  }
};

int main() {
  const int64_t r121[] = {1, 2, 1}, r122[] = {1, 2, 2}, r101[] = {1, 0, 1}, r221[] = {2, 2, 1};
  const int64_t n22[] = {2, 2}, n23[] = {2, 3};
  Mpo good(2, r121, n22, n22);
  tnrsvd_opts o{};
  o.k = 2;
  o.p = 2;
  o.seed = 1;
  tnrsvd_t h = nullptr;

  // tnrsvd_create
  EXPECT(tnrsvd_create(nullptr, 1, &good.m, &o), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_create(&h, 0, &good.m, &o), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_create(&h, 1, nullptr, &o), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_create(&h, 1, &good.m, nullptr), TNRSVD_E_INVALID);
  {
    tnrsvd_opts b = o;
    b.orientation = 5;
    EXPECT(tnrsvd_create(&h, 1, &good.m, &b), TNRSVD_E_INVALID);
    b = o;
    b.sketch_rank = 257;
    EXPECT(tnrsvd_create(&h, 1, &good.m, &b), TNRSVD_E_INVALID);
    b = o;
    b.k = 0;
    EXPECT(tnrsvd_create(&h, 1, &good.m, &b), TNRSVD_E_INVALID);
    b = o;
    b.round_tol = -1.0;
    EXPECT(tnrsvd_create(&h, 1, &good.m, &b), TNRSVD_E_INVALID);
  }
  {
    Mpo bad(2, r221, n22, n22);
    EXPECT(tnrsvd_create(&h, 1, &bad.m, &o), TNRSVD_E_SHAPE);
    Mpo zero(2, r101, n22, n22);
    EXPECT(tnrsvd_create(&h, 1, &zero.m, &o), TNRSVD_E_SHAPE);
  }
  // calls on a NULL handle
  EXPECT(tnrsvd_run(nullptr, nullptr), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_autotune_sweeps(nullptr, 1, nullptr), TNRSVD_E_INVALID);
  {
    const int c[2] = {129, 1};
    EXPECT(tnrsvd_set_sweep_config(nullptr, c), TNRSVD_E_INVALID);
  }
  EXPECT(tnrsvd_destroy(nullptr), TNRSVD_OK);

  // tnrsvd_round_mpo
  tnrsvd_rounded_t rr = nullptr;
  EXPECT(tnrsvd_round_mpo(&good.m, 1e-3, 0, nullptr, nullptr), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_round_mpo(nullptr, 1e-3, 0, nullptr, &rr), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_round_mpo(&good.m, -1.0, 0, nullptr, &rr), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_round_mpo(&good.m, 1e-3, -1, nullptr, &rr), TNRSVD_E_INVALID);
  {
    Mpo bad(2, r221, n22, n22);
    EXPECT(tnrsvd_round_mpo(&bad.m, 1e-3, 0, nullptr, &rr), TNRSVD_E_SHAPE);
  }

  // tnrsvd_complex_embed and tnrsvd_solve_complex
  void* outs[2] = {(void*)8, (void*)8};
  EXPECT(tnrsvd_complex_embed(nullptr, outs, nullptr), TNRSVD_E_INVALID);
  EXPECT(tnrsvd_complex_embed(&good.m, nullptr, nullptr), TNRSVD_E_INVALID);
  {
    Mpo bad(2, r122, n22, n22);
    EXPECT(tnrsvd_complex_embed(&bad.m, outs, nullptr), TNRSVD_E_SHAPE);
    double sig[4];
    EXPECT(tnrsvd_solve_complex(nullptr, &o, sig), TNRSVD_E_INVALID);
    EXPECT(tnrsvd_solve_complex(&good.m, &o, nullptr), TNRSVD_E_INVALID);
    EXPECT(tnrsvd_solve_complex(&bad.m, &o, sig), TNRSVD_E_SHAPE);
    tnrsvd_opts b = o;
    b.k = 0;
    EXPECT(tnrsvd_solve_complex(&good.m, &b, sig), TNRSVD_E_INVALID);
    Mpo bf(2, r121, n22, n22, TNRSVD_BF16);
    EXPECT(tnrsvd_solve_complex(&bf.m, &o, sig), TNRSVD_E_INVALID);
  }

  // tnrsvd_mpo_add
  {
    const int64_t r131[] = {1, 3, 1};
    Mpo other(2, r131, n22, n22), modes(2, r131, n23, n22), f32(2, r131, n22, n22, TNRSVD_F32);
    EXPECT(tnrsvd_mpo_add(nullptr, &other.m, outs, nullptr), TNRSVD_E_INVALID);
    EXPECT(tnrsvd_mpo_add(&good.m, &other.m, nullptr, nullptr), TNRSVD_E_INVALID);
    EXPECT(tnrsvd_mpo_add(&good.m, &f32.m, outs, nullptr), TNRSVD_E_INVALID);
    EXPECT(tnrsvd_mpo_add(&good.m, &modes.m, outs, nullptr), TNRSVD_E_SHAPE);
  }

  // sizes whose products overflow 64 bits are refused, not wrapped
  {
    const int64_t huge[] = {int64_t(2147483647), 2}, big[] = {int64_t(1) << 40, 2};
    Mpo h1(2, r121, huge, huge), b1(2, r121, big, big), b2(2, r121, big, big);
    EXPECT(tnrsvd_round_mpo(&h1.m, 1e-3, 0, nullptr, &rr), TNRSVD_E_SHAPE);
    EXPECT(tnrsvd_mpo_add(&b1.m, &b2.m, outs, nullptr), TNRSVD_E_SHAPE);
    const int64_t e31[] = {int64_t(1) << 31, 2};
    Mpo e1(2, r121, e31, e31);
    EXPECT(tnrsvd_complex_embed(&e1.m, outs, nullptr), TNRSVD_E_SHAPE);
  }

  // tnrsvd_sparse_to_mpo: null rank output, bad d
  {
    int64_t nb = 0;
    const int64_t rows[] = {4, 2}, cols[] = {4, 2};
    EXPECT(tnrsvd_sparse_to_mpo(2, rows, cols, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr),
           TNRSVD_E_INVALID);
    EXPECT(tnrsvd_sparse_to_mpo(0, rows, cols, 0, nullptr, nullptr, nullptr, &nb, nullptr, nullptr),
           TNRSVD_E_SHAPE);
  }

  std::printf("%s (%d failures)\n", fails ? "FAILED" : "all host rejections as documented", fails);
  return fails ? 1 : 0;
}
