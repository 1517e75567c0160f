// Round trips of the host layout builders (paper_2108_10591_amd/csrc/layout.cpp):
// every layout built from a CSR matrix is decoded here, from the layout's
// description alone, back into rows of (column, value) pairs that must equal the
// input, and the structural rules each layout promises are checked.  Built and
// run on the CPU under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py; exits non-zero with a message on the first failure.
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "layout.hpp"

namespace {

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

uint64_t g_state = 88172645463325252ull;
uint64_t next_u64() {  // xorshift64
  g_state ^= g_state << 13;
  g_state ^= g_state >> 7;
  g_state ^= g_state << 17;
  return g_state;
}
int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

[[noreturn]] void fail(const std::string &what) {
  std::fprintf(stderr, "layout check failed: %s\n", what.c_str());
  std::exit(1);
}

// rows of given lengths, columns within [row - band, row + band] clipped to [0, n)
Csr random_csr(const std::vector<int64_t> &len, int64_t band) {
  Csr A;
  A.n = (int64_t)len.size();
  A.rowptr.assign((size_t)A.n + 1, 0);
  for (int64_t r = 0; r < A.n; ++r) A.rowptr[(size_t)r + 1] = A.rowptr[(size_t)r] + len[(size_t)r];
  for (int64_t r = 0; r < A.n; ++r)
    for (int64_t k = 0; k < len[(size_t)r]; ++k) {
      const int64_t lo = std::max<int64_t>(0, r - band), hi = std::min<int64_t>(A.n - 1, r + band);
      A.col.push_back((int32_t)uniform(lo, hi));
      A.val.push_back((double)uniform(-1000000, 1000000) / 1024.0);
    }
  return A;
}

Csr stencil2d(int N) {
  Csr A;
  A.n = (int64_t)N * N;
  A.rowptr.push_back(0);
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N; ++i) {
      const int r = i + N * j;
      const int nb[5] = {j > 0 ? r - N : -1, i > 0 ? r - 1 : -1, r, i < N - 1 ? r + 1 : -1,
                         j < N - 1 ? r + N : -1};
      for (int c : nb)
        if (c >= 0) {
          A.col.push_back(c);
          A.val.push_back(c == r ? 4.0 : -1.0 - 0.001 * c);
        }
      A.rowptr.push_back((int64_t)A.col.size());
    }
  return A;
}

void check_csr(const Csr &A, int budget, const std::vector<int64_t> &cuts, bool order_rows,
               bool gsort, bool want16, const std::string &name) {
  psl::CsrLayout L;
  psl::build_csr(A.n, A.rowptr.data(), A.col.data(), A.val.data(), budget, cuts, order_rows, gsort,
                 want16, L);
  const std::string tag = name + " budget " + std::to_string(budget) + (order_rows ? " ordered" : "") +
                          (gsort ? " gather" : "") + (want16 ? " want16" : "");
  const int nblk = (int)L.blk.size() - 1;
  if (nblk < 0 || L.blk.front() != 0 || L.blk.back() != A.n) fail(tag + ": block bounds");
  for (int b = 0; b < nblk; ++b) {
    const int r0 = L.blk[(size_t)b], r1 = L.blk[(size_t)b + 1];
    if (r1 <= r0 || r1 - r0 > psl::kRowsPerBlock) fail(tag + ": block rows");
    const int64_t nz = A.rowptr[(size_t)r1] - A.rowptr[(size_t)r0];
    if (nz > budget && r1 - r0 != 1) fail(tag + ": block over budget holds several rows");
    for (int64_t c : cuts)
      if (c > r0 && c < r1) fail(tag + ": block crosses a system start");
  }
  for (int64_t r = 0; r <= A.n; ++r)
    if (L.rowptr[(size_t)r] != A.rowptr[(size_t)r]) fail(tag + ": row pointer");
  if (order_rows) {
    if ((int64_t)L.rord.size() != A.n) fail(tag + ": row order size");
    for (int b = 0; b < nblk; ++b) {
      const int r0 = L.blk[(size_t)b], r1 = L.blk[(size_t)b + 1];
      std::vector<char> seen((size_t)(r1 - r0), 0);
      int64_t prev = INT64_MAX;
      for (int i = r0; i < r1; ++i) {
        const int li = L.rord[(size_t)i];
        if (li >= r1 - r0 || seen[(size_t)li]) fail(tag + ": row order is not a permutation");
        seen[(size_t)li] = 1;
        const int64_t len = A.rowptr[(size_t)(r0 + li) + 1] - A.rowptr[(size_t)(r0 + li)];
        if (len > prev) fail(tag + ": rows not longest first");
        prev = len;
      }
    }
  } else if (!L.rord.empty()) {
    fail(tag + ": unexpected row order");
  }
  const bool is16 = L.index_bits == 16;
  if (is16 && !want16) fail(tag + ": 16-bit offsets not asked for");
  // decode each block back to row order
  for (int b = 0; b < nblk; ++b) {
    const int r0 = L.blk[(size_t)b];
    const int64_t k0 = A.rowptr[(size_t)r0], k1 = A.rowptr[(size_t)L.blk[(size_t)b + 1]];
    const bool fits = k1 - k0 <= budget;
    std::vector<char> seen((size_t)(k1 - k0), 0);
    int32_t prevc = INT32_MIN;
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t c = is16 ? (int64_t)r0 + L.col16[(size_t)k] : (int64_t)L.col[k];
      if (is16 && c != L.col[k]) fail(tag + ": 16-bit offset does not decode to the column");
      int64_t place = k;
      if (gsort) {
        if ((int64_t)L.pos.size() != A.rowptr[(size_t)A.n]) fail(tag + ": gather positions size");
        place = fits ? k0 + L.pos[(size_t)k] : k;
        if (fits && L.col[k] < prevc) fail(tag + ": block not in column order");
        prevc = L.col[k];
      }
      if (place < k0 || place >= k1 || seen[(size_t)(place - k0)]) fail(tag + ": positions not a permutation");
      seen[(size_t)(place - k0)] = 1;
      if (c != A.col[(size_t)place] || L.val[k] != A.val[(size_t)place]) fail(tag + ": entry differs");
    }
  }
}

void check_sell(const Csr &A, int rpl, bool want16, const std::string &name) {
  psl::SellLayout S;
  psl::build_sell(A.n, A.rowptr.data(), A.col.data(), A.val.data(), rpl, want16, S);
  const std::string tag = name + " sell rpl " + std::to_string(rpl) + (want16 ? " want16" : "");
  const int64_t SH = (int64_t)psl::kSliceRows * rpl;
  if (S.nslice != (A.n + SH - 1) / SH || (int64_t)S.off.size() != S.nslice + 1 || S.off[0] != 0)
    fail(tag + ": slices");
  if (S.slots != psl::sell_slots(A.n, A.rowptr.data(), rpl)) fail(tag + ": slot count");
  const bool is16 = S.index_bits == 16;
  if ((int64_t)(is16 ? S.col16.size() : S.col.size()) != S.slots || (int64_t)S.val.size() != S.slots)
    fail(tag + ": array sizes");
  std::vector<char> used((size_t)S.slots, 0);
  for (int64_t sl = 0; sl < S.nslice; ++sl) {
    const int64_t width = (S.off[(size_t)sl + 1] - S.off[(size_t)sl]) / SH;
    if ((S.off[(size_t)sl + 1] - S.off[(size_t)sl]) % SH) fail(tag + ": slice size");
    for (int64_t q = 0; q < SH; ++q) {
      const int64_t r = sl * SH + q;
      const int64_t len = r < A.n ? A.rowptr[(size_t)r + 1] - A.rowptr[(size_t)r] : 0;
      if (len > width) fail(tag + ": row longer than its slice");
      for (int64_t j = 0; j < width; ++j) {
        const size_t slot = (size_t)(S.off[(size_t)sl] + j * SH + q);
        used[slot] = 1;
        if (j < len) {
          const int64_t k = A.rowptr[(size_t)r] + j;
          const int64_t c = is16 ? r + S.col16[slot] : (int64_t)S.col[slot];
          if (is16 && S.col16[slot] == psl::kPad16) fail(tag + ": entry marked as padding");
          if (c != A.col[(size_t)k] || S.val[slot] != A.val[(size_t)k]) fail(tag + ": entry differs");
        } else {
          if (is16 ? S.col16[slot] != psl::kPad16 : S.col[slot] != -1) fail(tag + ": padding column");
          if (S.val[slot] != 0.0) fail(tag + ": padding value");
        }
      }
    }
  }
  for (char u : used)
    if (!u) fail(tag + ": slot outside every row");
}

void check_batch(const std::vector<int64_t> &sizes, const std::string &name) {
  std::vector<int64_t> sys_ptr(1, 0);
  Csr A;
  A.rowptr.push_back(0);
  for (int64_t m : sizes) {
    const int64_t base = sys_ptr.back();
    for (int64_t r = 0; r < m; ++r) {
      const int64_t len = uniform(0, 6);
      for (int64_t k = 0; k < len; ++k) {
        A.col.push_back((int32_t)(base + uniform(0, m - 1)));
        A.val.push_back((double)uniform(-99, 99));
      }
      A.rowptr.push_back((int64_t)A.col.size());
    }
    sys_ptr.push_back(base + m);
  }
  A.n = sys_ptr.back();
  psl::BatchPadding P;
  if (!psl::pad_batch((int32_t)sizes.size(), sys_ptr.data(), A.n, A.rowptr.data(), A.col.data(), P))
    fail(name + ": padding refused");
  const int nsys = (int)sizes.size();
  if (P.n_pad % psl::kBatchAlign || P.pstart[(size_t)nsys] != P.n_pad) fail(name + ": padded size");
  for (int k = 0; k < nsys; ++k) {
    const int64_t p0 = P.pstart[(size_t)k], p1 = P.pstart[(size_t)k + 1];
    if (p0 % psl::kBatchAlign || p1 - p0 < sizes[(size_t)k] || p1 - p0 >= sizes[(size_t)k] + psl::kBatchAlign)
      fail(name + ": system padding");
    if (P.first_blk[(size_t)k] * (int64_t)psl::kBatchAlign != p0) fail(name + ": first 512-row chunk");
    if (P.sys_end[(size_t)k] != p0 + sizes[(size_t)k]) fail(name + ": end of the system's own rows");
    for (int64_t c = p0 / 256; c < p1 / 256; ++c)
      if (P.chunk_sys[(size_t)c] != k) fail(name + ": chunk owner");
    const int64_t shift = p0 - sys_ptr[(size_t)k];
    for (int64_t r = sys_ptr[(size_t)k]; r < sys_ptr[(size_t)k + 1]; ++r) {
      const int64_t pr = P.row_map[(size_t)r];
      if (pr != r + shift) fail(name + ": row map");
      const int64_t len = A.rowptr[(size_t)r + 1] - A.rowptr[(size_t)r];
      if (P.rowptr[(size_t)pr + 1] - P.rowptr[(size_t)pr] != len) fail(name + ": padded row length");
      for (int64_t j = 0; j < len; ++j) {
        const int64_t pc = P.col[(size_t)(P.rowptr[(size_t)pr] + j)];
        if (pc != A.col[(size_t)(A.rowptr[(size_t)r] + j)] + shift || pc < p0 || pc >= p1)
          fail(name + ": padded column");
      }
    }
    for (int64_t pr = p0 + sizes[(size_t)k]; pr < p1; ++pr)
      if (P.rowptr[(size_t)pr + 1] != P.rowptr[(size_t)pr]) fail(name + ": padding row not empty");
  }
  if ((int64_t)P.chunk_sys.size() != P.n_pad / 256) fail(name + ": chunk map size");
  // the padded matrix through both layouts, blocks cut at every system start
  Csr Q;
  Q.n = P.n_pad;
  Q.rowptr = P.rowptr;
  Q.col.assign(P.col.begin(), P.col.begin() + (std::ptrdiff_t)A.col.size());
  Q.val = A.val;
  check_csr(Q, 2048, std::vector<int64_t>(P.pstart.begin() + 1, P.pstart.end()), false, false, true,
            name + " padded");
  check_sell(Q, 1, true, name + " padded");
}

}  // namespace

int main() {
  // uneven rows with empty rows, rows longer than a block's budget, unsorted and
  // repeated columns
  for (int64_t band : {50, 5000, 40000}) {
    std::vector<int64_t> len;
    for (int r = 0; r < 6000; ++r) {
      const int64_t u = uniform(0, 99);
      len.push_back(u < 8 ? 0 : (u < 12 ? uniform(300, 5000) : uniform(1, 60)));
    }
    const Csr A = random_csr(len, band);
    for (int budget : {1024, 2048, 4096})
      for (int ord = 0; ord <= 1; ++ord)
        for (int gs = 0; gs <= 1; ++gs)
          for (int w16 = 0; w16 <= 1; ++w16)
            check_csr(A, budget, {}, ord, gs, w16, "uneven band " + std::to_string(band));
    check_sell(A, 1, true, "uneven band " + std::to_string(band));
    check_sell(A, 2, false, "uneven band " + std::to_string(band));
  }
  // 16-bit limits: offsets of exactly +-32767 fit, +-32768 do not
  for (int64_t d : {32767, 32768}) {
    Csr A;
    A.n = 70000;
    A.rowptr.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) {
      A.col.push_back((int32_t)r);
      A.val.push_back(1.0);
      if (r == 39936) {
        A.col.push_back((int32_t)(r - d));
        A.val.push_back(-0.5);
      }
      if (r == 768) {
        A.col.push_back((int32_t)(r + d));
        A.val.push_back(-0.25);
      }
      A.rowptr.push_back((int64_t)A.col.size());
    }
    psl::SellLayout S;
    psl::build_sell(A.n, A.rowptr.data(), A.col.data(), A.val.data(), 1, true, S);
    if ((S.index_bits == 16) != (d == 32767)) fail("sliced 16-bit limit at " + std::to_string(d));
    check_sell(A, 1, true, "offset " + std::to_string(d));
    psl::CsrLayout L;
    psl::build_csr(A.n, A.rowptr.data(), A.col.data(), A.val.data(), 1024, {}, false, false, true, L);
    // rows 768 and 39936 start their blocks (256 rows each): their far entries lie d
    // from the block's first row
    if (L.blk[3] != 768 || L.blk[156] != 39936) fail("CSR blocks of the 16-bit limit case");
    if ((L.index_bits == 16) != (d == 32767)) fail("CSR 16-bit limit at " + std::to_string(d));
    check_csr(A, 1024, {}, false, false, true, "offset " + std::to_string(d));
    check_csr(A, 1024, {}, false, true, true, "offset " + std::to_string(d));
  }
  // a stencil, one-row systems, an empty matrix row
  const Csr St = stencil2d(100);
  for (int rpl = 1; rpl <= 2; ++rpl) check_sell(St, rpl, true, "stencil");
  check_csr(St, 1024, {}, false, true, true, "stencil");
  Csr One;
  One.n = 1;
  One.rowptr = {0, 1};
  One.col = {0};
  One.val = {2.0};
  check_csr(One, 1024, {}, true, true, true, "one row");
  check_sell(One, 1, true, "one row");
  Csr Empty;
  Empty.n = 3;
  Empty.rowptr = {0, 0, 0, 0};
  check_csr(Empty, 1024, {}, true, true, true, "empty rows");
  check_sell(Empty, 2, true, "empty rows");
  // uneven batches
  check_batch({1, 511, 512, 513, 1000, 3}, "batch");
  check_batch({4096}, "batch of one");
  std::printf("layout round trips: ok\n");
  return 0;
}
