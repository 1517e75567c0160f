// Host-side construction of the device layouts (see layout.hpp).
#include "layout.hpp"

#include <algorithm>
#include <climits>

namespace psl {

std::vector<int> row_blocks(int64_t n, const int64_t *rowptr, int budget,
                            const std::vector<int64_t> &cuts) {
  std::vector<int> blk;
  blk.push_back(0);
  int64_t r = 0;
  size_t c = 0;
  while (r < n) {
    const int64_t start = r;
    while (c < cuts.size() && cuts[c] <= start) ++c;
    const int64_t limit = c < cuts.size() ? std::min<int64_t>(n, cuts[c]) : n;
    int64_t nz = 0;
    while (r < limit && r - start < kRowsPerBlock) {
      const int64_t len = rowptr[r + 1] - rowptr[r];
      if (nz + len > budget) break;
      nz += len;
      ++r;
    }
    if (r == start) ++r;  // one row longer than the budget: a block of its own
    blk.push_back((int)r);
  }
  return blk;
}

int64_t sell_slots(int64_t n, const int64_t *rowptr, int rpl) {
  const int64_t SH = (int64_t)kSliceRows * rpl;
  int64_t slots = 0;
  for (int64_t r0 = 0; r0 < n; r0 += SH) {
    int64_t w = 0;
    for (int64_t r = r0; r < std::min<int64_t>(n, r0 + SH); ++r)
      w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
    slots += w * SH;
  }
  return slots;
}

bool csr_wide_blocks(const std::vector<int> &blk, const int64_t *rowptr, const int32_t *col,
                     int64_t budget, int64_t span) {
  std::vector<int64_t> spans;
  for (size_t b = 0; b + 1 < blk.size(); ++b) {
    const int64_t k0 = rowptr[blk[b]], k1 = rowptr[blk[b + 1]];
    if (k1 <= k0 || k1 - k0 > budget) continue;
    int32_t cmin = col[k0], cmax = col[k0];
    for (int64_t k = k0; k < k1; ++k) {
      cmin = std::min(cmin, col[k]);
      cmax = std::max(cmax, col[k]);
    }
    spans.push_back((int64_t)cmax - cmin + 1);
  }
  if (spans.empty()) return false;
  std::nth_element(spans.begin(), spans.begin() + spans.size() / 2, spans.end());
  return spans[spans.size() / 2] > span;
}

void build_csr(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
               int budget, const std::vector<int64_t> &cuts, bool order_rows, bool gather_sort,
               bool want16, CsrLayout &out) {
  const int64_t nnz = rowptr[n];
  out.blk = row_blocks(n, rowptr, budget, cuts);
  const int nblk = (int)out.blk.size() - 1;
  out.rowptr.resize((size_t)n + 1);
  for (int64_t i = 0; i <= n; ++i) out.rowptr[(size_t)i] = (int)rowptr[i];
  out.rord.clear();
  if (order_rows) {
    out.rord.resize((size_t)n);
    std::vector<int> loc;
    for (int b = 0; b < nblk; ++b) {
      const int64_t r0 = out.blk[b];
      loc.resize((size_t)(out.blk[b + 1] - r0));
      for (size_t i = 0; i < loc.size(); ++i) loc[i] = (int)i;
      std::stable_sort(loc.begin(), loc.end(), [&](int a, int c) {
        return rowptr[r0 + a + 1] - rowptr[r0 + a] > rowptr[r0 + c + 1] - rowptr[r0 + c];
      });
      for (size_t i = 0; i < loc.size(); ++i) out.rord[(size_t)r0 + i] = (unsigned char)loc[i];
    }
  }
  out.pos.clear();
  out.col_sorted.clear();
  out.val_sorted.clear();
  out.col = col;
  out.val = val;
  if (gather_sort && nnz > 0) {
    out.pos.assign((size_t)nnz, 0);
    out.col_sorted.resize((size_t)nnz);
    out.val_sorted.resize((size_t)nnz);
    std::vector<int> loc;
    for (int b = 0; b < nblk; ++b) {
      const int64_t k0 = rowptr[out.blk[b]], k1 = rowptr[out.blk[b + 1]];
      const bool fits = k1 - k0 <= budget;  // else one longer row: row order
      loc.resize((size_t)(k1 - k0));
      for (size_t i = 0; i < loc.size(); ++i) loc[i] = (int)i;
      if (fits)
        std::stable_sort(loc.begin(), loc.end(),
                         [&](int a, int c) { return col[k0 + a] < col[k0 + c]; });
      for (size_t i = 0; i < loc.size(); ++i) {
        out.pos[(size_t)k0 + i] = fits ? (unsigned short)loc[i] : (unsigned short)0;
        out.col_sorted[(size_t)k0 + i] = col[k0 + loc[i]];
        out.val_sorted[(size_t)k0 + i] = val[k0 + loc[i]];
      }
    }
    out.col = out.col_sorted.data();
    out.val = out.val_sorted.data();
  }
  // 16-bit offsets from each block's first row when every entry fits
  bool fits16 = want16;
  for (int b = 0; b < nblk && fits16; ++b)
    for (int64_t k = rowptr[out.blk[b]]; k < rowptr[out.blk[b + 1]]; ++k)
      if ((int64_t)out.col[k] - out.blk[b] > 32767 || (int64_t)out.blk[b] - out.col[k] > 32767) {
        fits16 = false;
        break;
      }
  out.index_bits = fits16 ? 16 : 32;
  out.col16.clear();
  if (fits16) {
    out.col16.resize((size_t)nnz);
    for (int b = 0; b < nblk; ++b)
      for (int64_t k = rowptr[out.blk[b]]; k < rowptr[out.blk[b + 1]]; ++k)
        out.col16[(size_t)k] = (short)(out.col[k] - out.blk[b]);
  }
}

void build_sell(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int rpl,
                bool want16, SellLayout &out) {
  const int64_t SH = (int64_t)kSliceRows * rpl;
  out.rpl = rpl;
  out.nslice = (n + SH - 1) / SH;
  out.off.assign((size_t)out.nslice + 1, 0);
  for (int64_t sl = 0; sl < out.nslice; ++sl) {
    int64_t w = 0;
    for (int64_t r = sl * SH; r < std::min<int64_t>(n, (sl + 1) * SH); ++r)
      w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
    out.off[(size_t)sl + 1] = (int)(out.off[(size_t)sl] + w * SH);
  }
  out.slots = out.off[(size_t)out.nslice];
  bool fits16 = want16;
  for (int64_t r = 0; r < n && fits16; ++r)
    for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
      if ((int64_t)col[k] - r > 32767 || r - (int64_t)col[k] > 32767) {
        fits16 = false;
        break;
      }
  out.index_bits = fits16 ? 16 : 32;
  out.col.clear();
  out.col16.clear();
  if (fits16) out.col16.assign((size_t)out.slots, kPad16);
  else out.col.assign((size_t)out.slots, -1);
  out.val.assign((size_t)out.slots, 0.0);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t base = out.off[(size_t)(r / SH)] + r % SH;
    for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
      const size_t slot = (size_t)(base + (k - rowptr[r]) * SH);
      if (fits16) out.col16[slot] = (short)(col[k] - r);
      else out.col[slot] = col[k];
      out.val[slot] = val[k];
    }
  }
}

bool pad_batch(int32_t nsys, const int64_t *sys_ptr, int64_t n, const int64_t *rowptr,
               const int32_t *col, BatchPadding &out) {
  out.nsys = nsys;
  out.n_orig = n;
  out.pstart.assign((size_t)nsys + 1, 0);
  for (int32_t k = 0; k < nsys; ++k)
    out.pstart[(size_t)k + 1] =
        out.pstart[(size_t)k] + (sys_ptr[k + 1] - sys_ptr[k] + kBatchAlign - 1) / kBatchAlign * kBatchAlign;
  const int64_t np = out.pstart[(size_t)nsys];
  if (np >= INT32_MAX - 1) return false;
  out.n_pad = np;
  const int64_t nnz = rowptr[n];
  out.rowptr.assign((size_t)np + 1, 0);
  out.col.resize((size_t)std::max<int64_t>(nnz, 1));
  out.row_map.resize((size_t)n);
  out.chunk_sys.resize((size_t)(np / 256));
  out.first_blk.resize((size_t)nsys + 1);
  out.sys_end.resize((size_t)nsys);
  for (int32_t k = 0; k < nsys; ++k) {
    const int64_t shift = out.pstart[(size_t)k] - sys_ptr[k];
    for (int64_t r = sys_ptr[k]; r < sys_ptr[k + 1]; ++r) {
      out.row_map[(size_t)r] = (int)(r + shift);
      out.rowptr[(size_t)(r + shift + 1)] = rowptr[r + 1] - rowptr[r];
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
        out.col[(size_t)e] = (int32_t)(col[e] + shift);
    }
    for (int64_t c = out.pstart[(size_t)k] / 256; c < out.pstart[(size_t)k + 1] / 256; ++c)
      out.chunk_sys[(size_t)c] = k;
    out.first_blk[(size_t)k] = (int)(out.pstart[(size_t)k] / kBatchAlign);
    out.sys_end[(size_t)k] = (int)(out.pstart[(size_t)k] + sys_ptr[k + 1] - sys_ptr[k]);
  }
  out.first_blk[(size_t)nsys] = (int)(np / kBatchAlign);
  for (int64_t r = 0; r < np; ++r) out.rowptr[(size_t)r + 1] += out.rowptr[(size_t)r];
  return true;
}

}  // namespace psl
