// Host-side construction of the device layouts of a sparse matrix (no HIP:
// this unit also builds for the CPU alone, where the tests run it under the
// address and undefined-behaviour sanitizers).
//
// Two layouts hold the same matrix and give the same products:
//   CSR   -- the caller's rows cut into row blocks of at most kRowsPerBlock rows
//            whose entries fit a per-block budget (a longer row gets a block of
//            its own); optionally each block's entries stored in column order
//            (gather order) with each one's place in the block's row order, the
//            columns as 16-bit offsets from the block's first row, and the
//            block's rows listed longest first;
//   SELL  -- sliced ELLPACK: slices of 64 * rpl consecutive rows, a slice's
//            entries stored column by column (entry j of the row in slice lane q
//            at off[slice] + j * 64 * rpl + q), each row in its CSR order, padded
//            to the slice's longest row; padding has column -1 (32-bit) or
//            kPad16 (16-bit offsets column - row) and value 0.
// A batch of independent systems is first padded, system by system, to a
// multiple of 512 rows with empty rows.
#pragma once

#include <cstdint>
#include <vector>

namespace psl {

constexpr int kRowsPerBlock = 256;   // rows of a CSR row block (one workgroup)
constexpr int kSliceRows = 64;       // rows of a slice per row of a lane (one wavefront)
constexpr short kPad16 = -32768;     // SELL padding in 16-bit offsets
constexpr int kBatchAlign = 512;     // rows each system of a batch is padded to

// Row blocks: ascending first rows, blk[0] = 0, blk.back() = n.  No block
// crosses one of the ascending row indices in `cuts`.
std::vector<int> row_blocks(int64_t n, const int64_t *rowptr, int budget,
                            const std::vector<int64_t> &cuts);

// Slots of the sliced layout with `rpl` rows per lane (each slice padded to its
// longest row).
int64_t sell_slots(int64_t n, const int64_t *rowptr, int rpl);

// Whether a typical block's columns span more than `span` (the median over the
// blocks whose entries fit the budget): the automatic gather-order rule.
bool csr_wide_blocks(const std::vector<int> &blk, const int64_t *rowptr, const int32_t *col,
                     int64_t budget, int64_t span);

struct CsrLayout {
  std::vector<int> blk;              // [nblk+1] first row of each row block
  std::vector<int> rowptr;           // [n+1] int32 row pointers
  std::vector<unsigned char> rord;   // [n] each block's rows, longest first (or empty)
  std::vector<unsigned short> pos;   // [nnz] gather order: an entry's place in its block's
                                     // row order (0 in a block of one longer row, whose
                                     // entries keep row order); empty in row order
  const int32_t *col = nullptr;      // [nnz] columns in storage order: the caller's array,
  const double *val = nullptr;       // or col_sorted / val_sorted in gather order
  std::vector<int32_t> col_sorted;
  std::vector<double> val_sorted;
  std::vector<short> col16;          // [nnz] column - first row of its block (or empty)
  int index_bits = 32;
};

// Build the CSR layout.  budget: entries a block may hold; order_rows: list
// each block's rows longest first; gather_sort: store blocks whose entries fit
// the budget in column order (a block holding one longer row keeps row order);
// want16: use 16-bit offsets if every entry's offset fits.
void build_csr(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
               int budget, const std::vector<int64_t> &cuts, bool order_rows, bool gather_sort,
               bool want16, CsrLayout &out);

struct SellLayout {
  int rpl = 1;
  int64_t nslice = 0, slots = 0;
  std::vector<int> off;              // [nslice+1] first slot of each slice
  std::vector<int32_t> col;          // [slots] column or -1 (32-bit layout)
  std::vector<short> col16;          // [slots] column - row or kPad16 (16-bit layout)
  std::vector<double> val;           // [slots]
  int index_bits = 32;
};

// Build the sliced layout (slots must not reach 2^31).  want16: 16-bit offsets
// if every entry lies within 32767 of its row.
void build_sell(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int rpl,
                bool want16, SellLayout &out);

struct BatchPadding {
  int nsys = 1;
  int64_t n_orig = 0, n_pad = 0;
  std::vector<int64_t> pstart;       // [nsys+1] first padded row of each system
  std::vector<int> row_map;          // [n_orig] padded row of each caller row
  std::vector<int> chunk_sys;        // [n_pad/256] system of each 256-row chunk
  std::vector<int> first_blk;        // [nsys+1] first 512-row chunk of each system
  std::vector<int> sys_end;          // [nsys] end of each system's own rows (before its padding)
  std::vector<int64_t> rowptr;       // [n_pad+1] the padded matrix
  std::vector<int32_t> col;          // [nnz] its columns (values keep the caller's order)
};

// Pad each system of a block-diagonal matrix (rows sys_ptr[k] .. sys_ptr[k+1]-1,
// columns within the same range) to a multiple of kBatchAlign rows.  Returns
// false if the padded size reaches 2^31 - 1 rows.
bool pad_batch(int32_t nsys, const int64_t *sys_ptr, int64_t n, const int64_t *rowptr,
               const int32_t *col, BatchPadding &out);

}  // namespace psl
