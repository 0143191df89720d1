// device_types.hpp -- plain structs uploaded to the device by the runtime and
// read by the kernels (all 8-byte aligned, no pointers: offsets only).
#pragma once
#include <cstdint>

namespace stc {

struct UpdTaskD {     // one output tile and its run of contributions
  int64_t c_off;
  int64_t part_off;     // this task's partial slots (nsplit - 1 of them)
  int64_t in_part_off;  // partial slots of an earlier split task to fold in
  int32_t c_rows, diag;
  int32_t c_begin, c_end;
  int32_t nsplit;       // K-step stream split across nsplit work-groups
  int32_t in_npart;     // number of partial slots to fold in
};

struct ContribD {     // C -= A(rows via rowmap) * B(rows via colmap)^T
  int64_t a_off, b_off;
  int32_t a_rows, b_rows;
  int32_t rowmap, colmap;  // offsets into the map pool, -1 = identity
};

struct TrsmTaskD {
  int64_t x_off, l_off;
  int32_t rows, k;
};

// C (+)= alpha * sum_q A(r, q) B(q, j), operands read through index maps
// (offsets into the map pool, -1 = identity; a map entry -1 = structural
// zero).  Buffers: 0 factor store, 1 selected-inverse store, 2 inverses of
// the diagonal tiles, 3 products L_mk inv(L_kk).
enum { CA_NORMAL = 0, CA_TRANS = 1, CA_SYM = 2 };

struct ConTermD {
  int64_t a_off, b_off;
  int32_t a_buf, a_mode, a_rmap, a_qmap;
  int32_t b_buf, b_qmap, K, pad;
};

struct ConTaskD {
  int64_t c_off;
  int32_t c_buf, c_rows, ncols, diag;
  int32_t t_begin, t_end;
  int32_t beta;     // 1: accumulate into C, 0: overwrite
  int32_t pad;
  double alpha;
};

struct FoldItemD {     // one 64 x 64 block of a split reverse-mode task's output and its partial slots
  int64_t c_off, slot_off;
  int32_t c_buf, c_rows, ncols, diag;
  int32_t nslots;
  int32_t bx, by;      // block row and column
  int32_t pad;
};

struct TileD {        // off-diagonal tile as the solve sees it
  int64_t off;        // store offset
  int64_t roff;       // offset of its active rows in the row pool
  int32_t m, k, cnt;
  int32_t imap;       // offset in the map pool of block row -> stored row (-1 absent), -1 if full
};

}  // namespace stc
