// kernels.hpp -- FP64 device kernels of the tile Cholesky for gfx950.
//
// Tile store (one per value set): diagonal tiles first, n_b x n_b row-major
// (lower triangle used; rows/columns past the matrix order of the last tile
// hold the identity), then every non-empty off-diagonal tile packed to its
// active rows, each row n_b contiguous doubles.  A packed row is a full-width
// row of L restricted to the tile's block column: the "active column stored
// at full height" of the stored transpose (Sec. 4, Sec. 4.1).
//
// Kernels of one factorization (Sec. 5.2, Algorithm 1 grouped per output
// tile):
//   k_update  C -= sum_n A_n B_n^T over all SYRK/GEMM contributions into one
//             output tile, operands gathered through the per-task maps (the
//             transpose of the paper's per-task scatter, Sec. 4.2), FP64 MFMA
//             16x16x4, accumulators in registers, one read-modify-write of C.
//   k_potrf   Cholesky of diagonal tiles, column panels staged in LDS.
//   k_trsm    X <- X L_kk^-T on the active rows of a panel tile.
// and the consumers of the resident factor: log-determinant, solve, export.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_types.hpp"

namespace stc {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// value load
// ---------------------------------------------------------------------------

__global__ void k_zero(double* __restrict__ store, int64_t n, int64_t mstride) {
  double* S = store + (int64_t)blockIdx.y * mstride;
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 2;
  for (; i + 1 < n; i += step) *reinterpret_cast<double2*>(S + i) = make_double2(0.0, 0.0);
  if (i < n) S[i] = 0.0;
}

// identity on the padded rows of the last diagonal tile
__global__ void k_pad(double* __restrict__ store, int64_t diag_off, int32_t nb, int32_t h,
                      int64_t mstride) {
  double* S = store + (int64_t)blockIdx.y * mstride;
  int32_t r = h + threadIdx.x;
  if (r < nb) S[diag_off + (int64_t)r * nb + r] = 1.0;
}

__global__ void k_value_load(const double* __restrict__ vals, const int64_t* __restrict__ vmap,
                             int64_t qnz, double* __restrict__ store, int64_t mstride) {
  const double* V = vals + (int64_t)blockIdx.y * qnz;
  double* S = store + (int64_t)blockIdx.y * mstride;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < qnz; i += step) S[vmap[i]] = V[i];
}

// One pass over the tile store per value set: block b of LBLK store doubles
// is assembled in LDS -- zeros, the identity on padded diagonal rows, the
// caller's values of the entries that land in it (a list per block, built
// once per pattern: input index, offset in the block; index -1 means 1.0) --
// and written out with coalesced 16-byte stores.  The values of one block
// come from short runs of consecutive input entries (rows ascend within a
// column), so both sides of the copy stay near sequential.  Block 0 of each
// value set also resets its failure flag to the sentinel `big` (no pivot
// has failed yet).
constexpr int LBLK = 4096;

__global__ __launch_bounds__(256) void k_value_gather(const double* __restrict__ vals, int64_t qnz,
                                                      const int32_t* __restrict__ bptr,
                                                      const int2* __restrict__ ent, int64_t total,
                                                      double* __restrict__ store, int64_t mstride,
                                                      int32_t* __restrict__ info, int32_t big) {
  __shared__ __align__(16) double buf[LBLK];
  const int32_t member = blockIdx.y;
  const double* V = vals + (int64_t)member * qnz;
  double* S = store + (int64_t)member * mstride;
  const int64_t b0 = (int64_t)blockIdx.x * LBLK;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) info[member] = big;
#pragma unroll
  for (int x = 2 * tid; x < LBLK; x += 512) *reinterpret_cast<double2*>(buf + x) = make_double2(0.0, 0.0);
  __syncthreads();
  const int32_t e0 = bptr[blockIdx.x], e1 = bptr[blockIdx.x + 1];
  for (int32_t e = e0 + tid; e < e1; e += 256) {
    const int2 q = ent[e];
    buf[q.y] = q.x >= 0 ? V[q.x] : 1.0;
  }
  __syncthreads();
  const int64_t n = min<int64_t>(LBLK, total - b0);  // a multiple of 2: the store size is even
  for (int x = 2 * tid; x < n; x += 512)
    *reinterpret_cast<double2*>(S + b0 + x) = *reinterpret_cast<const double2*>(buf + x);
}

// ---------------------------------------------------------------------------
// operand staging shared by the update kernels: K chunks of 16 doubles per
// row go from global memory straight into LDS, 16 bytes per lane (the lane's
// bytes land at the instruction's LDS base + 16 lane), rows unpadded
// ---------------------------------------------------------------------------

constexpr int DLD = 16;  // doubles per staged row

typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// position of the 16-byte pair p of staged row r within the row: p ^ key(r).
// Rows are 128 bytes, so without the swizzle every row would start on the
// same LDS bank; with it, the 8 (or 16) rows one 128-bit fragment read
// serves per cycle fall on distinct banks for 32 (or 64) banks of 4 bytes.
__device__ __forceinline__ int dkey(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// ---------------------------------------------------------------------------
// fused update: C -= sum_c A_c B_c^T on one 64 x 64 block of an output tile
// ---------------------------------------------------------------------------

// Entry i of the gather map at `base` (a contribution's row or column map;
// base < 0: the contribution has none), read whether or not the lane needs
// it, so that the reads of a contribution's map entries are in flight
// together instead of one conditional read after another.  A lane that needs
// no entry reads the first word of the zero row instead and discards it.
__device__ __forceinline__ int32_t map_entry(const int32_t* __restrict__ maps, int32_t base, int32_t i, bool need,
                                             const double* __restrict__ zrow) {
  const int32_t* q = (need && base >= 0) ? maps + base + i : reinterpret_cast<const int32_t*>(zrow);
  return *q;
}

constexpr int UB = 64;   // output block
constexpr int UKT = 16;  // K chunk staged in LDS
constexpr int USTAGE = 2 * UB * DLD;  // A and B rows of one K chunk
constexpr int UPD_LDS = 2 * USTAGE;   // two stages
static_assert(UPD_LDS >= 2 * 32 * UB, "the partial-slot fold streams two 32-row chunks through the stages");

template <int NB, bool CULL>
__device__ __forceinline__ void dev_update(int32_t it, const int32_t* __restrict__ items,
                                           const UpdTaskD* __restrict__ tasks,
                                           const ContribD* __restrict__ contribs,
                                           const int32_t* __restrict__ maps,
                                           double* __restrict__ S, double* __restrict__ parts,
                                           const double* __restrict__ zrow, double* smem) {
  const int32_t task = items[4 * it], bx = items[4 * it + 1], by = items[4 * it + 2];
  const int32_t part = items[4 * it + 3];
  const UpdTaskD u = tasks[task];
  const int32_t r0 = bx * UB, c0 = by * UB;
  const int32_t ncols = u.diag ? u.c_rows : NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: branches on a wave's rows are scalar
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // the partial slots of the split parts first (in slot order): the
  // accumulators start as their sum, streamed through LDS (before the K
  // loop uses it) in chunks of 32 rows x 64 columns:
  // each wave brings two rows per load instruction straight from global
  // memory, the next chunk's loads fly while the waves owning the current
  // chunk's rows add it, so a slot costs about one memory round trip
  // whatever its rows.  Rows past the tile read its last row and columns past
  // the block's real ones read the slot's own row: neither reaches a stored
  // value.
  if (part == 0 && u.in_npart > 0) {
    const int64_t slot = (int64_t)u.c_rows * NB;
    const int32_t nch = 2 * u.in_npart;
    auto load_chunk = [&](int32_t t) {
      const double* base = parts + u.in_part_off + (int64_t)(t >> 1) * slot;
      double* buf = smem + (t & 1) * (32 * UB);
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int pr = 4 * y + wave;  // rows 2 pr and 2 pr + 1 of the chunk
        const int32_t i = min(r0 + 32 * (t & 1) + 2 * pr + (lane >> 5), u.c_rows - 1);
        __builtin_amdgcn_global_load_lds((gvoid_t*)(base + (int64_t)i * NB + c0 + 2 * (lane & 31)),
                                         (lvoid_t*)(buf + 2 * pr * UB), 16, 0, 0);
      }
    };
    load_chunk(0);
    for (int32_t t = 0; t < nch; ++t) {
      __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's loads of chunk t are in LDS
      __syncthreads();  // everyone's are, and chunk t - 1 has been added
      if (t + 1 < nch) load_chunk(t + 1);
      if ((t & 1) == (wr >> 5)) {
        const double* buf = smem + (t & 1) * (32 * UB);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              acc[a][b][e] += buf[(a * 16 + (lane >> 4) + 4 * e) * UB + wc + b * 16 + (lane & 15)];
      }
    }
    __syncthreads();  // every wave has added the last chunk: the stages are free
  }
  // one stream of (contribution, 16-wide K chunk) steps through two LDS
  // stages: wave w fills rows 16 w + 8 j + lane / 8 (j = 0, 1) of A and of
  // B, lane l bringing the pair (l % 8) ^ key(row); a step's loads are issued
  // right after the barrier that opens the previous step and waited for
  // before the next barrier; rows a map leaves out load from zrow (zeros).
  // Part p of a task split nsplit ways runs steps [S p / nsplit,
  // S (p+1) / nsplit) of the task's S steps.
  constexpr int KSTEPS = NB / UKT;
  const int32_t tot = (u.c_end - u.c_begin) * KSTEPS;
  const int32_t g0 = (int32_t)((int64_t)tot * part / u.nsplit);
  const int32_t nsteps = (int32_t)((int64_t)tot * (part + 1) / u.nsplit) - g0;
  const int srow = 16 * wave + (lane >> 3);
  const double* pa[2];
  const double* pb[2];
  uint32_t cmask = 0xF, mk0 = 0xF, mk1 = 0xF;  // group masks: contribution being issued, stages 0 and 1
  auto open_contrib = [&](int32_t ci) {
    const ContribD c = contribs[ci];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int lr = srow + 8 * j;
      const int p2 = 2 * ((lane & 7) ^ dkey(lr));
      const int32_t r = r0 + lr, cc = c0 + lr;
      const bool ir = r < u.c_rows, ic = cc < ncols;
      const int32_t ma = map_entry(maps, c.rowmap, r, ir, zrow), mb = map_entry(maps, c.colmap, cc, ic, zrow);
      const int32_t sa = !ir ? -1 : c.rowmap < 0 ? (r < c.a_rows ? r : -1) : ma;
      const int32_t sb = !ic ? -1 : c.colmap < 0 ? (cc < c.b_rows ? cc : -1) : mb;
      pa[j] = (sa >= 0 ? S + c.a_off + (int64_t)sa * NB : zrow) + p2;
      pb[j] = (sb >= 0 ? S + c.b_off + (int64_t)sb * NB : zrow) + p2;
    }
    // which 16-row groups of this wave's A rows and B rows the contribution
    // fills (lanes 0..31, one row each); products with an empty group are skipped
    if constexpr (CULL) {
      const int32_t r = r0 + wr + lane, cc = c0 + wc + lane;
      const bool ir = lane < 32 && r < u.c_rows, ic = lane < 32 && cc < ncols;
      const int32_t ma = map_entry(maps, c.rowmap, r, ir, zrow), mb = map_entry(maps, c.colmap, cc, ic, zrow);
      const bool ha = ir && (c.rowmap < 0 ? r < c.a_rows : ma >= 0);
      const bool hb = ic && (c.colmap < 0 ? cc < c.b_rows : mb >= 0);
      const uint64_t ba = __ballot(ha), bb = __ballot(hb);
      cmask = ((ba & 0xFFFFull) ? 1u : 0u) | ((ba & 0xFFFF0000ull) ? 2u : 0u) | ((bb & 0xFFFFull) ? 4u : 0u) |
              ((bb & 0xFFFF0000ull) ? 8u : 0u);
    }
  };
  auto issue = [&](int32_t st, int32_t kn) {
    if (st & 1) mk1 = cmask;
    else mk0 = cmask;
    double* As = smem + (st & 1) * USTAGE;
    double* Bs = As + UB * DLD;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      __builtin_amdgcn_global_load_lds((gvoid_t*)(pa[j] + kn * UKT), (lvoid_t*)(As + (2 * wave + j) * 8 * DLD), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid_t*)(pb[j] + kn * UKT), (lvoid_t*)(Bs + (2 * wave + j) * 8 * DLD), 16, 0, 0);
    }
  };
  // fragments: lane holds the pair lane / 16 of a group of four pairs of
  // row lane % 16 (x feeds the first MFMA of the pair, y the second)
  const int fkey = dkey(lane & 15);
  if (nsteps > 0) {
    open_contrib(u.c_begin + g0 / KSTEPS);
    issue(0, g0 % KSTEPS);
  }
  for (int32_t st = 0; st < nsteps; ++st) {
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's loads of step st are in LDS
    __syncthreads();
    if (st + 1 < nsteps) {
      const int32_t g = g0 + st + 1, kn = g % KSTEPS;
      if (kn == 0) open_contrib(u.c_begin + g / KSTEPS);
      issue(st + 1, kn);
    }
    const double* As = smem + (st & 1) * USTAGE;
    const double* Bs = As + UB * DLD;
    const uint32_t m = CULL ? ((st & 1) ? mk1 : mk0) : 0xFu;
#pragma unroll
    for (int gq = 0; gq < 2; ++gq) {
      const int slot = (4 * gq + (lane >> 4)) ^ fkey;
      double2 af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        af[a] = *reinterpret_cast<const double2*>(As + (wr + a * 16 + (lane & 15)) * DLD + 2 * slot);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bf[b] = *reinterpret_cast<const double2*>(Bs + (wc + b * 16 + (lane & 15)) * DLD + 2 * slot);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if ((m >> a) & (m >> (2 + b)) & 1u)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].x, bf[b].x, acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if ((m >> a) & (m >> (2 + b)) & 1u)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].y, bf[b].y, acc[a][b], 0, 0, 0);
    }
  }
  // epilogue: lane holds D[i][j] with j = lane % 16, i = lane / 16 + 4 e;
  // parts > 0 of a split range write their partial slot, which the tile's
  // next update task folds in
  double* C = S + u.c_off;
  const int64_t slot = (int64_t)u.c_rows * NB;
  if (part > 0) {
    double* pp = parts + u.part_off + (part - 1) * slot;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
          const int32_t j = c0 + wc + b * 16 + (lane & 15);
          if (i < u.c_rows && j < ncols && (!u.diag || j <= i)) pp[(int64_t)i * NB + j] = acc[a][b][e];
        }
    return;
  }
  double cv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t i = min(r0 + wr + a * 16 + (lane >> 4) + 4 * e, u.c_rows - 1);
        const int32_t j = min(c0 + wc + b * 16 + (lane & 15), ncols - 1);
        cv[a][b][e] = C[(int64_t)i * NB + j];
      }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
        const int32_t j = c0 + wc + b * 16 + (lane & 15);
        if (i < u.c_rows && j < ncols && (!u.diag || j <= i))
          C[(int64_t)i * NB + j] = cv[a][b][e] - acc[a][b][e];
      }
}

// ---------------------------------------------------------------------------
// fused update on a 128 x 128 block (dense or nearly full tiles): four waves
// of 64 x 64, K staged in LDS in chunks of 16 through two stages filled by
// direct global-to-LDS loads.  A task may split its K stream over nsplit
// work-groups: part 0 updates the tile, parts s > 0 write partial sums that
// the tile's next update task folds in (in_part_off, in_npart).
// ---------------------------------------------------------------------------

constexpr int UB2 = 128;
constexpr int UKT2 = 16;
constexpr int DSTAGE = 2 * UB2 * DLD;      // A and B rows of one K chunk
constexpr int UPD2_LDS = 2 * DSTAGE;       // two stages
static_assert(UPD2_LDS >= 2 * 32 * UB2, "the partial-slot fold streams two 32-row chunks through the stages");

template <int NB, bool CULL>
__device__ __forceinline__ void dev_update_big(int32_t it, const int32_t* __restrict__ items,
                                               const UpdTaskD* __restrict__ tasks,
                                               const ContribD* __restrict__ contribs,
                                               const int32_t* __restrict__ maps,
                                               double* __restrict__ S, double* __restrict__ parts,
                                               const double* __restrict__ zrow, double* smem) {
  const int32_t task = items[4 * it], bx = items[4 * it + 1], by = items[4 * it + 2];
  const int32_t part = items[4 * it + 3];
  const UpdTaskD u = tasks[task];
  const int32_t r0 = bx * UB2, c0 = by * UB2;
  const int32_t ncols = u.diag ? u.c_rows : NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: branches on a wave's rows are scalar
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // the partial slots of the split parts first (in slot order): the
  // accumulators start as their sum, streamed through LDS before the K loop
  // uses it.  Chunk c of a slot holds row block
  // a = c of both halves of the block (rows 16 c .. 16 c + 15 and
  // 64 + 16 c .. 64 + 16 c + 15, 128 columns), so that every wave adds
  // one row block of its accumulators per chunk.  Each wave brings one row
  // per load instruction straight from global memory, and the next chunk's
  // loads fly while the current one is added.  Rows past the tile read its
  // last row and columns past the block's real ones read the slot's own row:
  // neither reaches a stored value.
  if (part == 0 && u.in_npart > 0) {
    const int64_t slot = (int64_t)u.c_rows * NB;
    const int32_t nch = 4 * u.in_npart;
    auto load_chunk = [&](int32_t t) {
      const double* base = parts + u.in_part_off + (int64_t)(t >> 2) * slot;
      double* buf = smem + (t & 1) * (32 * UB2);
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        const int lr = 4 * x + wave;  // chunk row: half lr / 16, row lr % 16 of row block t % 4
        int32_t i = min(r0 + (lr >> 4) * 64 + 16 * (t & 3) + (lr & 15), u.c_rows - 1);
        asm volatile("" : "+v"(i));  // formed per chunk, not hoisted out of the slot loop into live registers
        __builtin_amdgcn_global_load_lds((gvoid_t*)(base + (int64_t)i * NB + c0 + 2 * lane),
                                         (lvoid_t*)(buf + lr * UB2), 16, 0, 0);
      }
    };
    load_chunk(0);
    for (int32_t q = 0; q < u.in_npart; ++q) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int32_t t = 4 * q + a;
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's loads of chunk t are in LDS
        __syncthreads();  // everyone's are, and chunk t - 1 has been added
        if (t + 1 < nch) load_chunk(t + 1);
        const double* buf = smem + (a & 1) * (32 * UB2) + (wr >> 6) * 16 * UB2;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[a][b][e] += buf[((lane >> 4) + 4 * e) * UB2 + wc + b * 16 + (lane & 15)];
      }
    }
    __syncthreads();  // every wave has added the last chunk: the stages are free
  }
  // One stream of (contribution, 16-wide K chunk) steps.  The operand rows
  // of a step go from global memory straight into one of two LDS stages,
  // 16 bytes per lane: wave w fills rows 32 w + 8 j + lane / 8 (j = 0..3) of
  // A and of B, lane l bringing the pair (l % 8) ^ key(row) of its row, so
  // that the rows are stored swizzled.  A step's loads are issued right after
  // the barrier that opens the previous step (every wave has then finished
  // reading that stage) and waited for before the next barrier.  Rows a map
  // leaves out load from zrow (zeros).  Part p of a task split nsplit ways
  // runs steps [S p / nsplit, S (p+1) / nsplit) of the task's S steps.
  constexpr int KSTEPS = NB / UKT2;
  const int32_t tot = (u.c_end - u.c_begin) * KSTEPS;
  const int32_t g0 = (int32_t)((int64_t)tot * part / u.nsplit);
  const int32_t nsteps = (int32_t)((int64_t)tot * (part + 1) / u.nsplit) - g0;
  const int srow = 32 * wave + (lane >> 3);
  const double* pa[4];
  const double* pb[4];
  uint32_t cmask = 0xFF, mk0 = 0xFF, mk1 = 0xFF;  // group masks: contribution being issued, stages 0 and 1
  auto open_contrib = [&](int32_t ci) {
    const ContribD c = contribs[ci];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lr = srow + 8 * j;
      const int p2 = 2 * ((lane & 7) ^ dkey(lr));
      const int32_t r = r0 + lr, cc = c0 + lr;
      const bool ir = r < u.c_rows, ic = cc < ncols;
      const int32_t ma = map_entry(maps, c.rowmap, r, ir, zrow), mb = map_entry(maps, c.colmap, cc, ic, zrow);
      const int32_t sa = !ir ? -1 : c.rowmap < 0 ? (r < c.a_rows ? r : -1) : ma;
      const int32_t sb = !ic ? -1 : c.colmap < 0 ? (cc < c.b_rows ? cc : -1) : mb;
      pa[j] = (sa >= 0 ? S + c.a_off + (int64_t)sa * NB : zrow) + p2;
      pb[j] = (sb >= 0 ? S + c.b_off + (int64_t)sb * NB : zrow) + p2;
    }
    // which of this wave's 16-row groups of A (its output rows) and of B
    // (its output columns) the contribution fills: products of two groups
    // of which one is all absent rows are zero and are skipped
    if constexpr (CULL) {
      const int32_t r = r0 + wr + lane, cc = c0 + wc + lane;
      const bool ir = r < u.c_rows, ic = cc < ncols;
      const int32_t ma = map_entry(maps, c.rowmap, r, ir, zrow), mb = map_entry(maps, c.colmap, cc, ic, zrow);
      const bool ha = ir && (c.rowmap < 0 ? r < c.a_rows : ma >= 0);
      const bool hb = ic && (c.colmap < 0 ? cc < c.b_rows : mb >= 0);
      const uint64_t ba = __ballot(ha), bb = __ballot(hb);
      uint32_t m = 0;
#pragma unroll
      for (int g = 0; g < 4; ++g)
        m |= (((ba >> (16 * g)) & 0xFFFFull) ? 1u << g : 0u) | (((bb >> (16 * g)) & 0xFFFFull) ? 16u << g : 0u);
      cmask = m;
    }
  };
  auto issue = [&](int32_t st, int32_t kn) {
    if (st & 1) mk1 = cmask;
    else mk0 = cmask;
    double* As = smem + (st & 1) * DSTAGE;
    double* Bs = As + UB2 * DLD;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      __builtin_amdgcn_global_load_lds((gvoid_t*)(pa[j] + kn * UKT2), (lvoid_t*)(As + (4 * wave + j) * 8 * DLD), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid_t*)(pb[j] + kn * UKT2), (lvoid_t*)(Bs + (4 * wave + j) * 8 * DLD), 16, 0, 0);
    }
  };
  // A fragment: lane holds A[i = lane % 16][k] for the pair lane / 16 of a
  // group of four pairs, both k of the pair in one 128-bit read (x feeds the
  // first MFMA of the pair, y the second); B likewise -- the same order of
  // the K sum for both operands
  const int fkey = dkey(lane & 15);
  if (nsteps > 0) {
    open_contrib(u.c_begin + g0 / KSTEPS);
    issue(0, g0 % KSTEPS);
  }
  for (int32_t st = 0; st < nsteps; ++st) {
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's loads of step st are in LDS
    __syncthreads();
    if (st + 1 < nsteps) {
      const int32_t g = g0 + st + 1, kn = g % KSTEPS;
      if (kn == 0) open_contrib(u.c_begin + g / KSTEPS);
      issue(st + 1, kn);
    }
    const double* As = smem + (st & 1) * DSTAGE;
    const double* Bs = As + UB2 * DLD;
    const uint32_t m = CULL ? ((st & 1) ? mk1 : mk0) : 0xFFu;
#pragma unroll
    for (int gq = 0; gq < 2; ++gq) {
      const int slot = (4 * gq + (lane >> 4)) ^ fkey;
      double2 af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        af[a] = *reinterpret_cast<const double2*>(As + (wr + a * 16 + (lane & 15)) * DLD + 2 * slot);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bf[b] = *reinterpret_cast<const double2*>(Bs + (wc + b * 16 + (lane & 15)) * DLD + 2 * slot);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if ((m >> a) & (m >> (4 + b)) & 1u)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].x, bf[b].x, acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if ((m >> a) & (m >> (4 + b)) & 1u)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].y, bf[b].y, acc[a][b], 0, 0, 0);
    }
  }
  // epilogue: lane holds D[i][j] with j = lane % 16, i = lane / 16 + 4 e.
  // Reads are issued unconditionally (addresses clamped into the tile) so
  // that they are all in flight together; only the stores are masked.
  double* C = S + u.c_off;
  const int64_t slot = (int64_t)u.c_rows * NB;
  if (part > 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
          const int32_t j = c0 + wc + b * 16 + (lane & 15);
          if (i < u.c_rows && j < ncols && (!u.diag || j <= i))
            parts[u.part_off + (part - 1) * slot + (int64_t)i * NB + j] = acc[a][b][e];
        }
    return;
  }
  // one 16-row block at a time: its C values are read together (addresses
  // clamped into the tile), then the stores are masked
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double cv[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t i = min(r0 + wr + a * 16 + (lane >> 4) + 4 * e, u.c_rows - 1);
        const int32_t j = min(c0 + wc + b * 16 + (lane & 15), ncols - 1);
        cv[b][e] = C[(int64_t)i * NB + j];
      }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
        const int32_t j = c0 + wc + b * 16 + (lane & 15);
        if (i < u.c_rows && j < ncols && (!u.diag || j <= i))
          C[(int64_t)i * NB + j] = cv[b][e] - acc[a][b][e];
      }
  }
}

// ---------------------------------------------------------------------------
// POTRF of diagonal tiles.  As a by-product the inverse of every 32 x 32
// diagonal block of L is written to dinv (row-major, block J at
// dinv + J*32*32), for the blocked TRSM.
// ---------------------------------------------------------------------------

constexpr int PW = 32;
constexpr int PLD = PW + 1;

// Cholesky of the 32 x 32 block held in P's first 32 rows and the inverse of
// the factor, by one wave, right-looking.  Lanes 0..31 hold row r of A in
// registers; lanes 32..63 hold the unit vector e_r and become column r of
// L^-1 (forward substitution z_c = (e_rc - sum_{p<c} L_cp z_p) / L_cc is the
// same update on different registers, so one instruction stream serves both).
// Pivot c: every lane scales its entry c by 1 / L_cc (rows above the pivot
// keep a zero there), then subtracts x_c L_jc from its entries j > c.  Only
// the pivot chain is serial: the column's entry in row c + 1 (by readlane)
// updates x_{c+1}, and x_{c+1} of lane c + 1 (by readlane) is the next pivot.
// Row c + 2's entry also comes by readlane, so the next chain step finds
// x_{c+2} ready; the other entries of column c go through LDS (cb, 64
// doubles, 16-byte aligned: lanes 32..63 write a spare half) and are applied
// one column later, their loads long done.  Writes L (lower, diagonal
// included, zeros above) to P and the inverse (row-major, stride PLD) to Z.
// Returns the first failing pivot (0-based) or -1; uniform across the wave.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  return fma(fma(-d, r, 1.0), r, r);
}

__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y * fma(-0.5 * d * y, y, 1.5);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int chol32_wave(double* P, double* Z, double* cb, int lane) {
  const int r = lane & 31;
  const bool lo = lane < 32;
  double x[PW];
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    const double a = P[r * PLD + j];
    x[j] = lo ? a : (j == r ? 1.0 : 0.0);
  }
  double d = readlane_f64(x[0], 0);
  double myd = d;  // lane c keeps pivot c
  double rs = rsqrt_nr(d);
  double lc[PW];   // entries of column c - 1 of L, from LDS
#pragma unroll
  for (int c = 0; c < PW; ++c) {
    x[c] = (lo && r < c) ? 0.0 : x[c] * rs;
    if (c + 1 < PW) {
      const double l1 = readlane_f64(x[c], c + 1);
      x[c + 1] = fma(-x[c], l1, x[c + 1]);
      d = readlane_f64(x[c + 1], c + 1);
      myd = (r == c + 1) ? d : myd;
      const double rs1 = rsqrt_nr(d);
      if (c + 2 < PW) {
        const double l2 = readlane_f64(x[c], c + 2);
        x[c + 2] = fma(-x[c], l2, x[c + 2]);
      }
      if (c >= 1) {
#pragma unroll
        for (int j = c + 2; j < PW; ++j) x[j] = fma(-x[c - 1], lc[j], x[j]);
      }
      if (c + 3 < PW) {
        cb[lane] = x[c];
        int j = c + 3;
        if (j & 1) {
          lc[j] = cb[j];
          ++j;
        }
#pragma unroll
        for (; j < PW; j += 2) {
          const double2 lj = *reinterpret_cast<const double2*>(cb + j);
          lc[j] = lj.x;
          lc[j + 1] = lj.y;
        }
      }
      rs = rs1;
    }
    // keep each column's updates in place: left free, the compiler defers
    // them to their uses and holds every loaded column in registers
#pragma unroll
    for (int j = c + 1; j < PW; ++j) asm volatile("" : "+v"(x[j]));
  }
  double* dst = lo ? P + r * PLD : Z + r;
  const int step = lo ? 1 : PLD;
#pragma unroll
  for (int j = 0; j < PW; ++j) dst[j * step] = x[j];
  const unsigned long long m = __ballot(lo && (!(myd > 0.0) || !isfinite(myd)));
  return m ? (int)__builtin_ctzll(m) : -1;
}

template <int NB>
constexpr int potrf_lds() { return 2 * NB * PLD + PW * PLD + 2 * PW; }

// POTRF of one diagonal tile, left-looking over 32-column panels.  A panel
// (rows j0.., 32 columns) is loaded into LDS in bulk; the columns already
// factored are streamed in 32-column slabs (bulk load, next slab prefetched
// in registers) and applied with MFMA, accumulators in registers; the 32 x 32
// diagonal block is factored and inverted by one wave; the rows below are
// multiplied by that inverse on MFMA; the panel is written back once.
template <int NB>
__device__ __forceinline__ void dev_potrf(int32_t k, double* __restrict__ S,
                                          double* __restrict__ dinv_m, int32_t* __restrict__ inf,
                                          int32_t nreal, double* smem) {
  double* P = smem;
  double* Sl = smem + NB * PLD;
  double* Z = Sl + NB * PLD;
  double* cb = Z + PW * PLD;  // column broadcast of the 32 x 32 factor
  double* A = S + (int64_t)k * NB * NB;
  double* dinv = dinv_m + (int64_t)k * NB * PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int PER = NB * PW / 256;            // elements per thread of a full-height panel
  const int trow = tid >> 5, tcol = tid & 31;   // 8 rows x 32 columns per pass
  constexpr int RBW = NB >= 64 ? NB / 64 : 1;  // row blocks per wave at most
  for (int j0 = 0; j0 < NB; j0 += PW) {
    const int pr = NB - j0;
    // panel load: thread (trow, tcol) takes rows q*8 + trow; pr is a
    // multiple of 32, so a whole group of 8 rows is in or out (uniform skip)
    // and every address is one base plus a uniform offset
    {
      double v[PER];
      const double* src = A + (int64_t)(j0 + trow) * NB + j0 + tcol;
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (q * 8 < pr) v[q] = src[(int64_t)q * 8 * NB];
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (q * 8 < pr) P[(q * 8 + trow) * PLD + tcol] = v[q];
    }
    if (j0 > 0) {
      // P -= L[j0:, :j0] L[j0:j0+32, :j0]^T: 32-column slabs of the factored
      // columns staged through LDS (bulk load, next slab prefetched in
      // registers), MFMA with accumulators in registers
      d4 acc[RBW][2];
#pragma unroll
      for (int i = 0; i < RBW; ++i) acc[i][0] = acc[i][1] = d4{0.0, 0.0, 0.0, 0.0};
      double v[PER];
      const double* src = A + (int64_t)(j0 + trow) * NB + tcol;
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (q * 8 < pr) v[q] = src[(int64_t)q * 8 * NB];
      for (int s0 = 0; s0 < j0; s0 += PW) {
        __syncthreads();  // previous slab fully consumed
#pragma unroll
        for (int q = 0; q < PER; ++q)
          if (q * 8 < pr) Sl[(q * 8 + trow) * PLD + tcol] = v[q];
        __syncthreads();
        if (s0 + PW < j0) {
#pragma unroll
          for (int q = 0; q < PER; ++q)
            if (q * 8 < pr) v[q] = src[(int64_t)q * 8 * NB + s0 + PW];
        }
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
          const int t = wave + 4 * i;
          if (t < pr / 16) {
            const double* pa = Sl + (t * 16 + (lane & 15)) * PLD + (lane >> 4);
            const double* pb0 = Sl + (lane & 15) * PLD + (lane >> 4);
            const double* pb1 = Sl + (16 + (lane & 15)) * PLD + (lane >> 4);
#pragma unroll 2
            for (int kk = 0; kk < PW; kk += 4) {
              acc[i][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb0[kk], acc[i][0], 0, 0, 0);
              acc[i][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb1[kk], acc[i][1], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();  // P fully loaded before the accumulated update lands
#pragma unroll
      for (int i = 0; i < RBW; ++i) {
        const int t = wave + 4 * i;
        if (t < pr / 16) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double* row = P + (t * 16 + (lane >> 4) + 4 * e) * PLD;
            row[lane & 15] -= acc[i][0][e];
            row[16 + (lane & 15)] -= acc[i][1][e];
          }
        }
      }
    }
    __syncthreads();
    if (wave == 0) {
      const int bad = chol32_wave(P, Z, cb, lane);
      if (lane == 0 && bad >= 0 && k * NB + j0 + bad < nreal) atomicMin(inf, k * NB + j0 + bad + 1);
    }
    __syncthreads();
    // rows below the diagonal block: P_below <- P_below inv(L_top)^T on MFMA;
    // each wave owns whole 16-row blocks, reads them fully, then overwrites
    for (int t = wave; t < (pr - PW) / 16; t += 4) {
      d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
      const double* pa = P + (PW + t * 16 + (lane & 15)) * PLD + (lane >> 4);
      const double* z0 = Z + (lane & 15) * PLD + (lane >> 4);
      const double* z1 = Z + (16 + (lane & 15)) * PLD + (lane >> 4);
#pragma unroll
      for (int kk = 0; kk < PW; kk += 4) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], z0[kk], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], z1[kk], acc1, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double* row = P + (PW + t * 16 + (lane >> 4) + 4 * e) * PLD;
        row[lane & 15] = acc0[e];
        row[16 + (lane & 15)] = acc1[e];
      }
    }
    for (int x = tid; x < PW * PW; x += 256) dinv[(j0 / PW) * PW * PW + x] = Z[(x / PW) * PLD + x % PW];
    __syncthreads();
    {
      double* dst = A + (int64_t)(j0 + trow) * NB + j0 + tcol;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int r = q * 8 + trow;
        if (q * 8 < pr && (tcol <= r || r >= PW)) dst[(int64_t)q * 8 * NB] = P[r * PLD + tcol];
      }
    }
    __syncthreads();
  }
}

// POTRF with one panel of look-ahead (tiles of 128 and 256).  While wave 0
// factors and inverts the diagonal block of panel j, waves 1..3 accumulate
// the update of panel j+1 from the columns factored before panel j (read back
// from the tile, staged through LDS areas private to each wave, so no
// barrier involves wave 0); after panel j's rows below the diagonal block are
// solved, they add panel j's own contribution straight from LDS and subtract
// the total from panel j+1's freshly loaded values.  Same arithmetic as the
// left-looking dev_potrf, with the update of each panel taken in two parts.
constexpr int LKC = 16;          // K chunk of the look-ahead staging
constexpr int LKLD = LKC + 1;

template <int NB>
constexpr int la_rbw() { return ((NB - PW) / 16 + 2) / 3; }  // row blocks per waves 1..3

template <int NB>
constexpr int potrf_la_lds() { return NB * PLD + PW * PLD + 2 * PW + 3 * (la_rbw<NB>() * 16 + PW) * LKLD; }

template <int NB>
__device__ __forceinline__ void dev_potrf_la(int32_t k, double* __restrict__ S,
                                             double* __restrict__ dinv_m, int32_t* __restrict__ inf,
                                             int32_t nreal, double* smem) {
  constexpr int RB3 = la_rbw<NB>();
  constexpr int WROWS = RB3 * 16 + PW;  // staged rows per wave: its A rows, then the B rows
  double* P = smem;
  double* Z = P + NB * PLD;
  double* cb = Z + PW * PLD;  // column broadcast of the 32 x 32 factor
  double* Wall = cb + 2 * PW;
  double* A = S + (int64_t)k * NB * NB;
  double* dinv = dinv_m + (int64_t)k * NB * PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int PER = NB * PW / 256;
  const int trow = tid >> 5, tcol = tid & 31;
  // rows [j0, NB) x columns [j0, j0 + 32) of the tile into P (pr = NB - j0 is a
  // multiple of 32, so groups of 8 rows are wholly in or out)
  auto load_panel = [&](int j0) {
    const int pr = NB - j0;
    double v[PER];
    const double* src = A + (int64_t)(j0 + trow) * NB + j0 + tcol;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (q * 8 < pr) v[q] = src[(int64_t)q * 8 * NB];
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (q * 8 < pr) P[(q * 8 + trow) * PLD + tcol] = v[q];
  };
  load_panel(0);
  for (int j0 = 0; j0 < NB; j0 += PW) {
    const int pr = NB - j0, pr1 = pr - PW;  // rows of this panel and of the next
    const int nrb = pr1 / 16;               // 16-row blocks of the next panel
    d4 acc[RB3][2];
#pragma unroll
    for (int b = 0; b < RB3; ++b) acc[b][0] = acc[b][1] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // P holds this panel, fully updated
    if (wave == 0) {
      const int bad = chol32_wave(P, Z, cb, lane);
      if (lane == 0 && bad >= 0 && k * NB + j0 + bad < nreal) atomicMin(inf, k * NB + j0 + bad + 1);
    } else if (pr1 > 0 && j0 > 0) {
      const int w = wave - 1;
      double* WA = Wall + w * WROWS * LKLD;
      double* WB = WA + RB3 * 16 * LKLD;
      // 16 columns of this wave's rows of the next panel, and of the next
      // panel's first 32 rows, as 4-double segments: segment x of a chunk
      // goes to lane x % 64.  The next chunk's segments are loaded into
      // registers while the current one is multiplied, so the chunks' load
      // latencies overlap the MFMA work instead of adding up.
      constexpr int NIT = (WROWS * 4 + 63) / 64;
      double2 pv[NIT][2];
      auto fetch = [&](int s0) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          const int x = lane + 64 * it;
          const int rl = x >> 2, seg = (x & 3) * 4;
          int grow = -1;  // row of the tile, or -1 for a row block past the panel (or a spare segment)
          if (rl < RB3 * 16) {
            const int t = w + 3 * (rl >> 4);
            grow = t < nrb ? j0 + PW + t * 16 + (rl & 15) : -1;
          } else if (rl < WROWS) {
            grow = j0 + PW + (rl - RB3 * 16);
          }
          pv[it][0] = pv[it][1] = make_double2(0.0, 0.0);
          if (grow >= 0) {
            const double2* src = reinterpret_cast<const double2*>(A + (int64_t)grow * NB + s0 + seg);
            pv[it][0] = src[0];
            pv[it][1] = src[1];
          }
        }
      };
      fetch(0);
      for (int s0 = 0; s0 < j0; s0 += LKC) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          const int x = lane + 64 * it;
          const int rl = x >> 2, seg = (x & 3) * 4;
          if (rl < WROWS) {
            double* d = (rl < RB3 * 16 ? WA + rl * LKLD : WB + (rl - RB3 * 16) * LKLD) + seg;
            d[0] = pv[it][0].x;
            d[1] = pv[it][0].y;
            d[2] = pv[it][1].x;
            d[3] = pv[it][1].y;
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (s0 + LKC < j0) fetch(s0 + LKC);
#pragma unroll
        for (int b = 0; b < RB3; ++b) {
          if (w + 3 * b < nrb) {
#pragma unroll
            for (int kk = 0; kk < LKC; kk += 4) {
              const double af = WA[(b * 16 + (lane & 15)) * LKLD + kk + (lane >> 4)];
              const double b0 = WB[(lane & 15) * LKLD + kk + (lane >> 4)];
              const double b1 = WB[(16 + (lane & 15)) * LKLD + kk + (lane >> 4)];
              acc[b][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, b0, acc[b][0], 0, 0, 0);
              acc[b][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, b1, acc[b][1], 0, 0, 0);
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    // rows below the diagonal block: P_below <- P_below inv(L_top)^T on MFMA;
    // each wave owns whole 16-row blocks, reads them fully, then overwrites
    for (int t = wave; t < pr1 / 16; t += 4) {
      d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
      const double* pa = P + (PW + t * 16 + (lane & 15)) * PLD + (lane >> 4);
      const double* z0 = Z + (lane & 15) * PLD + (lane >> 4);
      const double* z1 = Z + (16 + (lane & 15)) * PLD + (lane >> 4);
#pragma unroll
      for (int kk = 0; kk < PW; kk += 4) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], z0[kk], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], z1[kk], acc1, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double* row = P + (PW + t * 16 + (lane >> 4) + 4 * e) * PLD;
        row[lane & 15] = acc0[e];
        row[16 + (lane & 15)] = acc1[e];
      }
    }
    for (int x = tid; x < PW * PW; x += 256) dinv[(j0 / PW) * PW * PW + x] = Z[(x / PW) * PLD + x % PW];
    __syncthreads();
    {
      double* dst = A + (int64_t)(j0 + trow) * NB + j0 + tcol;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int r = q * 8 + trow;
        if (q * 8 < pr && (tcol <= r || r >= PW)) dst[(int64_t)q * 8 * NB] = P[r * PLD + tcol];
      }
    }
    if (pr1 > 0) {
      // this panel's contribution to the next one, from LDS
      if (wave > 0) {
        const int w = wave - 1;
#pragma unroll
        for (int b = 0; b < RB3; ++b) {
          const int t = w + 3 * b;
          if (t < nrb) {
            const double* pa = P + (PW + t * 16 + (lane & 15)) * PLD + (lane >> 4);
            const double* pb0 = P + (PW + (lane & 15)) * PLD + (lane >> 4);
            const double* pb1 = P + (PW + 16 + (lane & 15)) * PLD + (lane >> 4);
#pragma unroll
            for (int kk = 0; kk < PW; kk += 4) {
              acc[b][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb0[kk], acc[b][0], 0, 0, 0);
              acc[b][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb1[kk], acc[b][1], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();  // P is no longer read as this panel
      load_panel(j0 + PW);
      __syncthreads();
      if (wave > 0) {
        const int w = wave - 1;
#pragma unroll
        for (int b = 0; b < RB3; ++b) {
          const int t = w + 3 * b;
          if (t < nrb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              double* row = P + (t * 16 + (lane >> 4) + 4 * e) * PLD;
              row[lane & 15] -= acc[b][0][e];
              row[16 + (lane & 15)] -= acc[b][1][e];
            }
          }
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// TRSM: rows of a panel tile times L_kk^-T, 32 rows per work item, blocked by
// 32 columns: X_J <- (X_J - X_<J L_J,<J^T) inv(L_JJ)^T, both products on MFMA
// ---------------------------------------------------------------------------

constexpr int TR = 32;
constexpr int TLD = 4;  // row padding of the LDS copies

template <int NB>
constexpr int trsm_lds() { return TR * (NB + TLD) + PW * (PW + 1); }

// X (the panel rows) sits in LDS; the rows of L a block column needs stream
// through one 32 x 32 LDS chunk, the next chunk and the next 32 x 32 inverse
// read into registers while the current one is used.  Keeping only X
// resident lets two work-groups share a compute unit.
template <int NB>
__device__ __forceinline__ void dev_trsm(int32_t it, const int32_t* __restrict__ items,
                                         const TrsmTaskD* __restrict__ tasks,
                                         double* __restrict__ S,
                                         const double* __restrict__ dinv_m, double* smem) {
  constexpr int XLD = NB + TLD;
  constexpr int CLDT = PW + 1;
  constexpr int PER = TR * NB / 256;
  double* X = smem;
  double* Lc = smem + TR * XLD;  // 32 x 32 chunk of L
  const TrsmTaskD t = tasks[items[2 * it]];
  const int32_t rb = items[2 * it + 1];
  const int32_t r0 = rb * TR;
  const int32_t nr = min(TR, t.rows - r0);
  double* Xg = S + t.x_off + (int64_t)r0 * NB;
  const double* L = S + t.l_off;
  const double* dinv = dinv_m + (int64_t)t.k * NB * PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = q * 256 + tid, rr = min(x / NB, nr - 1);
      v[q] = Xg[(int64_t)rr * NB + x % NB];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = q * 256 + tid;
      X[(x / NB) * XLD + x % NB] = (x / NB) < nr ? v[q] : 0.0;
    }
  }
  __syncthreads();  // X staged before block column 0 reads it
  // each wave owns one 16 x 16 tile of the 32 x 32 block column
  const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
  const int crow = tid >> 3, ccol = (tid & 7) * 4;  // this thread's 4 values of a chunk
  constexpr int NJ = NB / PW;
  // the chunks in use order: block column J needs rows J*32.. of L, column
  // chunks g = 0..J-1; chunk index s runs over all (J, g) pairs
  double cv[4];
  auto fetch_chunk = [&](int J, int g) {
    const double* src = L + (int64_t)(J * PW + crow) * NB + g * PW + ccol;
    const double2 a = reinterpret_cast<const double2*>(src)[0];
    const double2 b = reinterpret_cast<const double2*>(src)[1];
    cv[0] = a.x;
    cv[1] = a.y;
    cv[2] = b.x;
    cv[3] = b.y;
  };
  double dz[PW / 4];
  auto fetch_inv = [&](int J) {
    const double* db = dinv + J * PW * PW + (wc + (lane & 15)) * PW + (lane >> 4);
#pragma unroll
    for (int q = 0; q < PW / 4; ++q) dz[q] = db[4 * q];
  };
  fetch_inv(0);
  if (NJ > 1) fetch_chunk(1, 0);
  for (int J = 0; J < NJ; ++J) {
    const int j0 = J * PW;
    d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = acc;
    const double* xa = X + (wr + (lane & 15)) * XLD + (lane >> 4);
    const double* lb = Lc + (wc + (lane & 15)) * CLDT + (lane >> 4);
    for (int g = 0; g < J; ++g) {
      __syncthreads();  // previous chunk consumed
#pragma unroll
      for (int e = 0; e < 4; ++e) Lc[crow * CLDT + ccol + e] = cv[e];
      __syncthreads();
      if (g + 1 < J) fetch_chunk(J, g + 1);
      else if (J + 1 < NJ) fetch_chunk(J + 1, 0);
#pragma unroll
      for (int kk = 0; kk < PW; kk += 8) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[g * PW + kk], lb[kk], acc, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[g * PW + kk + 4], lb[kk + 4], acc2, 0, 0, 0);
      }
    }
    double dzc[PW / 4];
#pragma unroll
    for (int q = 0; q < PW / 4; ++q) dzc[q] = dz[q];
    if (J + 1 < NJ) fetch_inv(J + 1);
    // Y = X_J - acc, kept in registers until every wave has read X_<J
    double y[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      y[e] = X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] - (acc[e] + acc2[e]);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] = y[e];
    __syncthreads();
    // X_J = Y inv(L_JJ)^T
    d4 z = {0.0, 0.0, 0.0, 0.0};
    const double* ya = X + (wr + (lane & 15)) * XLD + j0 + (lane >> 4);
#pragma unroll
    for (int q = 0; q < PW / 4; ++q)
      z = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[4 * q], dzc[q], z, 0, 0, 0);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] = z[e];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int x = q * 256 + tid;
    if ((x / NB) < nr) Xg[x] = X[(x / NB) * XLD + x % NB];
  }
}

// ---------------------------------------------------------------------------
// one level of the schedule in one launch: work-groups [0, np) factor
// diagonal tiles, [np, np+nu) apply fused updates, the rest solve panel rows.
// POTRF work-groups come first so that the latency-bound factorizations start
// before the update work that fills the rest of the chip.
// ---------------------------------------------------------------------------

struct LevelArgs {
  const int32_t* potrf;   // block columns
  const int32_t* big;     // quads: task, block row, block col, part (128 blocks)
  const int32_t* upd;     // quads (64 blocks)
  const int32_t* trsm;    // pairs
  int32_t np, nbig, nu, nt;
  double* parts;          // partial-sum slots
  const double* zrow;     // n_b zeros: the source of rows a gather map leaves out
  int64_t pstride;
  const UpdTaskD* utasks;
  const ContribD* contribs;
  const int32_t* maps;
  const TrsmTaskD* ttasks;
  double* store;
  int64_t mstride;
  double* dinv;
  int64_t dstride;
  int32_t* info;
  int32_t nreal;
};

// The kernels of one level.  POTRF, the update blocks and the TRSM items of a
// level are independent of each other, so they are separate kernels (each
// with its own LDS and register budget, which sets how many work-groups share
// a compute unit) that the runtime runs concurrently on forked graph branches.
template <int NB>
constexpr int k_potrf_lds() { return NB >= 128 ? potrf_la_lds<NB>() : potrf_lds<NB>(); }

template <int NB>
__global__ __launch_bounds__(256) void k_potrf(LevelArgs a) {
  extern __shared__ double smem[];
  const int32_t member = blockIdx.y;
  if constexpr (NB >= 128)
    dev_potrf_la<NB>(a.potrf[blockIdx.x], a.store + (int64_t)member * a.mstride,
                     a.dinv + (int64_t)member * a.dstride, a.info + member, a.nreal, smem);
  else
    dev_potrf<NB>(a.potrf[blockIdx.x], a.store + (int64_t)member * a.mstride,
                  a.dinv + (int64_t)member * a.dstride, a.info + member, a.nreal, smem);
}

// HAS_G compiles the 128-block path in or out, so a level without it keeps
// the smaller register footprint of the 64-block path
// CULL: skip the products of 16-row operand groups that a contribution
// leaves empty (active-column plans; dense plans never have one)
template <int NB, bool HAS_G, bool CULL>
__global__ __launch_bounds__(256, HAS_G ? 2 : 3) void k_upd(LevelArgs a) {
  extern __shared__ double smem[];
  const int32_t member = blockIdx.y;
  double* S = a.store + (int64_t)member * a.mstride;
  double* parts = a.parts + (int64_t)member * a.pstride;
  int32_t b = blockIdx.x;
  if (HAS_G && b < a.nbig) {
    if constexpr (NB >= UB2 && HAS_G) dev_update_big<NB, CULL>(b, a.big, a.utasks, a.contribs, a.maps, S, parts, a.zrow, smem);
    return;
  }
  b -= a.nbig;
  dev_update<NB, CULL>(b, a.upd, a.utasks, a.contribs, a.maps, S, parts, a.zrow, smem);
}

template <int NB>
__global__ __launch_bounds__(256) void k_trsm(LevelArgs a) {
  extern __shared__ double smem[];
  const int32_t member = blockIdx.y;
  dev_trsm<NB>(blockIdx.x, a.trsm, a.ttasks, a.store + (int64_t)member * a.mstride,
               a.dinv + (int64_t)member * a.dstride, smem);
}

// ---------------------------------------------------------------------------
// measurement: FP64 MFMA issue rate with operands in registers, 16
// independent accumulators per wave, no memory traffic in the loop
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// reverse mode of log det: selected inverse by the blocked Takahashi
// recurrence (tile DAG in reverse)
// ---------------------------------------------------------------------------

// G_k = L_kk^-1, one 32-column block J per work-group: G_JJ = D_J (the 32 x 32
// inverse the factorization kept) and, down the block column,
// G_IJ = -D_I sum_{J <= P < I} L_IP G_PJ, both products on MFMA; the block
// column of G sits in LDS and is written out in full (zeros above).
constexpr int GLD = 33;

template <int NB>
constexpr int trtri_lds() { return NB * GLD + 32 * GLD; }

template <int NB>
__global__ __launch_bounds__(256) void k_trtri(const int32_t* __restrict__ items,
                                               const double* __restrict__ S,
                                               const double* __restrict__ dinv,
                                               double* __restrict__ G) {
  extern __shared__ double smem[];
  double* Gc = smem;            // NB x 32 block column
  double* T = smem + NB * GLD;  // 32 x 32
  const int32_t k = items[2 * blockIdx.x], J = items[2 * blockIdx.x + 1];
  const double* L = S + (int64_t)k * NB * NB;
  const double* D = dinv + (int64_t)k * NB * 32;
  double* Gk = G + (int64_t)k * NB * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = (wave >> 1) * 16, tc = (wave & 1) * 16;
  for (int x = tid; x < 32 * 32; x += 256) Gc[(J * 32 + x / 32) * GLD + x % 32] = D[J * 1024 + x];
  __syncthreads();
  for (int I = J + 1; I < NB / 32; ++I) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = J * 32; kk < I * 32; kk += 4) {
      const double a = L[(int64_t)(I * 32 + tr + (lane & 15)) * NB + kk + (lane >> 4)];
      const double b = Gc[(kk + (lane >> 4)) * GLD + tc + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) T[(tr + (lane >> 4) + 4 * e) * GLD + tc + (lane & 15)] = acc[e];
    __syncthreads();
    acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < 32; kk += 4) {
      const double a = D[I * 1024 + (tr + (lane & 15)) * 32 + kk + (lane >> 4)];
      const double b = T[(kk + (lane >> 4)) * GLD + tc + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Gc[(I * 32 + tr + (lane >> 4) + 4 * e) * GLD + tc + (lane & 15)] = -acc[e];
    __syncthreads();
  }
  for (int x = tid; x < NB * 32; x += 256) {
    const int r = x / 32, c = x % 32;
    Gk[(int64_t)r * NB + J * 32 + c] = (r >= J * 32) ? Gc[r * GLD + c] : 0.0;
  }
}

// One 64 x 64 block of C = beta C + alpha sum_t A_t B_t over the terms of a
// task.  A_t(r, p) is read through the term's row map and contraction map in
// one of three forms (stored tile, transposed tile, symmetric diagonal tile
// with its lower triangle stored); B_t(p, j) is row p of a tile (through an
// optional map), j the output column.  K is staged in LDS in chunks of 32.
constexpr int CB = 64;
constexpr int CKT = 32;
constexpr int CLD = CKT + 2;  // a staged row: 16 K pairs and one pair of padding
template <int NB>
constexpr int con_lds() { return 2 * CB * CLD + (2 * (CB + 2 * NB) + 1) / 2; }  // As, Bs, two sets of maps (row map, two K maps)

struct BackArgs {
  const int32_t* items;  // triples: task, block row, block column
  const ConTaskD* tasks;
  const ConTermD* terms;
  const int32_t* maps;
  const double* L;  // factor store
  double* Z;        // selected-inverse store (same layout)
  double* M;        // L_mk G_k in the off-diagonal slots, G_k in the diagonal slots
  double* P;        // partial slots of split tasks (output buffer 4)
};

template <int NB>
__global__ __launch_bounds__(256, 4) void k_backcon(BackArgs g) {
  extern __shared__ double smem[];
  double* As = smem;
  double* Bs = smem + CB * CLD;
  int32_t* mapsets = reinterpret_cast<int32_t*>(smem + 2 * CB * CLD);  // two sets: row map (CB), two K maps (NB each)
  constexpr int MSET = CB + 2 * NB;
  const int32_t task = g.items[3 * blockIdx.x], bx = g.items[3 * blockIdx.x + 1],
                by = g.items[3 * blockIdx.x + 2];
  const ConTaskD u = g.tasks[task];
  const int32_t r0 = bx * CB, c0 = by * CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // the wave's 16-row groups that hold output rows (the others are padding
  // of the block past the task's rows: their products are skipped)
  const bool row_g[2] = {r0 + wr < u.c_rows, r0 + wr + 16 < u.c_rows};
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // The task's terms run as one stream of 32-wide K chunks, the next chunk's
  // values read into registers while the current one is on MFMA, across term
  // boundaries too: a term's row map and both contraction maps sit in one of
  // two LDS sets (terms alternate), written from registers read a term
  // ahead, so that the first chunk of the next term is read during the last
  // chunk of the current one.  In LDS a row (an output row of A, an output
  // column of B) holds its chunk as 16 K pairs, padded so that 16 lanes
  // reading one pair of 16 consecutive rows touch every bank once.  Each
  // thread stages eight A and eight B values as four K pairs: a stored or
  // symmetric A gives row ra, pairs 4 (tid % 4) .. +3 (a run along the stored
  // row); a transposed A, like B, gives pair kp of rows (A) or columns (B)
  // jl + 16 x, x = 0..3 (16 lanes cover 16 consecutive values of the stored
  // row).
  const int ra = tid >> 2, pa = (tid & 3) * 4;
  const int kp = tid >> 4, jl = tid & 15;
  struct Term {  // what the fetches of a term need
    const double* A;
    const double* B;
    int32_t K, mode;
    bool tr, arun;
  };
  auto make_term = [&](const ConTermD& c) {
    Term s;
    s.K = c.K;
    s.mode = c.a_mode;
    s.A = (c.a_buf == 0 ? g.L : (c.a_buf == 1 ? g.Z : g.M)) + c.a_off;
    s.B = (c.b_buf == 0 ? g.L : (c.b_buf == 1 ? g.Z : g.M)) + c.b_off;
    s.tr = c.a_mode == CA_TRANS;
    // A's elements along a thread's run are contiguous in a stored row when
    // the index that varies along it is not mapped: p of a stored A with no
    // K map, r of a transposed A with no row map (tiles of 64 and more, so
    // the run stays inside the row; offsets even)
    s.arun = NB >= CB && ((c.a_mode == CA_NORMAL && c.a_qmap < 0) || (s.tr && c.a_rmap < 0));
    return s;
  };
  // thread tid's entries of a term's maps (row map entry tid, contraction map
  // entries tid: K <= n_b <= 256), read into registers, then put in a set
  int32_t mr = -1, ma = 0, mb = 0;
  auto map_regs = [&](const ConTermD& c) {
    const int32_t r = r0 + tid;
    mr = (tid < CB && r < u.c_rows) ? (c.a_rmap < 0 ? r : g.maps[c.a_rmap + r]) : -1;
    ma = tid < c.K ? (c.a_qmap < 0 ? tid : g.maps[c.a_qmap + tid]) : 0;
    mb = tid < c.K ? (c.b_qmap < 0 ? tid : g.maps[c.b_qmap + tid]) : 0;
  };
  auto put_maps = [&](int set, int32_t K) {
    int32_t* m = mapsets + set * MSET;
    if (tid < CB) m[tid] = mr;
    if (tid < K) {
      m[CB + tid] = ma;
      m[CB + NB + tid] = mb;
    }
  };
  double av[8], bv[8];
  auto fetch = [&](const Term& s, int set, int32_t k0) {
    const int32_t K = s.K;
    const double* A = s.A;
    const int32_t* arow = mapsets + set * MSET;
    const int32_t* aq = arow + CB;
    const int32_t* bq = aq + NB;
    if (s.tr) {  // av[2 x + y] = A(r0 + jl + 16 x, k0 + 2 kp + y)
      const int32_t p0 = k0 + 2 * kp;
      const int32_t q0 = p0 < K ? aq[p0] : -1, q1 = p0 + 1 < K ? aq[p0 + 1] : -1;
      if (s.arun) {  // rows r0 + jl + 16 x lie inside the stored row
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int32_t q = y ? q1 : q0;
          const double* ap = A + (int64_t)max(q, 0) * NB + r0 + jl;
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            const double v = ap[16 * x];
            av[2 * x + y] = (q >= 0 && r0 + jl + 16 * x < u.c_rows) ? v : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int32_t rr = arow[jl + 16 * x];
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const int32_t q = y ? q1 : q0;
            const double v = A[(int64_t)max(q, 0) * NB + max(rr, 0)];
            av[2 * x + y] = (rr >= 0 && q >= 0) ? v : 0.0;
          }
        }
      }
    } else {  // av[e] = A(r0 + ra, k0 + 2 pa + e)
      const int32_t rr = arow[ra];
      const int32_t s0 = k0 + 2 * pa;
      if (s.arun) {
        const double* ap = A + (int64_t)max(rr, 0) * NB + s0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double2 v = *reinterpret_cast<const double2*>(ap + 2 * e);
          av[2 * e] = (rr >= 0 && s0 + 2 * e < K) ? v.x : 0.0;
          av[2 * e + 1] = (rr >= 0 && s0 + 2 * e + 1 < K) ? v.y : 0.0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int32_t pl = s0 + e;
          const int32_t qq = pl < K ? aq[pl] : -1;
          const int32_t rc = max(rr, 0), qc = max(qq, 0);
          const int64_t off = s.mode == CA_NORMAL ? (int64_t)rc * NB + qc
                                                    : (int64_t)max(rc, qc) * NB + min(rc, qc);
          const double v = A[off];
          av[e] = (rr >= 0 && qq >= 0) ? v : 0.0;
        }
      }
    }
    // bv[2 x + y] = B(k0 + 2 kp + y, c0 + jl + 16 x)
    const int32_t p0 = k0 + 2 * kp;
    const int32_t q0 = p0 < K ? bq[p0] : -1, q1 = p0 + 1 < K ? bq[p0 + 1] : -1;
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int32_t q = y ? q1 : q0;
      const double* bp = s.B + (int64_t)max(q, 0) * NB;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int32_t j = c0 + jl + 16 * x;
        if constexpr (NB >= CB) {  // the block's columns lie inside the row
          const double v = bp[j];
          bv[2 * x + y] = q >= 0 ? v : 0.0;
        } else {
          const double v = bp[min(j, NB - 1)];
          bv[2 * x + y] = (q >= 0 && j < NB) ? v : 0.0;
        }
      }
    }
  };
  if (u.t_begin < u.t_end) {
    const ConTermD first = g.terms[u.t_begin];
    map_regs(first);
    put_maps(0, first.K);
    __syncthreads();
    Term cur = make_term(first);
    int set = 0;
    fetch(cur, set, 0);
    for (int32_t t = u.t_begin; t < u.t_end; ++t) {
      const bool more = t + 1 < u.t_end;
      Term nxt{};
      if (more) {  // the next term's maps, behind this term's first chunk
        const ConTermD c = g.terms[t + 1];
        map_regs(c);
        nxt = make_term(c);
      }
      for (int32_t k0 = 0; k0 < cur.K; k0 += CKT) {
        const bool last = k0 + CKT >= cur.K;
        if (cur.tr) {
#pragma unroll
          for (int x = 0; x < 4; ++x)
            *reinterpret_cast<double2*>(As + (jl + 16 * x) * CLD + 2 * kp) = double2{av[2 * x], av[2 * x + 1]};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            *reinterpret_cast<double2*>(As + ra * CLD + 2 * (pa + e)) = double2{av[2 * e], av[2 * e + 1]};
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
          *reinterpret_cast<double2*>(Bs + (jl + 16 * x) * CLD + 2 * kp) = double2{bv[2 * x], bv[2 * x + 1]};
        // the other set was last read by the fetches of the previous term,
        // before the barrier that closed its chunk
        if (last && more) put_maps(set ^ 1, nxt.K);
        __syncthreads();
        if (!last || more) {  // one call site: the next chunk of this term or the first of the next
          const Term& ft = last ? nxt : cur;
          fetch(ft, last ? set ^ 1 : set, last ? 0 : k0 + CKT);
        }
        // lane group lane / 16 takes pair 4 gq + lane / 16: its first K value
        // feeds the first product of the pair, its second the second, for A
        // and B alike
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          const int sl = 4 * gq + (lane >> 4);
          double2 af[2], bf[2];
#pragma unroll
          for (int a = 0; a < 2; ++a)
            if (row_g[a]) af[a] = *reinterpret_cast<const double2*>(As + (wr + a * 16 + (lane & 15)) * CLD + 2 * sl);
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            bf[b] = *reinterpret_cast<const double2*>(Bs + (wc + b * 16 + (lane & 15)) * CLD + 2 * sl);
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
            if (row_g[a])
#pragma unroll
              for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].x, bf[b].x, acc[a][b], 0, 0, 0);
#pragma unroll
          for (int a = 0; a < 2; ++a)
            if (row_g[a])
#pragma unroll
              for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a].y, bf[b].y, acc[a][b], 0, 0, 0);
        }
        __syncthreads();
      }
      if (more) {
        cur = nxt;
        set ^= 1;
      }
    }
  }
  double* C = (u.c_buf == 4 ? g.P : u.c_buf == 1 ? g.Z : g.M) + u.c_off;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
        const int32_t j = c0 + wc + b * 16 + (lane & 15);
        if (i < u.c_rows && j < u.ncols && (!u.diag || j <= i)) {
          double* cp = C + (int64_t)i * NB + j;
          const double v = u.alpha * acc[a][b][e];
          *cp = u.beta ? *cp + v : v;
        }
      }
}

// after a contraction level whose long tasks were split: each split task's
// output block (64 x 64, the contraction's blocking) gets the sum of its
// partial slots, added in slot order.  Work-group (item, y) covers rows
// 16 y .. 16 y + 15 of the item's block, thread t four consecutive columns
// 4 (t % 16) .. of row t / 16.  The item carries its whole descriptor, and
// the output's values are read beside the slots', so that a work-group waits
// for two rounds of loads; the slots' are read four slots at a time.
template <int NB>
__global__ __launch_bounds__(256) void k_backfold(const FoldItemD* __restrict__ items, double* __restrict__ Z,
                                                  double* __restrict__ M, const double* __restrict__ P) {
  const FoldItemD f = items[blockIdx.x];
  double* C = (f.c_buf == 1 ? Z : M) + f.c_off;
  const int32_t i = f.bx * CB + 16 * (int32_t)blockIdx.y + (int32_t)(threadIdx.x >> 4);
  const int32_t j = f.by * CB + 4 * (int32_t)(threadIdx.x & 15);
  if (i >= f.c_rows || j >= f.ncols || (f.diag && j > i)) return;
  double* c = C + (int64_t)i * NB + j;
  double cv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) cv[e] = c[j + e < f.ncols ? e : 0];  // columns past the tile read column j
  const int64_t slot = (int64_t)f.c_rows * NB;
  const double* p = P + f.slot_off + (int64_t)i * NB + j;  // j, NB and every offset even: 16-byte aligned pairs
  double4 sum = {0.0, 0.0, 0.0, 0.0};
  int32_t s = 0;
  for (; s + 4 <= f.nslots; s += 4) {
    double2 v[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q][0] = *reinterpret_cast<const double2*>(p + (s + q) * slot);
      v[q][1] = *reinterpret_cast<const double2*>(p + (s + q) * slot + 2);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sum.x += v[q][0].x;
      sum.y += v[q][0].y;
      sum.z += v[q][1].x;
      sum.w += v[q][1].y;
    }
  }
  for (; s < f.nslots; ++s) {
    const double2 a = *reinterpret_cast<const double2*>(p + s * slot);
    const double2 b = *reinterpret_cast<const double2*>(p + s * slot + 2);
    sum.x += a.x;
    sum.y += a.y;
    sum.z += b.x;
    sum.w += b.y;
  }
  const double add[4] = {sum.x, sum.y, sum.z, sum.w};
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (j + e < f.ncols && (!f.diag || j + e <= i)) c[e] = cv[e] + add[e];
}

// gradient of log det with respect to the input values (lower triangle of a
// symmetric matrix): gbar * Z_ij, doubled off the diagonal; NaN when the
// factorization failed
__global__ void k_logdet_grad(const double* __restrict__ Z, const int64_t* __restrict__ vmap,
                              const int8_t* __restrict__ diag, const double* __restrict__ gbar,
                              const int32_t* __restrict__ info, int64_t qnz,
                              double* __restrict__ out) {
  const double gb = gbar[0];
  const bool ok = info[0] == 0;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < qnz; i += step) {
    const double z = Z[vmap[i]];
    out[i] = ok ? gb * (diag[i] ? z : 2.0 * z) : __builtin_nan("");
  }
}

// diag(A^-1) in original numbering from the selected inverse in store
// layout: out[perm[i]] = Z_ii, NaN when the factorization failed
__global__ void k_selinv_diag(const double* __restrict__ Z, const int32_t* __restrict__ perm, int64_t np,
                              int32_t nb, const int32_t* __restrict__ info, double* __restrict__ out) {
  const bool ok = info[0] == 0;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < np; i += step) {
    const int64_t k = i / nb, r = i % nb;
    if (perm[i] >= 0) out[perm[i]] = ok ? Z[k * nb * nb + r * nb + r] : __builtin_nan("");
  }
}

__global__ __launch_bounds__(256) void k_mfma_issue(double* __restrict__ out, int32_t iters, double seed) {
  const int lane = threadIdx.x & 63;
  double a = seed + lane * 1e-3, b = seed - lane * 1e-3;
  d4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (s == 12345.678) out[blockIdx.x] = s;  // keeps the loop alive
}

// ---------------------------------------------------------------------------
// log-determinant: 2 sum log L_ii over the real rows, fixed summation order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_logdet(const double* __restrict__ store, int64_t mstride,
                                                int32_t nb, int64_t np,
                                                const int32_t* __restrict__ info,
                                                double* __restrict__ out) {
  __shared__ double part[256];
  const double* S = store + (int64_t)blockIdx.x * mstride;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < np; i += 256) {  // padding positions hold 1: log 1 = 0
    const int64_t k = i / nb, r = i % nb;
    s += log(S[k * nb * nb + r * nb + r]);
  }
  part[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[blockIdx.x] = info[blockIdx.x] ? __builtin_nan("") : 2.0 * part[0];
}

__global__ void k_info_reset(int32_t* info, int32_t count, int32_t big) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) info[i] = big;
}

// turn "no failure" (still the sentinel) into 0, and a failed grid position
// q + 1 into its column of P A P^T plus one (gcol; identity when null)
__global__ void k_info_finish(int32_t* info, int32_t count, int32_t big, int32_t* out,
                              const int32_t* __restrict__ gcol) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    int32_t v = info[i] == big ? 0 : info[i];
    if (v > 0 && gcol) v = gcol[v - 1] + 1;
    info[i] = v;
    if (out) out[i] = v;
  }
}

// ---------------------------------------------------------------------------
// factor export
// ---------------------------------------------------------------------------

__global__ void k_gather(const double* __restrict__ store, const int64_t* __restrict__ map,
                         int64_t cnt, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < cnt; i += step) out[i] = store[map[i]];
}

// ---------------------------------------------------------------------------
// solve: permute, forward and backward sweeps over block levels, unpermute
// ---------------------------------------------------------------------------

// y = P b for nrhs columns of value set blockIdx.y (y stride ystride per
// value set); perm[a] is the original index at grid position a, or -1 at a
// padding position, which gets zero
__global__ void k_perm_in(const double* __restrict__ b, const int32_t* __restrict__ perm,
                          int64_t n, int64_t np, int32_t nrhs, double* __restrict__ y, int64_t ystride) {
  b += (int64_t)blockIdx.y * n * nrhs;
  y += (int64_t)blockIdx.y * ystride;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np * nrhs) return;
  int64_t r = i / np, a = i % np;
  const int32_t o = perm[a];
  y[i] = o >= 0 ? b[r * n + o] : 0.0;
}

// x = P^T y; NaN throughout when the factorization that the sweeps used
// failed (info of the first value set non-zero)
__global__ void k_perm_out(const double* __restrict__ y, const int32_t* __restrict__ perm,
                           const int32_t* __restrict__ info, int64_t n, int64_t np, int32_t nrhs,
                           double* __restrict__ b, int64_t ystride) {
  b += (int64_t)blockIdx.y * n * nrhs;
  y += (int64_t)blockIdx.y * ystride;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np * nrhs) return;
  int64_t r = i / np, a = i % np;
  const int32_t o = perm[a];
  if (o >= 0) b[r * n + o] = info[blockIdx.y] != 0 ? __builtin_nan("") : y[i];
}

// Both sweeps run level by level over the blocks of the tile grid and read L
// once per group of up to SR right-hand sides (rhs-major in y, stride np).
// Launch q of a sweep holds two kinds of work items.  A step item owns a
// block of level q: it subtracts the products of the tiles that feed the
// block from blocks of level q - 1 (forward: b_m -= L_mk y_k; backward:
// y_k -= L_mk^T x_m), then solves the block's diagonal block with its
// right-hand sides held in LDS throughout.  A panel item subtracts the
// level q - 1 products for a 64-row (forward) or 64-column (backward) chunk
// of a block of a later level, in place in y.  A block of level q depends on
// at least one block of level q - 1 and all its other contributions come
// from earlier launches, so one launch per level suffices.  Every item runs
// through its tiles in a fixed order: no races, no atomics, and results are
// reproducible bit for bit.  Diagonal blocks are solved 32 rows at a time
// with the inverses of the 32 x 32 diagonal blocks of L that the
// factorization keeps (dinv).  The kernels are compiled for R = 1 (a single
// right-hand side) and R = SR (a group of 2 .. 8, the unused columns zero);
// every column is computed by the same operations in the same order whatever
// R, so its result does not depend on how many columns share the pass.
constexpr int SR = 8;      // right-hand sides per sweep
constexpr int SCH = 64;    // block rows of a forward panel chunk
constexpr int SBC = 64;    // columns of a backward panel chunk

// sum of each value over the 8 adjacent lanes of a row group, left in every
// lane of the group: ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7)), a_j
// the value of lane j (every lane forms the same sums, addition commuting)
template <int R>
__device__ __forceinline__ void rowsum8(double (&a)[R]) {
#pragma unroll
  for (int c = 0; c < R; ++c) {
    a[c] += __shfl_xor(a[c], 1);
    a[c] += __shfl_xor(a[c], 2);
    a[c] += __shfl_xor(a[c], 4);
  }
}

// the same sum of v[0], v[st], .., v[7 st] in one thread
__device__ __forceinline__ double tree8(const double* v, int st) {
  return ((v[0] + v[st]) + (v[2 * st] + v[3 * st])) + ((v[4 * st] + v[5 * st]) + (v[6 * st] + v[7 * st]));
}

// one 32-row diagonal step after the K-split parts: s = r_J - (sum of the 8
// parts of each entry), then r_J = D s (forward, D_J) or D^T s (backward),
// each entry's 32 products taken as 8 chains of 4 (q = z, z + 8, z + 16,
// z + 24) summed as above.  R = 1 keeps the parts in the 8 lanes of a row and
// sums by shuffles (three barriers per step); wider R, whose entries already
// fill the work-group, goes through LDS with one thread per (entry, column).
// Both forms do the same arithmetic, so a column's result does not depend on
// R.  acc holds this thread's parts (row = tid / 8, lane sub = tid % 8);
// enters after the step's staging barrier, ends with a barrier.
template <int R, bool TRANS>
__device__ __forceinline__ void diag_step(double (&acc)[R], double* rJ, double* s, double* part,
                                          const double* Ds) {
  const int tid = threadIdx.x, row = tid >> 3, sub = tid & 7;
  auto dv = [&](int i, int q) { return TRANS ? Ds[q * PLD + i] : Ds[i * PLD + q]; };
  if constexpr (R == 1) {
    rowsum8<1>(acc);
    if (sub == 0) s[row] = rJ[row] - acc[0];
    __syncthreads();
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) a = fma(dv(row, sub + 8 * t), s[sub + 8 * t], a);
    double b[1] = {a};
    rowsum8<1>(b);
    if (sub == 0) rJ[row] = b[0];
    __syncthreads();
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) part[(row * 8 + sub) * R + c] = acc[c];
    __syncthreads();
    if (tid < PW * R) {
      const int i = tid / R, c = tid % R;
      s[tid] = rJ[tid] - tree8(part + i * 8 * R + c, R);
    }
    __syncthreads();
    if (tid < PW * R) {
      const int i = tid / R, c = tid % R;
      double ch[8];
#pragma unroll
      for (int z = 0; z < 8; ++z) {
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) a = fma(dv(i, z + 8 * t), s[(z + 8 * t) * R + c], a);
        ch[z] = a;
      }
      rJ[tid] = tree8(ch, 1);
    }
    __syncthreads();
  }
}

// forward products for rows i0 .. i0 + 32 H - 1 (tiles [t0, t1)): for each row i,
// sum over the tiles (m, k) of L_mk(q(i)) y_k, q(i) the tile's stored row of
// block row i (its inverse row map; identity when the tile is full), handed
// to put(i, c, value) for right-hand side c.  8 lanes per row over
// interleaved column pairs, H rows per thread, reduced by shuffles.  A
// tile's rows are read into registers before y_k is gathered into ys, so the
// loads of both overlap.
template <int NB, int R, int H, class Put>
__device__ __forceinline__ void sfwd_panel(int32_t i0, int32_t t0, int32_t t1, const TileD* __restrict__ tlist,
                                           const int32_t* __restrict__ maps,
                                           const double* __restrict__ S, const double* __restrict__ y,
                                           int64_t np, int32_t nrhs, double* ys, Put put) {
  constexpr int NC = NB / 16;  // column pairs per lane
  const int tid = threadIdx.x;
  const int j = tid & 7, rl = tid >> 3;  // lane of the row group, row of the pass
  double acc[H][R];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[h][c] = 0.0;
  for (int32_t z = t0; z < t1; ++z) {
    const TileD tl = tlist[z];
    double2 lv[H][NC];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int i = i0 + rl + 32 * h;
      const int32_t q = i >= NB ? -1 : (tl.imap < 0 ? i : maps[tl.imap + i]);
      const double* Lr = S + tl.off + (int64_t)(q < 0 ? 0 : q) * NB + 2 * j;
#pragma unroll
      for (int u = 0; u < NC; ++u)
        lv[h][u] = q >= 0 ? *reinterpret_cast<const double2*>(Lr + 16 * u) : make_double2(0.0, 0.0);
    }
    __syncthreads();  // ys is free
    for (int x = tid; x < NB * R; x += 256) {
      const int col = x / R, c = x % R;
      ys[x] = c < nrhs ? y[(int64_t)c * np + (int64_t)tl.k * NB + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int col = 2 * j + 16 * u;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double y0 = ys[col * R + c], y1 = ys[(col + 1) * R + c];
#pragma unroll
        for (int h = 0; h < H; ++h) acc[h][c] = fma(lv[h][u].x, y0, fma(lv[h][u].y, y1, acc[h][c]));
      }
    }
  }
#pragma unroll
  for (int h = 0; h < H; ++h) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      acc[h][c] += __shfl_xor(acc[h][c], 1);
      acc[h][c] += __shfl_xor(acc[h][c], 2);
      acc[h][c] += __shfl_xor(acc[h][c], 4);
    }
    double mine = acc[h][0];  // lane j of the row group keeps right-hand side j
#pragma unroll
    for (int c = 1; c < R; ++c) mine = j == c ? acc[h][c] : mine;
    const int i = i0 + rl + 32 * h;
    if (i < NB && j < nrhs) put(i, j, mine);
  }
}

// forward products of a step item whose block has at most 128 rows: for
// each tile (m, k) in order, each stored row q takes r(rows(q)) -= L_mk(q)
// y_k.  A tile's stored rows are distinct block rows, so a tile's updates do
// not collide, and the tiles follow one another behind barriers.  Reading
// the stored rows directly (their block rows loaded beside them) keeps the
// tile's row map off the load chain.  Layout as in sfwd_panel, NB / 32 rows
// per thread.
template <int NB, int R>
__device__ __forceinline__ void sfwd_step_products(int32_t t0, int32_t t1, const TileD* __restrict__ tlist,
                                                   const int32_t* __restrict__ rows,
                                                   const double* __restrict__ S, const double* __restrict__ y,
                                                   int64_t np, int32_t nrhs, double* ys, double* r) {
  constexpr int NC = NB / 16, H = NB / 32;
  const int tid = threadIdx.x;
  const int j = tid & 7, rl = tid >> 3;
  for (int32_t z = t0; z < t1; ++z) {
    const TileD tl = tlist[z];
    double2 lv[H][NC];
    int32_t dst[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int q = rl + 32 * h;
      const bool ok = q < tl.cnt;
      dst[h] = ok ? rows[tl.roff + q] : -1;
      const double* Lr = S + tl.off + (int64_t)(ok ? q : 0) * NB + 2 * j;
#pragma unroll
      for (int u = 0; u < NC; ++u)
        lv[h][u] = ok ? *reinterpret_cast<const double2*>(Lr + 16 * u) : make_double2(0.0, 0.0);
    }
    __syncthreads();  // ys is free, the previous tile's updates are done
    for (int x = tid; x < NB * R; x += 256) {
      const int col = x / R, c = x % R;
      ys[x] = c < nrhs ? y[(int64_t)c * np + (int64_t)tl.k * NB + col] : 0.0;
    }
    __syncthreads();
    double acc[H][R];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int c = 0; c < R; ++c) acc[h][c] = 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int col = 2 * j + 16 * u;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double y0 = ys[col * R + c], y1 = ys[(col + 1) * R + c];
#pragma unroll
        for (int h = 0; h < H; ++h) acc[h][c] = fma(lv[h][u].x, y0, fma(lv[h][u].y, y1, acc[h][c]));
      }
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
        acc[h][c] += __shfl_xor(acc[h][c], 1);
        acc[h][c] += __shfl_xor(acc[h][c], 2);
        acc[h][c] += __shfl_xor(acc[h][c], 4);
      }
      double mine = acc[h][0];  // lane j of the row group keeps right-hand side j
#pragma unroll
      for (int c = 1; c < R; ++c) mine = j == c ? acc[h][c] : mine;
      if (dst[h] >= 0 && j < nrhs) r[dst[h] * R + j] -= mine;
    }
  }
}

// registers that carry a diagonal step's block row (forward) or block
// column (backward) of L_kk and its 32 x 32 inverse from global memory to LDS
template <int NB, class V>
struct DiagFetch {
  static constexpr int N = NB > PW ? (NB - PW) / (sizeof(V) / 8 * 8) : 1;
  V pf[N];
  double4 pd;
};

// forward step J's block row of L_kk (left of the diagonal block) and inverse
// into registers: 32 rows x 8 threads, interleaved column pairs
template <int NB>
__device__ __forceinline__ void sfwd_fetch(int32_t k, int J, const double* __restrict__ S,
                                           const double* __restrict__ dinv, DiagFetch<NB, double2>& f) {
  const int tid = threadIdx.x, row = tid >> 3, sub = tid & 7;
  const int w = J * PW;
  const double* src = S + (int64_t)k * NB * NB + (int64_t)(w + row) * NB;
#pragma unroll
  for (int q = 0; q < DiagFetch<NB, double2>::N; ++q)
    if (2 * sub + 16 * q < w) f.pf[q] = *reinterpret_cast<const double2*>(src + 2 * sub + 16 * q);
  f.pd = *reinterpret_cast<const double4*>(dinv + (int64_t)k * NB * PW + J * PW * PW + row * PW + 4 * sub);
}

// r <- L_kk^-1 r (r[i * R + c] in LDS): per 32-row block J, the block row of
// L_kk left of the diagonal block and the block's inverse are staged in LDS
// (coalesced), then s = r_J - L_(J,<J) r_(<J) with the K range split over
// the 8 adjacent lanes of a row (each keeping all right-hand sides), and
// r_J = D_J s (diag_step).  Steps alternate between two register
// sets, step J + 2's rows being read during step J; steps 0 and 1 must be in
// f0 and f1 on entry (sfwd_fetch).  Ends with a barrier.
template <int NB, int R>
__device__ __forceinline__ void sfwd_diag(int32_t k, const double* __restrict__ S, const double* __restrict__ dinv,
                                          DiagFetch<NB, double2>& f0, DiagFetch<NB, double2>& f1, double* r,
                                          double* s, double* part, double* Ls, double* Ds) {
  constexpr int LW = NB - PW + 1;
  constexpr int NPF = DiagFetch<NB, double2>::N;
  const int tid = threadIdx.x;
  const int row = tid >> 3, sub = tid & 7;  // staging and K-split layout: 32 rows x 8
#pragma unroll
  for (int J = 0; J < NB / PW; ++J) {
    DiagFetch<NB, double2>& f = (J & 1) ? f1 : f0;
    const double2* pf = f.pf;
    const double4 pd = f.pd;
    const int w = J * PW;
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int col = 2 * sub + 16 * q;
      if (col < w) {
        Ls[row * LW + col] = pf[q].x;
        Ls[row * LW + col + 1] = pf[q].y;
      }
    }
    Ds[row * PLD + 4 * sub] = pd.x;
    Ds[row * PLD + 4 * sub + 1] = pd.y;
    Ds[row * PLD + 4 * sub + 2] = pd.z;
    Ds[row * PLD + 4 * sub + 3] = pd.w;
    __syncthreads();
    if (J + 2 < NB / PW) sfwd_fetch<NB>(k, J + 2, S, dinv, f);
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int p = sub; p < w; p += 8) {
      const double l = Ls[row * LW + p];
#pragma unroll
      for (int c = 0; c < R; ++c) acc[c] = fma(l, r[p * R + c], acc[c]);
    }
    diag_step<R, false>(acc, r + w * R, s, part, Ds);
  }
}

// one forward launch: items [4 * b] = (block, first row, t0, t1), tiles
// [t0, t1) of tlist; the first nstep items are step items (first row unused),
// the rest panel chunks
template <int NB, int R>
__global__ __launch_bounds__(256) void k_sfwd_step(const int32_t* __restrict__ items, int32_t nstep,
                                                   const TileD* __restrict__ tlist,
                                                   const int32_t* __restrict__ maps,
                                                   const int32_t* __restrict__ rows,
                                                   const double* __restrict__ S,
                                                   const double* __restrict__ dinv,
                                                   double* __restrict__ y, int64_t np, int32_t nrhs,
                                                   int64_t mstride, int64_t dstride, int64_t ystride) {
  S += (int64_t)blockIdx.y * mstride;  // value set blockIdx.y: its factor, inverses and right-hand sides
  dinv += (int64_t)blockIdx.y * dstride;
  y += (int64_t)blockIdx.y * ystride;
  constexpr int LW = NB - PW + 1;
  __shared__ double r[NB * R];
  __shared__ double ys[(R == 1 ? NB : 256) * R];  // the gathered y_k of the products, then
                                                  // the diagonal steps' parts (R > 1)
  __shared__ double s[PW * R];
  __shared__ double Ls[PW * LW];
  __shared__ double Ds[PW * PLD];
  const int32_t m = items[4 * blockIdx.x], i0 = items[4 * blockIdx.x + 1];
  const int32_t t0 = items[4 * blockIdx.x + 2], t1 = items[4 * blockIdx.x + 3];
  double* ym = y + (int64_t)m * NB;
  if ((int32_t)blockIdx.x >= nstep) {
    sfwd_panel<NB, R, SCH / 32>(i0, t0, t1, tlist, maps, S, y, np, nrhs, ys,
                                [&](int i, int c, double v) { ym[(int64_t)c * np + i] -= v; });
    return;
  }
  DiagFetch<NB, double2> f0, f1;  // the diagonal phase's first loads overlap the products
  sfwd_fetch<NB>(m, 0, S, dinv, f0);
  if (NB / PW > 1) sfwd_fetch<NB>(m, 1, S, dinv, f1);
  const int tid = threadIdx.x;
  for (int x = tid; x < NB * R; x += 256) {
    const int i = x / R, c = x % R;
    r[x] = c < nrhs ? ym[(int64_t)c * np + i] : 0.0;
  }
  // up to n_b 128 one pass over the tiles' stored rows, else 64-row chunks
  auto put_r = [&](int i, int c, double v) { r[i * R + c] -= v; };
  if (t1 > t0) {
    if constexpr (NB <= 128) {
      sfwd_step_products<NB, R>(t0, t1, tlist, rows, S, y, np, nrhs, ys, r);
    } else {
      for (int c0 = 0; c0 < NB; c0 += SCH)
        sfwd_panel<NB, R, SCH / 32>(c0, t0, t1, tlist, maps, S, y, np, nrhs, ys, put_r);
    }
  }
  __syncthreads();
  sfwd_diag<NB, R>(m, S, dinv, f0, f1, r, s, ys, Ls, Ds);
  for (int x = tid; x < NB * R; x += 256) {
    const int i = x / R, c = x % R;
    if (c < nrhs) ym[(int64_t)c * np + i] = r[x];
  }
}

// backward panel chunk (columns j0 .. j0 + CW - 1 of block k, tiles [t0, t1)):
// for each column j, sum over the tiles (m, k) of (L_mk^T x_m)(j), handed to
// put(x, value) with x = (j - j0) * R + c.  A thread owns two adjacent
// columns and every SH-th stored row; its rows of a tile are read into
// registers before the entries of x_m at the tile's active rows are gathered
// into xg.  The SH row shares are summed in red in a fixed order.  Ends with
// a barrier.
template <int NB, int CW_>
struct SbwdShape {
  static constexpr int CW = CW_;       // columns per pass
  static constexpr int CP = CW / 2;    // column pairs
  static constexpr int SH = 256 / CP;  // row shares
  static constexpr int NQ = NB / SH;   // stored rows per thread at most
};
constexpr int sbwd_chunk(int nb) { return nb < SBC ? nb : SBC; }

template <int NB, int R, int CW_, class Put>
__device__ __forceinline__ void sbwd_panel(int32_t j0, int32_t t0, int32_t t1, const TileD* __restrict__ tlist,
                                           const int32_t* __restrict__ rows,
                                           const double* __restrict__ S, const double* __restrict__ y,
                                           int64_t np, int32_t nrhs, double* xg, double* red, Put put) {
  constexpr int CW = SbwdShape<NB, CW_>::CW, CP = SbwdShape<NB, CW_>::CP;
  constexpr int SH = SbwdShape<NB, CW_>::SH, NQ = SbwdShape<NB, CW_>::NQ;
  const int tid = threadIdx.x;
  const int cp = tid % CP, sh = tid / CP;
  double acc[2][R];
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[e][c] = 0.0;
  for (int32_t z = t0; z < t1; ++z) {
    const TileD tl = tlist[z];
    const double* P = S + tl.off + j0 + 2 * cp;
    double2 lv[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int q = sh + SH * u;
      lv[u] = q < tl.cnt ? *reinterpret_cast<const double2*>(P + (int64_t)q * NB) : make_double2(0.0, 0.0);
    }
    __syncthreads();  // xg is free
    for (int x = tid; x < tl.cnt * R; x += 256) {
      const int q = x / R, c = x % R;
      xg[x] = c < nrhs ? y[(int64_t)c * np + (int64_t)tl.m * NB + rows[tl.roff + q]] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int q = sh + SH * u;
      if (q < tl.cnt) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const double xv = xg[q * R + c];
          acc[0][c] = fma(lv[u].x, xv, acc[0][c]);
          acc[1][c] = fma(lv[u].y, xv, acc[1][c]);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int c = 0; c < R; ++c) red[(sh * CW + 2 * cp + e) * R + c] = acc[e][c];
  __syncthreads();
  for (int x = tid; x < CW * R; x += 256) {
    double v = 0.0;
    for (int z = 0; z < SH; ++z) v += red[z * CW * R + x];
    if (x % R < nrhs) put(x, v);
  }
  __syncthreads();
}

// backward step J's block column of L_kk (below the diagonal block) and
// inverse into registers: 32 rows x 8 threads, four columns each
template <int NB>
__device__ __forceinline__ void sbwd_fetch(int32_t k, int J, const double* __restrict__ S,
                                           const double* __restrict__ dinv, DiagFetch<NB, double4>& f) {
  const int tid = threadIdx.x, row = tid >> 3, sub = tid & 7;
  const int p0 = (J + 1) * PW, h = NB - p0;
  const double* L = S + (int64_t)k * NB * NB;
#pragma unroll
  for (int q = 0; q < DiagFetch<NB, double4>::N; ++q)
    if (row + 32 * q < h)
      f.pf[q] = *reinterpret_cast<const double4*>(L + (int64_t)(p0 + row + 32 * q) * NB + J * PW + 4 * sub);
  f.pd = *reinterpret_cast<const double4*>(dinv + (int64_t)k * NB * PW + J * PW * PW + row * PW + 4 * sub);
}

// r <- L_kk^-T r (r[i * R + c] in LDS): per 32-row block J from the last, the
// block column of L_kk below the diagonal block and the block's inverse are
// staged in LDS (coalesced), then s = r_J - L_(>J,J)^T r_(>J) with the row
// range split over the 8 adjacent lanes of a column, and r_J = D_J^T s
// (diag_step).  Steps alternate between two register sets, step J - 2's
// rows being read during step J; the last two steps' must be in f0 (the last)
// and f1 on entry (sbwd_fetch).  Ends with a barrier.
template <int NB, int R>
__device__ __forceinline__ void sbwd_diag(int32_t k, const double* __restrict__ S, const double* __restrict__ dinv,
                                          DiagFetch<NB, double4>& f0, DiagFetch<NB, double4>& f1, double* r,
                                          double* s, double* part, double* Lc, double* Ds) {
  constexpr int NPF = DiagFetch<NB, double4>::N;
  constexpr int NJ = NB / PW;
  const int tid = threadIdx.x;
  const int row = tid >> 3, sub = tid & 7;
#pragma unroll
  for (int J = NJ - 1; J >= 0; --J) {
    DiagFetch<NB, double4>& f = ((NJ - 1 - J) & 1) ? f1 : f0;
    const double4* pf = f.pf;
    const double4 pd = f.pd;
    const int p0 = (J + 1) * PW, h = NB - p0;  // rows below the diagonal block
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int p = row + 32 * q;
      if (p < h) {
        Lc[p * PLD + 4 * sub] = pf[q].x;
        Lc[p * PLD + 4 * sub + 1] = pf[q].y;
        Lc[p * PLD + 4 * sub + 2] = pf[q].z;
        Lc[p * PLD + 4 * sub + 3] = pf[q].w;
      }
    }
    Ds[row * PLD + 4 * sub] = pd.x;
    Ds[row * PLD + 4 * sub + 1] = pd.y;
    Ds[row * PLD + 4 * sub + 2] = pd.z;
    Ds[row * PLD + 4 * sub + 3] = pd.w;
    __syncthreads();
    if (J > 1) sbwd_fetch<NB>(k, J - 2, S, dinv, f);
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int p = sub; p < h; p += 8) {
      const double l = Lc[p * PLD + row];
#pragma unroll
      for (int c = 0; c < R; ++c) acc[c] = fma(l, r[(p0 + p) * R + c], acc[c]);
    }
    diag_step<R, true>(acc, r + J * PW * R, s, part, Ds);
  }
}

// one backward launch: items [4 * b] = (block, first column, t0, t1), tiles
// [t0, t1) of tlist; the first nstep items are step items (first column
// unused), the rest panel chunks.  The diagonal phase's LDS (s | parts |
// Lc | Ds) and the products' LDS (xg | red) share one buffer.
template <int NB, int R>
struct SbwdLds {
  static constexpr int DIAG = PW * R + (R == 1 ? 0 : PW * 8 * R) + (NB - PW) * PLD + 1 + PW * PLD;
  static constexpr int PROD = NB * R + 512 * R;  // xg, then SH x CW x R partial sums
  static constexpr int SIZE = DIAG > PROD ? DIAG : PROD;
};

template <int NB, int R>
__global__ __launch_bounds__(256) void k_sbwd_step(const int32_t* __restrict__ items, int32_t nstep,
                                                   const TileD* __restrict__ tlist,
                                                   const int32_t* __restrict__ rows,
                                                   const double* __restrict__ S,
                                                   const double* __restrict__ dinv,
                                                   double* __restrict__ y, int64_t np, int32_t nrhs,
                                                   int64_t mstride, int64_t dstride, int64_t ystride) {
  S += (int64_t)blockIdx.y * mstride;  // value set blockIdx.y: its factor, inverses and right-hand sides
  dinv += (int64_t)blockIdx.y * dstride;
  y += (int64_t)blockIdx.y * ystride;
  __shared__ double r[NB * R];
  __shared__ double sm[SbwdLds<NB, R>::SIZE];
  double* xg = sm;
  double* red = sm + NB * R;
  const int32_t k = items[4 * blockIdx.x], j0 = items[4 * blockIdx.x + 1];
  const int32_t t0 = items[4 * blockIdx.x + 2], t1 = items[4 * blockIdx.x + 3];
  double* yk = y + (int64_t)k * NB;
  if ((int32_t)blockIdx.x >= nstep) {
    sbwd_panel<NB, R, sbwd_chunk(NB)>(j0, t0, t1, tlist, rows, S, y, np, nrhs, xg, red,
                                      [&](int x, double v) { yk[(int64_t)(x % R) * np + j0 + x / R] -= v; });
    return;
  }
  DiagFetch<NB, double4> f0, f1;  // the diagonal phase's first loads overlap the products
  sbwd_fetch<NB>(k, NB / PW - 1, S, dinv, f0);
  if (NB / PW > 1) sbwd_fetch<NB>(k, NB / PW - 2, S, dinv, f1);
  const int tid = threadIdx.x;
  for (int x = tid; x < NB * R; x += 256) {
    const int i = x / R, c = x % R;
    r[x] = c < nrhs ? yk[(int64_t)c * np + i] : 0.0;
  }
  // up to n_b 128 one pass over the tiles covers every column, else chunks
  if (t1 > t0) {
    if constexpr (NB <= 128) {
      sbwd_panel<NB, R, NB>(0, t0, t1, tlist, rows, S, y, np, nrhs, xg, red,
                            [&](int x, double v) { r[x] -= v; });
    } else {
      for (int c0 = 0; c0 < NB; c0 += SBC)
        sbwd_panel<NB, R, SBC>(c0, t0, t1, tlist, rows, S, y, np, nrhs, xg, red,
                               [&](int x, double v) { r[c0 * R + x] -= v; });
    }
  }
  __syncthreads();
  double* s = sm;
  double* part = s + PW * R;
  double* Lc = part + (R == 1 ? 0 : PW * 8 * R);
  double* Ds = Lc + (NB - PW) * PLD + 1;
  sbwd_diag<NB, R>(k, S, dinv, f0, f1, r, s, part, Lc, Ds);
  for (int x = tid; x < NB * R; x += 256) {
    const int i = x / R, c = x % R;
    if (c < nrhs) yk[(int64_t)c * np + i] = r[x];
  }
}

}  // namespace stc
