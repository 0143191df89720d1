// analyse.hpp -- host-side symbolic analysis and static execution plan of the
// structure-adaptive tile Cholesky (arXiv 2609.29765, Sec. 3 and Sec. 5.1-5.3).
//
// Symbolic part: dense-row set-aside and ordering (Sec. 3), elimination tree
// and exact fill pattern of L, uniform n_b tile grid with the active rows of
// every off-diagonal tile (the active columns of the stored transpose, Sec.
// 4.1), full/contiguous flags and diagonal half-width kd (Sec. 4.2-4.3,
// Sec. 5.2 "Per-tile metadata"), selector features and route (Sec. 5.1), and
// the ordered task list of Algorithm 1.
//
// Plan part (device-facing): tile-store layout, value map from input entries
// to the store, per-task gather maps (the transpose of the paper's per-task
// scatter, Sec. 4.2 and Sec. 5.2 "Per-task scatter"), and a level schedule
// whose edges are those Algorithm 2 synchronises through its progress matrix.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace stc {

enum Ordering { kNatural = 0, kRcm = 1, kNd = 2, kAuto = 3, kGiven = 4 };
enum Mode { kModeAuto = 0, kModeDense = 1, kModeSemisparse = 2 };
enum Route { kRouteDense = 0, kRouteSemisparse = 1, kRouteSupernodal = 2 };
enum Op { kPotrf = 1, kSyrk = 2, kTrsm = 3, kGemm = 4 };

struct TileInfo {
  int32_t m, k;      // block row, block column (m > k)
  int32_t cnt;       // stored active rows
  int32_t true_cnt;  // active rows of the pattern
  int8_t contig;     // active rows form one interval
  int64_t roff;      // offset of this tile's rows in Symbolic::rows
};

struct Symbolic {
  int64_t n = 0, qnz = 0;
  std::vector<int64_t> qp;
  std::vector<int32_t> qi;
  std::vector<int32_t> perm, iperm;  // perm[new] = old
  int32_t ndense = 0;
  int32_t method = 0;
  std::vector<int32_t> parent;       // elimination tree of P A P^T
  std::vector<int64_t> lp;           // pattern of L, CSC, rows ascending
  std::vector<int32_t> li;
  int64_t lnz = 0;
  int32_t nb = 64, NT = 0, mode = 0, route = 0;
  std::vector<TileInfo> tiles;       // k ascending, then m ascending
  std::vector<int32_t> rows;         // active rows, local to block m
  std::vector<int32_t> kd;           // per diagonal tile
  double phi = 0, rho = 0, sigma = 0;
  int64_t tact = 0;
  std::vector<int32_t> tasks;        // 4 ints per task: op, m, k, n (-1 unused)
  // tile grid aligned to the elimination tree (align_tiles): column j of
  // P A P^T sits at position pos[j] of a padded order npad, tile t covering
  // positions [t nb, (t + 1) nb); empty pos means position = column
  int64_t align = 0;                 // minimum subtree size of an aligned start (0: uniform grid)
  int64_t npad = 0;
  std::vector<int64_t> pos;
};

// position of column j in the tile grid
inline int64_t grid_pos(const Symbolic& s, int64_t j) { return s.pos.empty() ? j : s.pos[(size_t)j]; }

// Validate a lower CSC pattern; returns 0 or a negative STC_ERR_* code.
int check_pattern(int64_t n, const int64_t* cp, const int32_t* ri, std::string* why);

// Full symbolic analysis. method in Ordering; mode in Mode; perm read for kGiven.
int analyse(int64_t n, const int64_t* cp, const int32_t* ri, int method, int nb, int mode,
            const int32_t* perm, Symbolic* out, std::string* why);

// Re-tile an analysed pattern on a grid aligned to its elimination tree:
// every subtree of at least min_subtree columns whose columns are
// consecutive starts on a tile boundary (the columns before it are padded
// to the boundary).  Tiles and tasks are rebuilt on that grid; the
// features, the route and the storage mode stay those of the uniform grid.
void align_tiles(Symbolic* s, int64_t min_subtree);

// ---------------------------------------------------------------------------
// execution plan
// ---------------------------------------------------------------------------

// One contribution to an output tile: C -= A_rows(a) * B_rows(b)^T, where the
// A operand rows are gathered through rowmap (identity if < 0) and the B
// operand rows through the inverse active-row map of tile b (identity if the
// tile is full).  For a diagonal output (SYRK) a == b.
struct Contrib {
  int64_t a_off, b_off;  // store offsets (doubles) of the operand tiles
  int32_t a_rows, b_rows;
  int32_t rowmap;        // offset into Plan::maps, or -1 for identity
  int32_t colmap;        // offset into Plan::maps, or -1 for identity
};

// A fused update of one output tile by all its contributions (the SYRK or
// GEMM tasks of Algorithm 1 that write it), accumulated in registers.
struct UpdTask {
  int64_t c_off;          // output tile offset
  int32_t c_rows;         // output rows (stored active rows, or h for a diagonal)
  int32_t diag;           // 1 for a diagonal tile (lower blocks only)
  int32_t c_begin, c_end; // contributions [c_begin, c_end)
  int32_t level = 0;
  int32_t big = 0;        // 128 x 128 blocks (else 64 x 64)
  int32_t partner = -1;   // for an early group: the tile's last group
  int32_t nsplit = 1;     // K-step stream split over this many work-groups
  int64_t part_off = 0;   // partial slots written when nsplit > 1
  int64_t in_part_off = 0;
  int32_t in_npart = 0;   // partial slots folded in by this task
};

struct TrsmTask {
  int64_t x_off;   // panel tile offset
  int64_t l_off;   // diagonal tile offset
  int32_t rows;    // stored rows of the panel tile
  int32_t k;       // block column
};

struct Level {
  std::vector<int32_t> big_items;   // quads: task, block row, block col, part (128 blocks)
  std::vector<int32_t> upd_items;   // quads: task, block row, block col, part (64 blocks)
  int32_t big_last = 0, upd_last = 0;  // leading items of each list that belong to last groups
  std::vector<int32_t> potrf;       // block columns
  std::vector<int32_t> trsm_items;  // pairs: trsm task, row block
  double flops = 0;                 // tile-algorithmic flops of the level's tasks
  double flops_potrf = 0, flops_upd = 0, flops_trsm = 0;  // the same, by kernel
};

struct Plan {
  int32_t nb = 64, NT = 0;
  int64_t wg_slots = 448;  // concurrent update work-groups the split balances for
  int32_t max_split = 64;  // most work-groups one early group's K stream is split over
  int32_t fold_pct = 100;  // weight of folding a partial slot in the split's cost model, percent of the measured
  int32_t bm = 64;          // small update block (rows and columns)
  int64_t parts = 0;        // doubles of partial-sum slots per value set
  int32_t br = 32;          // rows per TRSM work item
  int64_t store = 0;        // doubles per value set
  std::vector<int64_t> tile_off;    // per off-diagonal tile
  std::vector<int64_t> vmap;        // input entry -> store offset
  std::vector<int64_t> lmap;        // L entry (CSC order) -> store offset
  std::vector<int32_t> maps;        // gather maps
  std::vector<int32_t> diag_h;      // real rows of each diagonal tile
  std::vector<int32_t> tile_imap;   // per off-diagonal tile: offset in maps of its inverse row map
                                    // (block row -> stored row, -1 if absent), or -1 when full
  std::vector<Contrib> contribs;
  std::vector<UpdTask> upd;
  std::vector<TrsmTask> trsm;
  std::vector<Level> levels;
  // solve schedule: owner-computes block rows (forward) / block columns (back)
  std::vector<int32_t> row_tiles_ptr, row_tiles;  // tiles of block row m (n < m)
  std::vector<int32_t> col_tiles_ptr, col_tiles;  // tiles of block column k (m > k)
  std::vector<int32_t> fwd_level_ptr, fwd_level_blk;
  std::vector<int32_t> bwd_level_ptr, bwd_level_blk;
  double flops_tile = 0;    // tile-algorithmic flops of one factorization
  double flops_update = 0;  // of which SYRK + GEMM contributions
  double flops_potrf = 0;
  double flops_trsm = 0;
  double flops_exact = 0;   // sum_j c_j^2, c_j = entries of column j of L
  double bytes_update = 0;  // operand rows read + output tiles read and written
};

// wg_slots: concurrent update work-groups the per-level split of long
// contribution ranges is balanced for (0 = default_wg_slots(n_b))
int64_t default_wg_slots(int nb);
int build_plan(const Symbolic& s, int bm, int br, int64_t wg_slots, Plan* p, std::string* why, int max_split = 0,
               int fold_pct = 0);

// The kernels of the level schedule as a dependency graph, in place of a
// barrier between consecutive levels: node (level, kind) with kind 0 POTRF,
// 1 the early groups' updates, 2 TRSM, 3 the last groups' updates, for every
// non-empty kernel, in level order.  A node
// depends on the earlier nodes that last wrote what it reads (a tile, a
// diagonal tile with its 32 x 32 inverses, a split task's partial slots) and
// on those that last wrote or since read what it writes -- the edges
// Algorithm 2 waits for through its progress matrix -- transitively reduced.
struct KernelNode {
  int32_t level, kind;
  std::vector<int32_t> deps;
};
void kernel_dag(const Plan& p, std::vector<KernelNode>* out);

// Reverse mode of log det through the factorization.  For the logdet
// cotangent the adjoint of the blocked Cholesky restricted to pattern(L) is
// the selected inverse Z = (P A P^T)^-1 on pattern(L); it is computed by the
// blocked Takahashi recurrence over the tile DAG in reverse:
//   G_k = L_kk^-1, M_mk = L_mk G_k, H_k = G_k^T G_k,
//   Z_ik = - sum_{m in C_k} Z_im M_mk          (i in C_k, rows R_ik)
//   Z_kk = H_k - sum_{m in C_k} M_mk^T Z_mk
// with C_k the non-empty tiles below diagonal tile k.
struct ConTerm {
  int64_t a_off, b_off;
  int32_t a_buf, a_mode, a_rmap, a_qmap;
  int32_t b_buf, b_qmap, K;
};

struct ConTask {
  int64_t c_off;
  int32_t c_buf, c_rows, ncols, diag;
  int32_t t_begin, t_end;
  int32_t beta;
  double alpha;
};

// A task whose terms are split over several work-group sets: its first part
// writes the output tile as the task would, part s > 0 writes alpha times its
// own terms' sum into partial slot s - 1 (c_rows x n_b doubles, row stride
// n_b, starting at slot_off), and after the level's contraction kernel a fold
// kernel adds the slots, in slot order, to the output.
struct FoldTask {
  int64_t c_off;
  int32_t c_buf, c_rows, ncols, diag;
  int64_t slot_off;
  int32_t nslots;
};

struct BackPlan {
  std::vector<ConTerm> terms;
  std::vector<ConTask> tasks;
  std::vector<std::vector<int32_t>> level_items;  // per level: task, block row, block col
  std::vector<int32_t> trtri_items;               // level 0: pairs (k, block column)
  std::vector<int8_t> diagflag;                   // input entry is a diagonal entry
  std::vector<FoldTask> folds;
  std::vector<std::vector<int32_t>> fold_items;   // per level: fold, block row, block col
  int64_t slots = 0;  // doubles of partial-slot scratch, reused level after level
  double flops = 0;
};

int build_backward(const Symbolic& s, Plan* p, BackPlan* b, std::string* why);

// Plan::lmap (the store offset of every entry of L, for the host-side factor
// and selected-inverse exports) from the tiles and their store offsets.
void build_lmap(const Symbolic& s, Plan* p);

// The analysed state as a byte stream and back (persist.cpp): magic, format
// version, type sizes, the three structures (Plan::lmap left out and rebuilt
// on reading), a checksum.  deserialize_plan returns STC_ERR_ARG with a
// message for a stream it cannot read.
int serialize_plan(Symbolic& s, Plan& p, BackPlan& b, std::vector<char>* out);
int deserialize_plan(const char* data, size_t bytes, Symbolic* s, Plan* p, BackPlan* b, std::string* why);

}  // namespace stc
