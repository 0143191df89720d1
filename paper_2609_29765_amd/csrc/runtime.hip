// runtime.hip -- C ABI of libstc.so (declared in include/stc.h): workspace
// layout, metadata upload, the static tile schedule as a HIP graph, and the
// consumers of the resident factor.
//
// The schedule is Algorithm 1's task set with the dependencies Algorithm 2
// enforces through its progress matrix (a SYRK/GEMM reads finished TRSM
// tiles, a TRSM reads its finished diagonal tile), grouped into levels whose
// kernels (POTRF, updates, TRSM) touch disjoint data.  The graph holds one
// node per kernel with edges only to the kernels whose data it uses, so graph
// edges and kernel boundaries replace the spin-waits on the progress matrix
// and kernels of consecutive levels overlap where the data allows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/stc.h"
#include "analyse.hpp"
#include "kernels.hpp"

using namespace stc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail(STC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int32_t kInfoNone = 0x7fffffff;
constexpr int32_t kMaxRhs = 64;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Device scratch of stc_solve_noalloc: the permuted right-hand sides that its
// sweeps work on, padded rows included.  One copy per device, held until the
// process ends; host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol) but the per-device address from
// hipGetSymbolAddress.
constexpr int64_t kScratchDoubles = int64_t(1) << 22;  // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // by device ordinal, null until looked up

// address of `scratch` on the current device, looked up once per device
int scratch_address(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[(size_t)dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(STC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[(size_t)dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[(size_t)dev];
  return 0;
}

struct LevelOffsets {
  int32_t u_off, u_cnt, g_off, g_cnt, p_off, p_cnt, t_off, t_cnt, u_last, g_last;
};

// arguments of k_value_gather, kept with the graph whose root node it is so
// that a new values pointer can be written into the instantiated graph
struct LoadArgs {
  const double* vals;
  int64_t qnz;
  const int32_t* bptr;
  const int2* ent;
  int64_t total;
  double* store;
  int64_t mstride;
  int32_t* info;
  int32_t big;
  void* ptrs[9];
  void point() {
    void* p[9] = {&vals, &qnz, &bptr, &ent, &total, &store, &mstride, &info, &big};
    for (int i = 0; i < 9; ++i) ptrs[i] = p[i];
  }
};

struct GraphRec {
  hipGraph_t graph = nullptr;  // kept: the root node's handle must stay valid for updates
  hipGraphExec_t ex = nullptr;
  hipGraphNode_t load = nullptr;  // root: the value load
  LoadArgs la;
  dim3 grid;
};

}  // namespace

struct stc_handle {
  Symbolic sym;
  Plan plan;
  std::vector<LevelOffsets> lv;
  // flattened level work lists (host)
  std::vector<int32_t> upd_items, big_items, potrf_list, trsm_items;
  // solve sweeps: per level, the panel work items (forward: fed block, first
  // block row, range in the tile list; backward: fed block, range) and their
  // offsets, and the tile lists the ranges point into
  std::vector<int32_t> sfwd_items, sfwd_ptr, sbwd_items, sbwd_ptr, sfwd_tl, sbwd_tl;
  std::vector<int32_t> sfwd_nstep, sbwd_nstep;  // step items leading each launch
  int32_t* d_sfwd_items = nullptr;
  int32_t* d_sbwd_items = nullptr;
  TileD* d_sfwd_tl = nullptr;  // descriptors of each item's tiles, in item order
  TileD* d_sbwd_tl = nullptr;
  std::map<int64_t, hipGraphExec_t> solve_graphs;  // by right-hand sides per sweep (batched: negative keys)
  // binding
  int device = -1;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t batch = 0;
  hipStream_t last_stream = nullptr;
  bool factored = false;
  bool zs_ready = false;       // d_zs holds the selected inverse of the last single factorization
  int32_t fact_members = 0;    // value sets whose stores hold a factor (stc_solve_batched)
  // device views into the workspace (set by bind)
  int64_t* d_vmap = nullptr;
  int32_t* d_maps = nullptr;
  UpdTaskD* d_upd = nullptr;
  ContribD* d_contrib = nullptr;
  TrsmTaskD* d_trsm = nullptr;
  int32_t* d_upd_items = nullptr;
  int32_t* d_big_items = nullptr;
  double* d_parts = nullptr;  // partial-sum slots, per member
  double* d_zrow = nullptr;   // n_b zeros (rows a gather map leaves out)
  int32_t* d_potrf = nullptr;
  int32_t* d_trsm_items = nullptr;
  int32_t* d_perm = nullptr;  // per grid position: the original index there, or -1 (padding)
  int32_t* d_gcol = nullptr;  // per grid position: the column of P A P^T there, or -1
  int32_t* d_rows = nullptr;
  double* d_store = nullptr;  // batch stores
  double* d_y = nullptr;      // solve scratch
  double* d_scratch = nullptr;  // this device's `scratch` (stc_solve_noalloc)
  double* d_dinv = nullptr;   // inverses of the 32 x 32 diagonal blocks, per member
  int32_t* d_info = nullptr;  // batch
  double* d_ld = nullptr;     // batch
  std::map<int32_t, GraphRec> graphs;  // by member count
  // value load: per block of LBLK store doubles, its entries (input index or
  // -1 for a padded diagonal one, offset in the block)
  std::vector<int32_t> ld_ptr;
  std::vector<int2> ld_ent;
  std::vector<int32_t> gperm, gcol;  // host copies of d_perm and d_gcol
  int32_t* d_ldptr = nullptr;
  int2* d_ldent = nullptr;
  // reverse mode of log det
  BackPlan back;
  std::vector<int32_t> back_items;       // flattened per level
  std::vector<int32_t> back_level_ptr;   // items of level L: [ptr[L], ptr[L+1])
  std::vector<int32_t> fold_items;       // fold items of split tasks, flattened per level
  std::vector<int32_t> fold_level_ptr;
  FoldItemD* d_bfitems = nullptr;
  double* d_bslots = nullptr;  // partial slots of split reverse-mode tasks
  ConTermD* d_bterms = nullptr;
  ConTaskD* d_btasks = nullptr;
  int32_t* d_bitems = nullptr;
  int32_t* d_trtri = nullptr;
  int8_t* d_bdiag = nullptr;
  double* d_zs = nullptr;  // selected inverse, store layout
  double* d_ms = nullptr;  // G_k (diagonal slots) and L_mk G_k (off-diagonal slots)
  hipGraphExec_t back_graph = nullptr;
  ~stc_handle() {
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.second.ex);
      (void)hipGraphDestroy(g.second.graph);
    }
    for (auto& g : solve_graphs) (void)hipGraphExecDestroy(g.second);
    if (back_graph) (void)hipGraphExecDestroy(back_graph);
  }
};

namespace {

int64_t padded_n(const stc_handle* h) { return (int64_t)h->plan.NT * h->plan.nb; }
int64_t dinv_stride(const stc_handle* h) { return (int64_t)h->plan.NT * h->plan.nb * 32; }

// workspace layout; returns total bytes.  With base == null only the size is
// computed (the handle's pointers are left alone).
size_t layout(const stc_handle* hc, int32_t batch, char* base) {
  stc_handle* h = const_cast<stc_handle*>(hc);
  const Plan& p = h->plan;
  const Symbolic& s = h->sym;
  size_t off = 0;
  auto take = [&](auto** dst, size_t bytes) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(dst)>>;
    if (base) *dst = (T)(base + off);
    off = align256(off + std::max<size_t>(bytes, 8));
  };
  take(&h->d_vmap, sizeof(int64_t) * p.vmap.size());
  take(&h->d_ldptr, sizeof(int32_t) * h->ld_ptr.size());
  take(&h->d_ldent, sizeof(int2) * h->ld_ent.size());
  take(&h->d_maps, sizeof(int32_t) * p.maps.size());
  take(&h->d_upd, sizeof(UpdTaskD) * p.upd.size());
  take(&h->d_contrib, sizeof(ContribD) * p.contribs.size());
  take(&h->d_trsm, sizeof(TrsmTaskD) * p.trsm.size());
  take(&h->d_upd_items, sizeof(int32_t) * h->upd_items.size());
  take(&h->d_big_items, sizeof(int32_t) * h->big_items.size());
  take(&h->d_potrf, sizeof(int32_t) * h->potrf_list.size());
  take(&h->d_trsm_items, sizeof(int32_t) * h->trsm_items.size());
  take(&h->d_perm, sizeof(int32_t) * (size_t)padded_n(h));
  take(&h->d_gcol, sizeof(int32_t) * (size_t)padded_n(h));
  take(&h->d_rows, sizeof(int32_t) * s.rows.size());
  take(&h->d_info, sizeof(int32_t) * (size_t)batch);
  take(&h->d_ld, sizeof(double) * (size_t)batch);
  take(&h->d_y, sizeof(double) * (size_t)padded_n(h) * std::max<size_t>(kMaxRhs, (size_t)SR * (size_t)batch));
  take(&h->d_sfwd_items, sizeof(int32_t) * h->sfwd_items.size());
  take(&h->d_sbwd_items, sizeof(int32_t) * h->sbwd_items.size());
  take(&h->d_sfwd_tl, sizeof(TileD) * h->sfwd_tl.size());
  take(&h->d_sbwd_tl, sizeof(TileD) * h->sbwd_tl.size());
  take(&h->d_dinv, sizeof(double) * (size_t)dinv_stride(h) * (size_t)batch);
  take(&h->d_parts, sizeof(double) * (size_t)p.parts * (size_t)batch);
  take(&h->d_zrow, sizeof(double) * (size_t)p.nb);
  take(&h->d_bterms, sizeof(ConTermD) * h->back.terms.size());
  take(&h->d_btasks, sizeof(ConTaskD) * h->back.tasks.size());
  take(&h->d_bitems, sizeof(int32_t) * h->back_items.size());
  take(&h->d_bfitems, sizeof(FoldItemD) * (h->fold_items.size() / 3));
  take(&h->d_bslots, sizeof(double) * (size_t)h->back.slots);
  take(&h->d_trtri, sizeof(int32_t) * h->back.trtri_items.size());
  take(&h->d_bdiag, sizeof(int8_t) * h->back.diagflag.size());
  take(&h->d_zs, sizeof(double) * (size_t)p.store);
  take(&h->d_ms, sizeof(double) * (size_t)p.store);
  take(&h->d_store, sizeof(double) * (size_t)p.store * (size_t)batch);
  return off;
}

template <typename T>
int upload(T* dst, const std::vector<T>& src) {
  if (src.empty()) return 0;
  HIPCHK(hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return 0;
}

// event pairs around individual launches (measurement only)
struct Prof {
  struct Mark {
    int kind;
    double flops;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  int begin(hipStream_t st, hipEvent_t* a) {
    HIPCHK(hipEventCreate(a));
    HIPCHK(hipEventRecord(*a, st));
    return 0;
  }
  int end(int kind, double flops, hipStream_t st, hipEvent_t a) {
    hipEvent_t b;
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(b, st));
    marks.push_back({kind, flops, a, b});
    return 0;
  }
};

// active-column plans skip the MFMA products of empty 16-row groups; dense
// plans have none and keep the unconditional loop
bool uses_cull(const stc_handle* h) { return h->sym.mode != kModeDense; }

// measurement kinds: the value load and the level kernels
enum { kKindLoad = 0, kKindPotrf = 1, kKindUpdBig = 2, kKindUpd = 3, kKindTrsm = 4, kKinds = 5 };

// arguments of kernel `kind` (0 POTRF, 1 early-group updates, 2 TRSM, 3
// last-group updates) of level li; the last groups' items lead the level's
// item lists
LevelArgs level_args(const stc_handle* h, size_t li, int kind) {
  LevelArgs a;
  a.utasks = h->d_upd;
  a.contribs = h->d_contrib;
  a.maps = h->d_maps;
  a.ttasks = h->d_trsm;
  a.store = h->d_store;
  a.mstride = h->plan.store;
  a.dinv = h->d_dinv;
  a.dstride = dinv_stride(h);
  a.info = h->d_info;
  a.nreal = (int32_t)padded_n(h);  // padding positions hold identity rows and never fail
  a.parts = h->d_parts;
  a.zrow = h->d_zrow;
  a.pstride = h->plan.parts;
  const LevelOffsets& L = h->lv[li];
  a.potrf = h->d_potrf + L.p_off;
  a.big = h->d_big_items + 4 * (int64_t)L.g_off;
  a.upd = h->d_upd_items + 4 * (int64_t)L.u_off;
  a.trsm = h->d_trsm_items + 2 * (int64_t)L.t_off;
  a.np = L.p_cnt;
  a.nbig = L.g_cnt;
  a.nu = L.u_cnt;
  a.nt = L.t_cnt;
  if (kind == 3) {
    a.nbig = L.g_last;
    a.nu = L.u_last;
  } else if (kind == 1) {
    a.big += 4 * (int64_t)L.g_last;
    a.upd += 4 * (int64_t)L.u_last;
    a.nbig = L.g_cnt - L.g_last;
    a.nu = L.u_cnt - L.u_last;
  }
  return a;
}

// kernel, grid and dynamic LDS of a level's kernel with arguments a
template <int NB>
void level_kernel(const LevelArgs& a, int kind, int32_t members, bool cull, const void** fn, dim3* grid,
                  size_t* lds) {
  if (kind == 0) {
    *fn = reinterpret_cast<const void*>(&k_potrf<NB>);
    *grid = dim3(a.np, members);
    *lds = sizeof(double) * k_potrf_lds<NB>();
  } else if (kind == 1 || kind == 3) {
    if (cull)
      *fn = a.nbig ? reinterpret_cast<const void*>(&k_upd<NB, true, true>)
                   : reinterpret_cast<const void*>(&k_upd<NB, false, true>);
    else
      *fn = a.nbig ? reinterpret_cast<const void*>(&k_upd<NB, true, false>)
                   : reinterpret_cast<const void*>(&k_upd<NB, false, false>);
    *grid = dim3(a.nbig + a.nu, members);
    *lds = sizeof(double) * std::max(a.nbig ? UPD2_LDS : 0, a.nu ? UPD_LDS : 0);
  } else {
    *fn = reinterpret_cast<const void*>(&k_trsm<NB>);
    *grid = dim3(a.nt, members);
    *lds = sizeof(double) * trsm_lds<NB>();
  }
}

int kernel_count(const LevelArgs& a, int kind) {
  return kind == 0 ? a.np : kind == 2 ? a.nt : a.nbig + a.nu;
}

// launch every level of the schedule for `members` value sets one kernel
// after another on `st`, each timed and charged to its kernel with the
// tile-algorithmic flops of its tasks (measurement path; the factorization
// itself replays the dependency graph built by get_graph)
template <int NB>
int launch_levels_nb(stc_handle* h, int32_t members, hipStream_t st, Prof* prof) {
  for (size_t li = 0; li < h->lv.size(); ++li) {
    const LevelOffsets& L = h->lv[li];
    const Level& PL = h->plan.levels[li];
    // the level's updates as one launch (kind 1 with every item), so each
    // kernel is charged the level's flops of its kind
    for (int kind = 0; kind < 3; ++kind) {
      LevelArgs a = level_args(h, li, 2);
      if (kernel_count(a, kind) == 0) continue;
      const void* fn;
      dim3 grid;
      size_t lds;
      level_kernel<NB>(a, kind, members, uses_cull(h), &fn, &grid, &lds);
      hipEvent_t ev = nullptr;
      if (prof && prof->begin(st, &ev)) return STC_ERR_HIP;
      void* args[] = {&a};
      HIPCHK(hipLaunchKernel(fn, grid, dim3(256), args, lds, st));
      const int pk = kind == 0 ? kKindPotrf : kind == 2 ? kKindTrsm : (L.g_cnt ? kKindUpdBig : kKindUpd);
      const double fl = kind == 0 ? PL.flops_potrf : kind == 1 ? PL.flops_upd : PL.flops_trsm;
      if (prof && prof->end(pk, fl * members, st, ev)) return STC_ERR_HIP;
    }
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// the value load's kernel arguments for `members` value sets starting at vals
void load_args(stc_handle* h, const double* vals, int32_t members, LoadArgs* la, dim3* grid) {
  la->vals = vals;
  la->qnz = h->sym.qnz;
  la->bptr = h->d_ldptr;
  la->ent = h->d_ldent;
  la->total = h->plan.store;
  la->store = h->d_store;
  la->mstride = h->plan.store;
  la->info = h->d_info;
  la->big = kInfoNone;
  la->point();
  *grid = dim3((unsigned)(h->ld_ptr.size() - 1), members);
}

hipKernelNodeParams load_node_params(GraphRec* g) {
  hipKernelNodeParams kp{};
  kp.blockDim = dim3(256);
  kp.gridDim = g->grid;
  kp.func = reinterpret_cast<void*>(&k_value_gather);
  kp.kernelParams = g->la.ptrs;
  kp.extra = nullptr;
  kp.sharedMemBytes = 0;
  return kp;
}

// the factorization as one HIP graph: the value load (root), every non-empty
// kernel of a level as a node that waits only for the kernels whose data it
// uses (kernel_dag), so the kernels of consecutive levels overlap wherever
// the data allows, and the failure-flag finish after the last kernels
template <int NB>
int build_graph_nb(stc_handle* h, int32_t members, GraphRec* out) {
  std::vector<KernelNode> dag;
  kernel_dag(h->plan, &dag);
  // the argument blocks stay alive until the graph is instantiated
  std::vector<LevelArgs> args(dag.size());
  std::vector<void*> kargs(dag.size());
  std::vector<hipGraphNode_t> nodes(dag.size());
  std::vector<hipGraphNode_t> deps;
  std::vector<char> has_dependent(dag.size(), 0);
  hipGraph_t g;
  HIPCHK(hipGraphCreate(&g, 0));
  auto bail = [&](const char* what, hipError_t e) {
    (void)hipGraphDestroy(g);
    return fail(STC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  load_args(h, nullptr, members, &out->la, &out->grid);
  hipKernelNodeParams lp = load_node_params(out);
  hipError_t e = hipGraphAddKernelNode(&out->load, g, nullptr, 0, &lp);
  if (e != hipSuccess) return bail("hipGraphAddKernelNode", e);
  for (size_t x = 0; x < dag.size(); ++x) {
    args[x] = level_args(h, (size_t)dag[x].level, dag[x].kind);
    const void* fn;
    dim3 grid;
    size_t lds;
    level_kernel<NB>(args[x], dag[x].kind, members, uses_cull(h), &fn, &grid, &lds);
    kargs[x] = &args[x];
    hipKernelNodeParams kp{};
    kp.blockDim = dim3(256);
    kp.gridDim = grid;
    kp.func = const_cast<void*>(fn);
    kp.kernelParams = &kargs[x];
    kp.extra = nullptr;
    kp.sharedMemBytes = (unsigned)lds;
    deps.clear();
    for (int32_t d : dag[x].deps) {
      deps.push_back(nodes[(size_t)d]);
      has_dependent[(size_t)d] = 1;
    }
    if (deps.empty()) deps.push_back(out->load);
    e = hipGraphAddKernelNode(&nodes[x], g, deps.data(), deps.size(), &kp);
    if (e != hipSuccess) return bail("hipGraphAddKernelNode", e);
  }
  deps.clear();
  for (size_t x = 0; x < dag.size(); ++x)
    if (!has_dependent[x]) deps.push_back(nodes[x]);
  if (deps.empty()) deps.push_back(out->load);
  int32_t* info = h->d_info;
  int32_t count = members, big = kInfoNone;
  int32_t* none = nullptr;
  const int32_t* gcol = h->d_gcol;
  void* fargs[] = {&info, &count, &big, &none, &gcol};
  hipKernelNodeParams fp{};
  fp.blockDim = dim3(256);
  fp.gridDim = dim3((unsigned)((members + 255) / 256));
  fp.func = reinterpret_cast<void*>(&k_info_finish);
  fp.kernelParams = fargs;
  fp.extra = nullptr;
  fp.sharedMemBytes = 0;
  hipGraphNode_t fin;
  e = hipGraphAddKernelNode(&fin, g, deps.data(), deps.size(), &fp);
  if (e != hipSuccess) return bail("hipGraphAddKernelNode", e);
  e = hipGraphInstantiate(&out->ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(STC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  out->graph = g;
  return 0;
}

int launch_levels(stc_handle* h, int32_t members, hipStream_t st, Prof* prof) {
  switch (h->plan.nb) {
    case 32: return launch_levels_nb<32>(h, members, st, prof);
    case 64: return launch_levels_nb<64>(h, members, st, prof);
    case 128: return launch_levels_nb<128>(h, members, st, prof);
    case 256: return launch_levels_nb<256>(h, members, st, prof);
  }
  return fail(STC_ERR_ARG, "unsupported tile size");
}

int build_graph(stc_handle* h, int32_t members, GraphRec* ex) {
  switch (h->plan.nb) {
    case 32: return build_graph_nb<32>(h, members, ex);
    case 64: return build_graph_nb<64>(h, members, ex);
    case 128: return build_graph_nb<128>(h, members, ex);
    case 256: return build_graph_nb<256>(h, members, ex);
  }
  return fail(STC_ERR_ARG, "unsupported tile size");
}

// the forward and backward sweeps over right-hand sides [g0, g0 + nr) of
// d_y: one launch per level, each solving that level's blocks after the
// products of the level before
template <int NB, int R>
void launch_sweeps_r(stc_handle* h, double* y0, int32_t nr, int32_t g0, int32_t members, int64_t ystride,
                     hipStream_t st) {
  const int64_t np = padded_n(h), ms = h->plan.store, ds = dinv_stride(h);
  double* y = y0 + (int64_t)g0 * np;
  for (size_t q = 0; q < h->sfwd_nstep.size(); ++q) {
    const int32_t c = h->sfwd_ptr[q], d = h->sfwd_ptr[q + 1];
    if (d > c)
      hipLaunchKernelGGL((k_sfwd_step<NB, R>), dim3(d - c, members), dim3(256), 0, st,
                         h->d_sfwd_items + 4 * (int64_t)c, h->sfwd_nstep[q], h->d_sfwd_tl, h->d_maps, h->d_rows,
                         h->d_store, h->d_dinv, y, np, nr, ms, ds, ystride);
  }
  for (size_t q = 0; q < h->sbwd_nstep.size(); ++q) {
    const int32_t c = h->sbwd_ptr[q], d = h->sbwd_ptr[q + 1];
    if (d > c)
      hipLaunchKernelGGL((k_sbwd_step<NB, R>), dim3(d - c, members), dim3(256), 0, st,
                         h->d_sbwd_items + 4 * (int64_t)c, h->sbwd_nstep[q], h->d_sbwd_tl, h->d_rows, h->d_store,
                         h->d_dinv, y, np, nr, ms, ds, ystride);
  }
}

template <int NB>
void launch_sweeps_nb(stc_handle* h, double* y0, int32_t nr, int32_t g0, int32_t members, int64_t ystride,
                      hipStream_t st) {
  if (nr == 1) launch_sweeps_r<NB, 1>(h, y0, nr, g0, members, ystride, st);
  else launch_sweeps_r<NB, SR>(h, y0, nr, g0, members, ystride, st);
}

// the sweeps of right-hand sides [g0, g0 + nr) of y0 (stride padded_n), for
// value sets 0..members-1 (value set b's right-hand sides at y0 + b ystride)
void launch_sweeps(stc_handle* h, double* y0, int32_t nr, int32_t g0, hipStream_t st, int32_t members = 1,
                   int64_t ystride = 0) {
  switch (h->plan.nb) {
    case 32: launch_sweeps_nb<32>(h, y0, nr, g0, members, ystride, st); break;
    case 64: launch_sweeps_nb<64>(h, y0, nr, g0, members, ystride, st); break;
    case 128: launch_sweeps_nb<128>(h, y0, nr, g0, members, ystride, st); break;
    case 256: launch_sweeps_nb<256>(h, y0, nr, g0, members, ystride, st); break;
  }
}

int get_solve_graph(stc_handle* h, int32_t nr, int32_t g0, hipGraphExec_t* out, int32_t members = 1) {
  const int64_t key = members > 1 ? -((int64_t)members * 16 + nr) : (int64_t)nr * 1024 + g0;
  auto it = h->solve_graphs.find(key);
  if (it != h->solve_graphs.end()) {
    *out = it->second;
    return 0;
  }
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  launch_sweeps(h, h->d_y, nr, g0, cs, members, (int64_t)SR * padded_n(h));
  hipGraph_t g;
  hipError_t e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return fail(STC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(STC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  h->solve_graphs[key] = ex;
  *out = ex;
  return 0;
}

int get_graph(stc_handle* h, int32_t members, GraphRec** out) {
  auto it = h->graphs.find(members);
  if (it == h->graphs.end()) {
    GraphRec rec;
    const int rc = build_graph(h, members, &rec);
    if (rc) return rc;
    it = h->graphs.emplace(members, rec).first;
    it->second.la.point();  // the record moved: its argument pointers follow it
  }
  *out = &it->second;
  return 0;
}

// value load + schedule for `members` value sets starting at vals: one graph
// launch (the values pointer written into its root node when it changes);
// with prof, the same kernels launched one by one, each timed
int run_factor(stc_handle* h, const double* vals, int32_t members, hipStream_t st,
               Prof* prof = nullptr) {
  if (!prof) {
    GraphRec* g;
    int rc = get_graph(h, members, &g);
    if (rc) return rc;
    if (g->la.vals != vals) {
      g->la.vals = vals;
      hipKernelNodeParams kp = load_node_params(g);
      HIPCHK(hipGraphExecKernelNodeSetParams(g->ex, g->load, &kp));
    }
    HIPCHK(hipGraphLaunch(g->ex, st));
    return 0;
  }
  LoadArgs la;
  dim3 grid;
  load_args(h, vals, members, &la, &grid);
  hipEvent_t ev = nullptr;
  if (prof->begin(st, &ev)) return STC_ERR_HIP;
  HIPCHK(hipLaunchKernel(reinterpret_cast<const void*>(&k_value_gather), grid, dim3(256), la.ptrs, 0, st));
  if (prof->end(kKindLoad, 0.0, st, ev)) return STC_ERR_HIP;
  int rc = launch_levels(h, members, st, prof);
  if (rc) return rc;
  hipLaunchKernelGGL(k_info_finish, dim3((members + 255) / 256), dim3(256), 0, st, h->d_info, members,
                     kInfoNone, (int32_t*)nullptr, (const int32_t*)h->d_gcol);
  HIPCHK(hipGetLastError());
  return 0;
}

// selected inverse of the last single factorization into d_zs: the G_k
// level, then one contraction kernel per level of the reverse tile DAG
template <int NB>
int launch_backward_nb(stc_handle* h, hipStream_t st) {
  const int32_t ntr = (int32_t)(h->back.trtri_items.size() / 2);
  hipLaunchKernelGGL((k_trtri<NB>), dim3(ntr), dim3(256), sizeof(double) * trtri_lds<NB>(), st,
                     h->d_trtri, h->d_store, h->d_dinv, h->d_ms);
  BackArgs g;
  g.tasks = h->d_btasks;
  g.terms = h->d_bterms;
  g.maps = h->d_maps;
  g.L = h->d_store;
  g.Z = h->d_zs;
  g.M = h->d_ms;
  g.P = h->d_bslots;
  for (size_t L = 0; L + 1 < h->back_level_ptr.size(); ++L) {
    const int32_t a = h->back_level_ptr[L], b = h->back_level_ptr[L + 1];
    if (b == a) continue;
    g.items = h->d_bitems + 3 * (int64_t)a;
    hipLaunchKernelGGL((k_backcon<NB>), dim3(b - a), dim3(256), sizeof(double) * con_lds<NB>(), st, g);
    const int32_t fa = h->fold_level_ptr[L], fb = h->fold_level_ptr[L + 1];
    if (fb > fa)
      hipLaunchKernelGGL((k_backfold<NB>), dim3(fb - fa, CB / 16), dim3(256), 0, st,
                         (const FoldItemD*)h->d_bfitems + fa, h->d_zs, h->d_ms, (const double*)h->d_bslots);
  }
  HIPCHK(hipGetLastError());
  return 0;
}

int launch_backward(stc_handle* h, hipStream_t st) {
  switch (h->plan.nb) {
    case 32: return launch_backward_nb<32>(h, st);
    case 64: return launch_backward_nb<64>(h, st);
    case 128: return launch_backward_nb<128>(h, st);
    case 256: return launch_backward_nb<256>(h, st);
  }
  return fail(STC_ERR_ARG, "unsupported tile size");
}

int get_back_graph(stc_handle* h, hipGraphExec_t* out) {
  if (h->back_graph) {
    *out = h->back_graph;
    return 0;
  }
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  int rc = launch_backward(h, cs);
  hipGraph_t g;
  hipError_t e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc) return rc;
  if (e != hipSuccess) return fail(STC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(STC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  h->back_graph = ex;
  *out = ex;
  return 0;
}

int check_bound(const stc_handle* h) {
  if (!h) return fail(STC_ERR_ARG, "null handle");
  if (!h->ws) return fail(STC_ERR_STATE, "handle is not bound to a workspace");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(STC_ERR_STATE, "current device differs from the bound device");
  return 0;
}

}  // namespace

// one sweep's work items against its tile dependencies: launches run in
// order, the items of one launch concurrently
static int check_sweep(const stc_handle* h, bool fwd, const std::vector<int32_t>& items,
                       const std::vector<int32_t>& ptr, const std::vector<int32_t>& nstep,
                       const std::vector<int32_t>& tl, int32_t chunk, int64_t* st) {
  const char* sw = fwd ? "forward" : "backward";
  const int32_t NT = h->sym.NT, nb = h->plan.nb;
  const int32_t nch = (nb + chunk - 1) / chunk;
  const size_t ntl = h->sym.tiles.size();
  auto bad = [&](const std::string& why) { return fail(STC_ERR_SCHEDULE, std::string(sw) + " solve: " + why); };
  if (ptr.size() != nstep.size() + 1 || ptr.front() != 0 || (size_t)ptr.back() * 4 != items.size())
    return bad("launch table does not cover the items");
  std::vector<int32_t> solved((size_t)NT, -1), need((size_t)NT, 0), got((size_t)NT, 0);
  std::vector<int64_t> done(ntl, 0);  // bit c: chunk c applied; all bits: whole tile
  const int64_t all = (nch >= 63) ? -1 : ((int64_t(1) << nch) - 1);
  for (const TileInfo& t : h->sym.tiles) ++need[(size_t)(fwd ? t.m : t.k)];
  std::map<int64_t, int32_t> owner;  // (block, chunk) -> item, per launch
  for (size_t q = 0; q < nstep.size(); ++q) {
    owner.clear();
    const int32_t a = ptr[q], b = ptr[q + 1];
    if (b < a || nstep[q] < 0 || nstep[q] > b - a) return bad("bad launch bounds");
    for (int32_t it = a; it < b; ++it) {
      const int32_t blk = items[4 * (size_t)it], i0 = items[4 * (size_t)it + 1];
      const int32_t t0 = items[4 * (size_t)it + 2], t1 = items[4 * (size_t)it + 3];
      const bool step = it - a < nstep[q];
      if (blk < 0 || blk >= NT || t0 < 0 || t1 < t0 || (size_t)t1 > tl.size()) return bad("item out of range");
      if (solved[(size_t)blk] >= 0) return bad("block " + std::to_string(blk) + " written after it was solved");
      if (!step && (i0 < 0 || i0 >= nb || i0 % chunk)) return bad("chunk offset out of range");
      for (int32_t c = step ? 0 : i0 / chunk; c < (step ? nch : i0 / chunk + 1); ++c)
        if (!owner.emplace((int64_t)blk * nch + c, it).second)
          return bad("two items of one launch write block " + std::to_string(blk));
      for (int32_t z = t0; z < t1; ++z) {
        const int32_t t = tl[(size_t)z];
        if (t < 0 || (size_t)t >= ntl) return bad("tile out of range");
        const TileInfo& ti = h->sym.tiles[(size_t)t];
        const int32_t fed = fwd ? ti.m : ti.k, src = fwd ? ti.k : ti.m;
        if (fed != blk) return bad("tile " + std::to_string(t) + " applied to a block it does not feed");
        if (solved[(size_t)src] < 0 || solved[(size_t)src] >= (int32_t)q)
          return bad("tile " + std::to_string(t) + " applied before its source block was solved");
        const int64_t bits = step ? all : (int64_t(1) << (i0 / chunk));
        if (done[(size_t)t] & bits) return bad("tile " + std::to_string(t) + " applied twice");
        done[(size_t)t] |= bits;
        if (done[(size_t)t] == all) ++got[(size_t)blk];
      }
      if (step) {
        ++st[1];
        if (got[(size_t)blk] != need[(size_t)blk])
          return bad("block " + std::to_string(blk) + " solved before all its tiles were applied");
      } else {
        ++st[2];
      }
    }
    // blocks are marked solved after the launch: no item of a launch reads
    // a block that another item of it solves
    for (int32_t it = a; it < a + nstep[q]; ++it) solved[(size_t)items[4 * (size_t)it]] = (int32_t)q;
    st[0] += 1;
    if (nstep[q] > 0 && b - a > nstep[q]) st[3] += 1;
  }
  for (int32_t k = 0; k < NT; ++k)
    if (solved[(size_t)k] < 0) return bad("block " + std::to_string(k) + " never solved");
  return 0;
}

// the host-side lists derived from the symbolic analysis and the plans:
// flattened level work lists and the solve sweeps' work items
static void finish_handle(stc_handle* h) {
  // grid positions: the original index and the permuted column at each
  {
    const int64_t np = padded_n(h);
    h->gperm.assign((size_t)np, -1);
    h->gcol.assign((size_t)np, -1);
    for (int64_t j = 0; j < h->sym.n; ++j) {
      const int64_t q = grid_pos(h->sym, j);
      h->gperm[(size_t)q] = h->sym.perm[(size_t)j];
      h->gcol[(size_t)q] = (int32_t)j;
    }
  }
  // the value load's per-block entry lists: input entries by store block
  // (ascending input index within a block), then the padded diagonal ones
  {
    const Plan& p = h->plan;
    const int64_t nblk = (p.store + LBLK - 1) / LBLK;
    std::vector<int64_t> pad;
    for (int32_t k = 0; k < p.NT; ++k)
      for (int32_t r = p.diag_h[(size_t)k]; r < p.nb; ++r) pad.push_back((int64_t)k * p.nb * p.nb + (int64_t)r * p.nb + r);
    h->ld_ptr.assign((size_t)nblk + 1, 0);
    for (int64_t v : p.vmap) h->ld_ptr[(size_t)(v / LBLK) + 1]++;
    for (int64_t v : pad) h->ld_ptr[(size_t)(v / LBLK) + 1]++;
    for (int64_t b = 0; b < nblk; ++b) h->ld_ptr[(size_t)b + 1] += h->ld_ptr[(size_t)b];
    h->ld_ent.resize((size_t)h->ld_ptr.back());
    std::vector<int32_t> fill(h->ld_ptr.begin(), h->ld_ptr.end() - 1);
    for (size_t q = 0; q < p.vmap.size(); ++q) {
      const int64_t v = p.vmap[q];
      h->ld_ent[(size_t)fill[(size_t)(v / LBLK)]++] = make_int2((int32_t)q, (int32_t)(v % LBLK));
    }
    for (int64_t v : pad) h->ld_ent[(size_t)fill[(size_t)(v / LBLK)]++] = make_int2(-1, (int32_t)(v % LBLK));
  }
  h->back_level_ptr.push_back(0);
  for (const auto& li : h->back.level_items) {
    h->back_items.insert(h->back_items.end(), li.begin(), li.end());
    h->back_level_ptr.push_back((int32_t)(h->back_items.size() / 3));
  }
  h->fold_level_ptr.assign(1, 0);
  for (size_t L = 0; L < h->back.level_items.size(); ++L) {
    if (L < h->back.fold_items.size())
      h->fold_items.insert(h->fold_items.end(), h->back.fold_items[L].begin(), h->back.fold_items[L].end());
    h->fold_level_ptr.push_back((int32_t)(h->fold_items.size() / 3));
  }
  // flatten the level lists
  for (const Level& L : h->plan.levels) {
    LevelOffsets x;
    x.u_off = (int32_t)(h->upd_items.size() / 4);
    x.u_cnt = (int32_t)(L.upd_items.size() / 4);
    x.u_last = L.upd_last;
    x.g_last = L.big_last;
    h->upd_items.insert(h->upd_items.end(), L.upd_items.begin(), L.upd_items.end());
    x.g_off = (int32_t)(h->big_items.size() / 4);
    x.g_cnt = (int32_t)(L.big_items.size() / 4);
    h->big_items.insert(h->big_items.end(), L.big_items.begin(), L.big_items.end());
    x.p_off = (int32_t)h->potrf_list.size();
    x.p_cnt = (int32_t)L.potrf.size();
    h->potrf_list.insert(h->potrf_list.end(), L.potrf.begin(), L.potrf.end());
    x.t_off = (int32_t)(h->trsm_items.size() / 2);
    x.t_cnt = (int32_t)(L.trsm_items.size() / 2);
    h->trsm_items.insert(h->trsm_items.end(), L.trsm_items.begin(), L.trsm_items.end());
    h->lv.push_back(x);
  }
  // solve work items.  Level q's blocks are solved by step items that
  // first apply the tiles feeding them from level q - 1, in one launch with
  // the panel chunks for later blocks that level q - 1 feeds.  A step item
  // reads its tiles whole where a panel chunk reads a 1 / (n_b / chunk)
  // share of them, so where that serial excess passes kStepFuseBytes at
  // some block of the level (a saved launch is worth well under a
  // microsecond) the level gets two launches instead: every chunk of level
  // q - 1's products, then step items with no tiles.  Tiles of one item are
  // taken in a fixed order.
  const Plan& pl = h->plan;
  constexpr double kStepFuseBytes = 65536.0;
  auto sweep_items = [&](const std::vector<int32_t>& lptr, const std::vector<int32_t>& lblk,
                         const std::vector<int32_t>& tptr, const std::vector<int32_t>& tix, bool fwd,
                         int32_t chunk, std::vector<int32_t>* items, std::vector<int32_t>* ptr,
                         std::vector<int32_t>* nstep, std::vector<int32_t>* tl) {
    const int32_t nlev = (int32_t)lptr.size() - 1;
    std::vector<int32_t> lev((size_t)h->sym.NT, -1);
    for (int32_t L = 0; L < nlev; ++L)
      for (int32_t b = lptr[(size_t)L]; b < lptr[(size_t)L + 1]; ++b) lev[(size_t)lblk[(size_t)b]] = L;
    std::map<int32_t, std::vector<int32_t>> feed;
    auto close_launch = [&](int32_t ns) {
      nstep->push_back(ns);
      ptr->push_back((int32_t)(items->size() / 4));
    };
    auto panel_chunks = [&](int32_t fed, const std::vector<int32_t>& ts) {
      const int32_t t0 = (int32_t)tl->size();
      tl->insert(tl->end(), ts.begin(), ts.end());
      const int32_t t1 = (int32_t)tl->size();
      for (int32_t i0 = 0; i0 < pl.nb; i0 += chunk) items->insert(items->end(), {fed, i0, t0, t1});
    };
    ptr->push_back(0);
    for (int32_t q = 0; q < nlev; ++q) {
      feed.clear();
      if (q > 0)
        for (int32_t b = lptr[(size_t)q - 1]; b < lptr[(size_t)q]; ++b) {
          const int32_t k = lblk[(size_t)b];
          for (int32_t z = tptr[(size_t)k]; z < tptr[(size_t)k + 1]; ++z) {
            const int32_t t = tix[(size_t)z];
            const TileInfo& ti = h->sym.tiles[(size_t)t];
            feed[fwd ? ti.m : ti.k].push_back(t);
          }
        }
      double excess = 0.0;  // largest serial excess of a step item, bytes
      for (int32_t b = lptr[(size_t)q]; b < lptr[(size_t)q + 1]; ++b) {
        auto it = feed.find(lblk[(size_t)b]);
        if (it == feed.end()) continue;
        double rows = 0.0;
        for (int32_t t : it->second) rows += h->sym.tiles[(size_t)t].cnt;
        excess = std::max(excess, rows * (double)std::max(0, pl.nb - chunk) * sizeof(double));
      }
      const bool fuse = excess <= kStepFuseBytes;
      if (!fuse) {
        for (const auto& kv : feed) panel_chunks(kv.first, kv.second);
        close_launch(0);
      }
      int32_t ns = 0;
      for (int32_t b = lptr[(size_t)q]; b < lptr[(size_t)q + 1]; ++b) {
        const int32_t m = lblk[(size_t)b];
        const int32_t t0 = (int32_t)tl->size();
        auto it = feed.find(m);
        if (fuse && it != feed.end()) tl->insert(tl->end(), it->second.begin(), it->second.end());
        items->insert(items->end(), {m, 0, t0, (int32_t)tl->size()});
        ++ns;
      }
      if (fuse)
        for (const auto& kv : feed)
          if (lev[(size_t)kv.first] != q) panel_chunks(kv.first, kv.second);
      close_launch(ns);
    }
  };
  sweep_items(pl.fwd_level_ptr, pl.fwd_level_blk, pl.col_tiles_ptr, pl.col_tiles, true, SCH, &h->sfwd_items,
              &h->sfwd_ptr, &h->sfwd_nstep, &h->sfwd_tl);
  sweep_items(pl.bwd_level_ptr, pl.bwd_level_blk, pl.row_tiles_ptr, pl.row_tiles, false, SBC, &h->sbwd_items,
              &h->sbwd_ptr, &h->sbwd_nstep, &h->sbwd_tl);
}

extern "C" {

const char* stc_last_error(void) { return g_err.c_str(); }

int stc_analyse(int64_t n, const int64_t* colptr, const int32_t* rowind, const stc_opts* opts,
                stc_handle** out) {
  if (!out) return fail(STC_ERR_ARG, "null output handle");
  *out = nullptr;
  stc_opts o{0, STC_MODE_AUTO, STC_ORD_AUTO, nullptr, 0, 0, 0, 0, 0};
  if (opts) o = *opts;
  const bool auto_nb = o.nb == 0;
  if (auto_nb) o.nb = 64;
  if (o.nb != 32 && o.nb != 64 && o.nb != 128 && o.nb != 256)
    return fail(STC_ERR_ARG, "nb must be 0, 32, 64, 128 or 256");
  if (o.wg_slots < 0) return fail(STC_ERR_ARG, "wg_slots must be >= 0");
  if (o.align < 0) return fail(STC_ERR_ARG, "align must be >= 0");
  if (o.max_split < 0 || o.max_split > 64 || o.fold_pct < 0)
    return fail(STC_ERR_ARG, "max_split must be in [0, 64] and fold_pct >= 0");
  if (o.batch < 0) return fail(STC_ERR_ARG, "batch must be >= 0");
  try {
    auto* h = new stc_handle();
    std::string why;
    int rc = analyse(n, colptr, rowind, o.ordering, o.nb, o.mode, o.perm, &h->sym, &why);
    // automatic tile size: 64, or larger tiles when the pattern takes the
    // dense route there (fewer, larger tiles keep the FP64 matrix cores
    // busy; tile 256 from n = 2048, 128 from n = 512)
    if (rc == 0 && auto_nb && h->sym.mode == kModeDense && n >= 512) {
      o.nb = n >= 2048 ? 256 : 128;
      h->sym = Symbolic();
      rc = analyse(n, colptr, rowind, o.ordering, o.nb, o.mode, o.perm, &h->sym, &why);
    }
    if (rc) {
      delete h;
      return fail(rc, why);
    }
    // the supernodal route (Sec. 5.4) replaces the fixed grid by tiles that
    // follow the fill; here its patterns keep the fixed-width tiles the
    // kernels take, on a grid aligned to the elimination tree at n_b columns
    // (unless the caller fixed the mode or the grid)
    const int64_t align = o.align > 0 ? o.align
                          : (o.mode == STC_MODE_AUTO && h->sym.route == kRouteSupernodal) ? o.nb
                                                                                           : 0;
    if (align > 0) align_tiles(&h->sym, align);
    if (h->sym.qnz + o.nb >= INT32_MAX || (int64_t)h->sym.NT * o.nb >= INT32_MAX) {
      delete h;
      return fail(STC_ERR_ARG, "more than 2^31 - 1 input entries or grid positions");
    }
    // a batch of value sets shares the device: each set's split is balanced
    // for its share of the work-groups (at least 16, the best of a sweep on
    // the 128-member Laplacian batch)
    int64_t slots = o.wg_slots;
    if (o.batch > 1) slots = std::max<int64_t>(16, (slots > 0 ? slots : default_wg_slots(h->sym.nb)) / o.batch);
    rc = build_plan(h->sym, UB, TR, slots, &h->plan, &why, o.max_split, o.fold_pct);
    if (rc == 0) rc = build_backward(h->sym, &h->plan, &h->back, &why);
    if (rc) {
      delete h;
      return fail(rc, why);
    }
    finish_handle(h);
    *out = h;
    return 0;
  } catch (const std::bad_alloc&) {
    return fail(STC_ERR_ALLOC, "host allocation failed during analysis");
  } catch (const std::exception& e) {
    return fail(STC_ERR_ARG, e.what());
  }
}

int stc_workspace_bytes(const stc_handle* h, int32_t batch, size_t* bytes) {
  if (!h || !bytes || batch < 1) return fail(STC_ERR_ARG, "null argument or batch < 1");
  *bytes = layout(h, batch, nullptr);
  return 0;
}

int stc_bind(stc_handle* h, void* d_ws, size_t bytes, int32_t batch, void* stream) {
  (void)stream;
  if (!h || !d_ws || batch < 1) return fail(STC_ERR_ARG, "null handle/workspace or batch < 1");
  if (((uintptr_t)d_ws & 255) != 0) return fail(STC_ERR_ARG, "workspace must be 256-byte aligned");
  size_t need = 0;
  stc_workspace_bytes(h, batch, &need);
  if (bytes < need)
    return fail(STC_ERR_ALLOC, "workspace too small: need " + std::to_string(need) + " bytes");
  for (auto& g : h->graphs) {
    (void)hipGraphExecDestroy(g.second.ex);
    (void)hipGraphDestroy(g.second.graph);
  }
  h->graphs.clear();
  for (auto& g : h->solve_graphs) (void)hipGraphExecDestroy(g.second);
  h->solve_graphs.clear();
  if (h->back_graph) (void)hipGraphExecDestroy(h->back_graph);
  h->back_graph = nullptr;
  h->factored = false;
  h->zs_ready = false;
  h->fact_members = 0;
  HIPCHK(hipGetDevice(&h->device));
  if (int rc0 = scratch_address(&h->d_scratch)) return rc0;
  h->ws = (char*)d_ws;
  h->ws_bytes = bytes;
  h->batch = batch;
  layout(h, batch, h->ws);
  const Plan& p = h->plan;
  const Symbolic& s = h->sym;
  std::vector<UpdTaskD> upd(p.upd.size());
  for (size_t i = 0; i < upd.size(); ++i) {
    const UpdTask& u = p.upd[i];
    upd[i] = UpdTaskD{u.c_off, u.part_off, u.in_part_off, u.c_rows, u.diag, u.c_begin, u.c_end,
                      u.nsplit, u.in_npart};
  }
  std::vector<ContribD> con(p.contribs.size());
  for (size_t i = 0; i < con.size(); ++i) {
    const Contrib& c = p.contribs[i];
    con[i] = ContribD{c.a_off, c.b_off, c.a_rows, c.b_rows, c.rowmap, c.colmap};
  }
  std::vector<TrsmTaskD> tr(p.trsm.size());
  for (size_t i = 0; i < tr.size(); ++i)
    tr[i] = TrsmTaskD{p.trsm[i].x_off, p.trsm[i].l_off, p.trsm[i].rows, p.trsm[i].k};
  std::vector<TileD> tl(s.tiles.size());
  for (size_t i = 0; i < tl.size(); ++i)
    tl[i] = TileD{p.tile_off[i], s.tiles[i].roff, s.tiles[i].m, s.tiles[i].k, s.tiles[i].cnt, p.tile_imap[i]};
  std::vector<TileD> ftl(h->sfwd_tl.size()), btl(h->sbwd_tl.size());
  for (size_t i = 0; i < ftl.size(); ++i) ftl[i] = tl[(size_t)h->sfwd_tl[i]];
  for (size_t i = 0; i < btl.size(); ++i) btl[i] = tl[(size_t)h->sbwd_tl[i]];
  int rc = 0;
  if ((rc = upload(h->d_vmap, p.vmap)) || (rc = upload(h->d_ldptr, h->ld_ptr)) ||
      (rc = upload(h->d_ldent, h->ld_ent)) || (rc = upload(h->d_maps, p.maps)) ||
      (rc = upload(h->d_upd, upd)) || (rc = upload(h->d_contrib, con)) ||
      (rc = upload(h->d_trsm, tr)) || (rc = upload(h->d_upd_items, h->upd_items)) ||
      (rc = upload(h->d_big_items, h->big_items)) ||
      (rc = upload(h->d_potrf, h->potrf_list)) || (rc = upload(h->d_trsm_items, h->trsm_items)) ||
      (rc = upload(h->d_perm, h->gperm)) || (rc = upload(h->d_gcol, h->gcol)) ||
      (rc = upload(h->d_rows, s.rows)) || (rc = upload(h->d_sfwd_items, h->sfwd_items)) ||
      (rc = upload(h->d_sbwd_items, h->sbwd_items)) || (rc = upload(h->d_sfwd_tl, ftl)) ||
      (rc = upload(h->d_sbwd_tl, btl)))
    return rc;
  HIPCHK(hipMemset(h->d_zrow, 0, sizeof(double) * (size_t)p.nb));
  const BackPlan& bp = h->back;
  std::vector<ConTermD> bt(bp.terms.size());
  for (size_t i = 0; i < bt.size(); ++i) {
    const ConTerm& c = bp.terms[i];
    bt[i] = ConTermD{c.a_off, c.b_off, c.a_buf, c.a_mode, c.a_rmap, c.a_qmap, c.b_buf, c.b_qmap, c.K, 0};
  }
  std::vector<ConTaskD> bk(bp.tasks.size());
  for (size_t i = 0; i < bk.size(); ++i) {
    const ConTask& t = bp.tasks[i];
    bk[i] = ConTaskD{t.c_off, t.c_buf, t.c_rows, t.ncols, t.diag, t.t_begin, t.t_end, t.beta, 0, t.alpha};
  }
  std::vector<FoldItemD> bf(h->fold_items.size() / 3);
  for (size_t i = 0; i < bf.size(); ++i) {
    const FoldTask& f = bp.folds[(size_t)h->fold_items[3 * i]];
    bf[i] = FoldItemD{f.c_off, f.slot_off, f.c_buf, f.c_rows, f.ncols, f.diag, f.nslots,
                      h->fold_items[3 * i + 1], h->fold_items[3 * i + 2], 0};
  }
  if ((rc = upload(h->d_bfitems, bf))) return rc;
  if ((rc = upload(h->d_bterms, bt)) || (rc = upload(h->d_btasks, bk)) ||
      (rc = upload(h->d_bitems, h->back_items)) || (rc = upload(h->d_trtri, bp.trtri_items)) ||
      (rc = upload(h->d_bdiag, bp.diagflag)))
    return rc;
  GraphRec* gr;
  return get_graph(h, 1, &gr);
}

int stc_factorize(stc_handle* h, const double* d_values, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_values) return fail(STC_ERR_ARG, "null values");
  hipStream_t st = (hipStream_t)stream;
  rc = run_factor(h, d_values, 1, st);
  if (rc) return rc;
  h->last_stream = st;
  h->factored = true;
  h->zs_ready = false;
  h->fact_members = std::max<int32_t>(h->fact_members, 1);
  return 0;
}

int stc_factorize_batched(stc_handle* h, const double* d_values, int32_t B, double* d_logdet,
                          int32_t* d_info, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_values || !d_logdet || !d_info) return fail(STC_ERR_ARG, "null pointer");
  if (B < 1 || B > h->batch) return fail(STC_ERR_ARG, "B must be in [1, bound batch]");
  hipStream_t st = (hipStream_t)stream;
  rc = run_factor(h, d_values, B, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_logdet, dim3(B), dim3(256), 0, st, h->d_store, h->plan.store, h->plan.nb,
                     padded_n(h), h->d_info, d_logdet);
  HIPCHK(hipMemcpyAsync(d_info, h->d_info, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipGetLastError());
  h->last_stream = st;
  h->factored = B >= 1;  // member 0 is the "last single factorization" too
  h->zs_ready = false;
  h->fact_members = B;
  return 0;
}

int stc_logdet(stc_handle* h, double* d_out, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_out) return fail(STC_ERR_ARG, "null output");
  if (!h->factored) return fail(STC_ERR_STATE, "logdet before factorize");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_logdet, dim3(1), dim3(256), 0, st, h->d_store, h->plan.store, h->plan.nb,
                     padded_n(h), h->d_info, d_out);
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_solve(stc_handle* h, double* d_b, int32_t nrhs, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_b) return fail(STC_ERR_ARG, "null right-hand side");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(STC_ERR_ARG, "nrhs must be in [1, 64]");
  if (!h->factored) return fail(STC_ERR_STATE, "solve before factorize");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = h->sym.n, np = padded_n(h);
  hipLaunchKernelGGL(k_perm_in, dim3((unsigned)((np * nrhs + 255) / 256)), dim3(256), 0, st, d_b,
                     h->d_perm, n, np, nrhs, h->d_y, np * nrhs);
  // groups of up to SR right-hand sides, each one replay of the captured sweeps
  for (int32_t g0 = 0; g0 < nrhs; g0 += SR) {
    const int32_t nr = std::min<int32_t>(SR, nrhs - g0);
    hipGraphExec_t ex;
    rc = get_solve_graph(h, nr, g0, &ex);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(ex, st));
  }
  hipLaunchKernelGGL(k_perm_out, dim3((unsigned)((np * nrhs + 255) / 256)), dim3(256), 0, st, h->d_y,
                     h->d_perm, h->d_info, n, np, nrhs, d_b, np * nrhs);
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_solve_batched(stc_handle* h, double* d_b, int32_t B, int32_t nrhs, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_b) return fail(STC_ERR_ARG, "null right-hand sides");
  if (nrhs < 1 || nrhs > SR) return fail(STC_ERR_ARG, "nrhs must be in [1, 8] for a batched solve");
  if (B < 1 || B > h->batch) return fail(STC_ERR_ARG, "B must be in [1, bound batch]");
  if (B > h->fact_members)
    return fail(STC_ERR_STATE, "batched solve needs a batched factorization of at least B value sets");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = h->sym.n, np = padded_n(h), ys = (int64_t)SR * np;
  hipLaunchKernelGGL(k_perm_in, dim3((unsigned)((np * nrhs + 255) / 256), B), dim3(256), 0, st, d_b, h->d_perm, n,
                     np, nrhs, h->d_y, ys);
  hipGraphExec_t ex;
  rc = get_solve_graph(h, nrhs == 1 ? 1 : SR, 0, &ex, B);
  if (rc) return rc;
  HIPCHK(hipGraphLaunch(ex, st));
  hipLaunchKernelGGL(k_perm_out, dim3((unsigned)((np * nrhs + 255) / 256), B), dim3(256), 0, st, h->d_y, h->d_perm,
                     h->d_info, n, np, nrhs, d_b, ys);
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_solve_noalloc(stc_handle* h, double* d_b, int32_t nrhs, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_b) return fail(STC_ERR_ARG, "null right-hand side");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(STC_ERR_ARG, "nrhs must be in [1, 64]");
  if (!h->factored) return fail(STC_ERR_STATE, "solve before factorize");
  const int64_t n = h->sym.n, np = padded_n(h);
  if (np * nrhs > kScratchDoubles)
    return fail(STC_ERR_ARG, "padded order x nrhs = " + std::to_string(np * nrhs) +
                                 " doubles exceeds the allocation-free solve's scratch of " +
                                 std::to_string(kScratchDoubles));
  if (!h->d_scratch) return fail(STC_ERR_STATE, "device scratch not looked up (bind first)");
  hipStream_t st = (hipStream_t)stream;
  double* y = h->d_scratch;  // k_perm_in writes every entry the sweeps read
  hipLaunchKernelGGL(k_perm_in, dim3((unsigned)((np * nrhs + 255) / 256)), dim3(256), 0, st, d_b,
                     h->d_perm, n, np, nrhs, y, np * nrhs);
  for (int32_t g0 = 0; g0 < nrhs; g0 += SR) launch_sweeps(h, y, std::min<int32_t>(SR, nrhs - g0), g0, st);
  hipLaunchKernelGGL(k_perm_out, dim3((unsigned)((np * nrhs + 255) / 256)), dim3(256), 0, st, y,
                     h->d_perm, h->d_info, n, np, nrhs, d_b, np * nrhs);
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_logdet_backward(stc_handle* h, const double* d_gbar, double* d_grad_values, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_gbar || !d_grad_values) return fail(STC_ERR_ARG, "null pointer");
  if (!h->factored) return fail(STC_ERR_STATE, "logdet backward before factorize");
  hipStream_t st = (hipStream_t)stream;
  hipGraphExec_t ex;
  rc = get_back_graph(h, &ex);
  if (rc) return rc;
  HIPCHK(hipGraphLaunch(ex, st));
  h->zs_ready = true;
  h->last_stream = st;
  const int64_t qnz = h->sym.qnz;
  const int64_t grid = std::min<int64_t>(4096, (qnz + 255) / 256);
  hipLaunchKernelGGL(k_logdet_grad, dim3((unsigned)grid), dim3(256), 0, st, h->d_zs, h->d_vmap,
                     h->d_bdiag, d_gbar, h->d_info, qnz, d_grad_values);
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_selinv(stc_handle* h, double* d_diag, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h->factored) return fail(STC_ERR_STATE, "selected inversion before factorize");
  hipStream_t st = (hipStream_t)stream;
  hipGraphExec_t ex;
  rc = get_back_graph(h, &ex);
  if (rc) return rc;
  HIPCHK(hipGraphLaunch(ex, st));
  h->zs_ready = true;
  h->last_stream = st;
  if (d_diag) {
    const int64_t np = padded_n(h);
    const int64_t grid = std::min<int64_t>(4096, (np + 255) / 256);
    hipLaunchKernelGGL(k_selinv_diag, dim3((unsigned)grid), dim3(256), 0, st, h->d_zs, h->d_perm, np, h->plan.nb,
                       h->d_info, d_diag);
  }
  HIPCHK(hipGetLastError());
  return 0;
}

int stc_get_selinv(stc_handle* h, double* h_Zx, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h_Zx) return fail(STC_ERR_ARG, "null output");
  if (!h->zs_ready) return fail(STC_ERR_STATE, "selected inverse export before stc_selinv");
  std::vector<double> store((size_t)h->plan.store);
  HIPCHK(hipMemcpyAsync(store.data(), h->d_zs, sizeof(double) * store.size(), hipMemcpyDeviceToHost,
                        (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  int32_t info = 0;
  HIPCHK(hipMemcpy(&info, h->d_info, sizeof(int32_t), hipMemcpyDeviceToHost));
  const auto& lm = h->plan.lmap;
  for (size_t q = 0; q < lm.size(); ++q) h_Zx[q] = info ? std::nan("") : store[(size_t)lm[q]];
  return 0;
}

int stc_info(stc_handle* h, int32_t* info) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!info) return fail(STC_ERR_ARG, "null output");
  if (!h->factored) return fail(STC_ERR_STATE, "info before factorize");
  HIPCHK(hipStreamSynchronize(h->last_stream));
  HIPCHK(hipMemcpy(info, h->d_info, sizeof(int32_t), hipMemcpyDeviceToHost));
  return 0;
}

int stc_get_factor(stc_handle* h, double* h_Lx, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h_Lx) return fail(STC_ERR_ARG, "null output");
  if (!h->factored) return fail(STC_ERR_STATE, "factor export before factorize");
  std::vector<double> store((size_t)h->plan.store);
  HIPCHK(hipMemcpyAsync(store.data(), h->d_store, sizeof(double) * store.size(), hipMemcpyDeviceToHost,
                        (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  const auto& lm = h->plan.lmap;
  for (size_t q = 0; q < lm.size(); ++q) h_Lx[q] = store[(size_t)lm[q]];
  return 0;
}

int stc_get_batch_factor(stc_handle* h, int32_t member, double* h_Lx, void* stream) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h_Lx) return fail(STC_ERR_ARG, "null output");
  if (!h->factored) return fail(STC_ERR_STATE, "factor export before factorize");
  if (member < 0 || member >= h->batch) return fail(STC_ERR_ARG, "member out of [0, bound batch)");
  std::vector<double> store((size_t)h->plan.store);
  HIPCHK(hipMemcpyAsync(store.data(), h->d_store + (int64_t)member * h->plan.store, sizeof(double) * store.size(),
                        hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  const auto& lm = h->plan.lmap;
  for (size_t q = 0; q < lm.size(); ++q) h_Lx[q] = store[(size_t)lm[q]];
  return 0;
}

int stc_get_sizes(const stc_handle* h, int64_t* z) {
  if (!h || !z) return fail(STC_ERR_ARG, "null argument");
  const Symbolic& s = h->sym;
  int64_t rows = 0;
  for (const TileInfo& t : s.tiles) rows += t.cnt;
  int64_t v[16] = {s.n, s.qnz, s.lnz, s.nb, s.NT, (int64_t)s.tiles.size(), rows,
                   (int64_t)(s.tasks.size() / 4), s.mode, s.route, s.ndense, s.method, s.tact,
                   h->plan.store, (int64_t)h->plan.levels.size(),
                   (int64_t)(h->sfwd_nstep.size() + h->sbwd_nstep.size())};
  std::memcpy(z, v, sizeof(v));
  return 0;
}

int stc_get_grid_positions(const stc_handle* h, int64_t* pos, int64_t* align) {
  if (!h || !pos) return fail(STC_ERR_ARG, "null argument");
  for (int64_t j = 0; j < h->sym.n; ++j) pos[j] = grid_pos(h->sym, j);
  if (align) *align = h->sym.align;
  return 0;
}

int stc_get_features(const stc_handle* h, double* f) {
  if (!h || !f) return fail(STC_ERR_ARG, "null argument");
  f[0] = h->sym.phi;
  f[1] = h->sym.rho;
  f[2] = h->sym.sigma;
  return 0;
}

int stc_get_perm(const stc_handle* h, int32_t* perm) {
  if (!h || !perm) return fail(STC_ERR_ARG, "null argument");
  std::copy(h->sym.perm.begin(), h->sym.perm.end(), perm);
  return 0;
}

int stc_get_etree(const stc_handle* h, int32_t* parent) {
  if (!h || !parent) return fail(STC_ERR_ARG, "null argument");
  std::copy(h->sym.parent.begin(), h->sym.parent.end(), parent);
  return 0;
}

int stc_get_L_pattern(const stc_handle* h, int64_t* colptr, int32_t* rowind) {
  if (!h || !colptr || !rowind) return fail(STC_ERR_ARG, "null argument");
  std::copy(h->sym.lp.begin(), h->sym.lp.end(), colptr);
  std::copy(h->sym.li.begin(), h->sym.li.end(), rowind);
  return 0;
}

int stc_get_tiles(const stc_handle* h, int32_t* m, int32_t* k, int32_t* cnt, int32_t* true_cnt,
                  int8_t* contig, int64_t* roff, int32_t* rows, int32_t* kd) {
  if (!h || !m || !k || !cnt || !true_cnt || !contig || !roff || !rows || !kd)
    return fail(STC_ERR_ARG, "null argument");
  const Symbolic& s = h->sym;
  for (size_t t = 0; t < s.tiles.size(); ++t) {
    m[t] = s.tiles[t].m;
    k[t] = s.tiles[t].k;
    cnt[t] = s.tiles[t].cnt;
    true_cnt[t] = s.tiles[t].true_cnt;
    contig[t] = s.tiles[t].contig;
    roff[t] = s.tiles[t].roff;
  }
  roff[s.tiles.size()] = (int64_t)s.rows.size();
  std::copy(s.rows.begin(), s.rows.end(), rows);
  std::copy(s.kd.begin(), s.kd.end(), kd);
  return 0;
}

int stc_get_tasks(const stc_handle* h, int32_t* tasks) {
  if (!h || !tasks) return fail(STC_ERR_ARG, "null argument");
  std::copy(h->sym.tasks.begin(), h->sym.tasks.end(), tasks);
  return 0;
}

// Host check of the reverse-mode plan: levels run in order (one contraction
// launch each, then a fold launch where tasks were split).
int stc_check_backward(const stc_handle* h, int64_t* stats) {
  if (!h || !stats) return fail(STC_ERR_ARG, "null argument");
  const BackPlan& b = h->back;
  const int64_t nb = h->plan.nb;
  enum { BUF_Z = 1, BUF_G = 2, BUF_M = 3, BUF_P = 4 };
  // every term belongs to exactly one task
  std::vector<int32_t> owner(b.terms.size(), 0);
  for (const ConTask& t : b.tasks) {
    if (t.t_begin < 0 || t.t_end > (int32_t)b.terms.size() || t.t_begin > t.t_end)
      return fail(STC_ERR_SCHEDULE, "reverse-mode task with a term range outside the terms");
    for (int32_t x = t.t_begin; x < t.t_end; ++x) owner[(size_t)x]++;
  }
  for (int32_t o : owner)
    if (o != 1) return fail(STC_ERR_SCHEDULE, "a reverse-mode term belongs to no task or to several");
  // the contraction kernel streams K chunks across a task's terms and reads
  // the next term's first chunk during a term's last: every term has one
  for (const ConTerm& c : b.terms)
    if (c.K < 1 || c.K > nb) return fail(STC_ERR_SCHEDULE, "a reverse-mode term's contraction length is outside 1..n_b");
  // level at which each Z / M tile is written: M tiles and the diagonal H_k
  // at level 1 (G_k by the inverses before it, level 0), the rest once each
  std::map<std::pair<int32_t, int64_t>, int32_t> written;  // (buffer, offset) -> level
  auto key = [](int32_t buf, int64_t off) { return std::make_pair(buf == BUF_G ? (int32_t)BUF_M : buf, off); };
  for (int32_t k = 0; k < h->plan.NT; ++k) written[key(BUF_G, (int64_t)k * nb * nb)] = 0;
  int64_t reads = 0, slots_used = 0;
  for (size_t L = 1; L < b.level_items.size(); ++L) {
    const std::vector<int32_t>& it = b.level_items[L];
    std::vector<int32_t> ids;
    for (size_t q = 0; q < it.size(); q += 3) ids.push_back(it[q]);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    std::vector<std::pair<int64_t, int64_t>> slot_rng;
    std::vector<std::pair<int32_t, int64_t>> outs;
    for (int32_t id : ids) {
      const ConTask& t = b.tasks[(size_t)id];
      // inputs: Z tiles written at an earlier level, M and G tiles before the
      // contraction levels
      for (int32_t x = t.t_begin; x < t.t_end; ++x) {
        const ConTerm& c = b.terms[(size_t)x];
        for (const auto& in : {std::make_pair(c.a_buf, c.a_off), std::make_pair(c.b_buf, c.b_off)}) {
          if (in.first == 0) continue;  // the factor itself
          auto w = written.find(key(in.first, in.second));
          if (w == written.end() || w->second >= (int32_t)L)
            return fail(STC_ERR_SCHEDULE, "reverse-mode level " + std::to_string(L) +
                                              " reads a tile not written at an earlier level");
          ++reads;
        }
      }
      if (t.c_buf == BUF_P) {
        if (t.c_off < 0 || t.c_off + (int64_t)t.c_rows * nb > b.slots)
          return fail(STC_ERR_SCHEDULE, "reverse-mode partial slot outside the slot scratch");
        slot_rng.emplace_back(t.c_off, t.c_off + (int64_t)t.c_rows * nb);
      } else {
        outs.push_back(key(t.c_buf, t.c_off));
      }
    }
    std::sort(slot_rng.begin(), slot_rng.end());
    for (size_t i = 1; i < slot_rng.size(); ++i)
      if (slot_rng[i].first < slot_rng[i - 1].second)
        return fail(STC_ERR_SCHEDULE, "reverse-mode partial slots of one level overlap");
    slots_used += (int64_t)slot_rng.size();
    for (const auto& o : outs) {
      auto w = written.find(o);
      // the diagonal Z_kk accumulates into H_k, written at level 1
      const bool acc_diag = w != written.end() && w->second == 1 && o.first == BUF_Z && L > 1;
      if (w != written.end() && !acc_diag)
        return fail(STC_ERR_SCHEDULE, "a reverse-mode tile is written twice");
      written[o] = (int32_t)L;
    }
    if (outs.size() != std::set<std::pair<int32_t, int64_t>>(outs.begin(), outs.end()).size())
      return fail(STC_ERR_SCHEDULE, "two tasks of one reverse-mode level write one tile");
    // folds of this level: each adds slots that this level's parts wrote to
    // a tile this level wrote
    if (L < b.fold_items.size())
      for (size_t q = 0; q < b.fold_items[L].size(); q += 3) {
        const FoldTask& f = b.folds[(size_t)b.fold_items[L][q]];
        if (std::find(outs.begin(), outs.end(), key(f.c_buf, f.c_off)) == outs.end())
          return fail(STC_ERR_SCHEDULE, "a fold adds to a tile its level does not write");
        for (int32_t x = 0; x < f.nslots; ++x) {
          const int64_t lo = f.slot_off + (int64_t)x * f.c_rows * nb;
          if (!std::binary_search(slot_rng.begin(), slot_rng.end(), std::make_pair(lo, lo + (int64_t)f.c_rows * nb)))
            return fail(STC_ERR_SCHEDULE, "a fold reads a slot no part of its level writes");
        }
      }
  }
  stats[0] = (int64_t)b.level_items.size();
  stats[1] = (int64_t)b.tasks.size();
  stats[2] = reads;
  stats[3] = (int64_t)b.folds.size();
  stats[4] = slots_used;
  return 0;
}

int stc_check_solve_schedule(const stc_handle* h, int64_t* stats) {
  if (!h || !stats) return fail(STC_ERR_ARG, "null argument");
  int64_t st[4] = {0, 0, 0, 0};
  int rc = check_sweep(h, true, h->sfwd_items, h->sfwd_ptr, h->sfwd_nstep, h->sfwd_tl, SCH, st);
  if (rc) return rc;
  rc = check_sweep(h, false, h->sbwd_items, h->sbwd_ptr, h->sbwd_nstep, h->sbwd_tl, SBC, st);
  if (rc) return rc;
  std::memcpy(stats, st, sizeof(st));
  return 0;
}

int stc_check_schedule(const stc_handle* h, int64_t* stats) {
  if (!h || !stats) return fail(STC_ERR_ARG, "null argument");
  const Plan& p = h->plan;
  std::vector<KernelNode> dag;
  kernel_dag(p, &dag);
  const size_t N = dag.size();
  // objects: tiles by store offset, per object the nodes that read and that
  // write it; partial slots as ranges of the slot memory, which slots share
  std::map<int64_t, std::vector<std::pair<int32_t, bool>>> touch;
  std::vector<std::vector<std::pair<int64_t, bool>>> acc(N);
  struct SlotUse {
    int64_t lo, hi;
    int32_t node;
    bool write;
  };
  std::vector<SlotUse> slot_use;
  for (size_t x = 0; x < N; ++x) {
    const Level& lv = p.levels[(size_t)dag[x].level];
    auto& a = acc[x];
    if (dag[x].kind == 0) {
      for (int32_t k : lv.potrf) a.emplace_back((int64_t)k * p.nb * p.nb, true);
    } else if (dag[x].kind == 2) {
      for (size_t q = 0; q < lv.trsm_items.size(); q += 2) {
        const TrsmTask& t = p.trsm[(size_t)lv.trsm_items[q]];
        a.emplace_back(t.l_off, false);
        a.emplace_back(t.x_off, true);
      }
    } else {
      for (const std::vector<int32_t>* v : {&lv.big_items, &lv.upd_items}) {
        const size_t nl = 4 * (size_t)(v == &lv.big_items ? lv.big_last : lv.upd_last);
        for (size_t q = 0; q < v->size(); q += 4) {
          if ((q < nl) != (dag[x].kind == 3)) continue;
          const UpdTask& u = p.upd[(size_t)(*v)[q]];
          a.emplace_back(u.c_off, true);
          for (int32_t c = u.c_begin; c < u.c_end; ++c) {
            a.emplace_back(p.contribs[(size_t)c].a_off, false);
            a.emplace_back(p.contribs[(size_t)c].b_off, false);
          }
          const int64_t slot = (int64_t)u.c_rows * p.nb;
          if (u.nsplit > 1) slot_use.push_back({u.part_off, u.part_off + (u.nsplit - 1) * slot, (int32_t)x, true});
          if (u.in_npart > 0) slot_use.push_back({u.in_part_off, u.in_part_off + u.in_npart * slot, (int32_t)x, false});
        }
      }
    }
    std::sort(a.begin(), a.end());
    // an object both read and written by one node counts as written
    std::vector<std::pair<int64_t, bool>> m;
    for (const auto& e : a) {
      if (!m.empty() && m.back().first == e.first) m.back().second = m.back().second || e.second;
      else m.push_back(e);
    }
    a.swap(m);
    for (const auto& e : a) touch[e.first].emplace_back((int32_t)x, e.second);
  }
  // ancestors of every node
  const size_t W = N / 64 + 1;
  std::vector<uint64_t> anc(N * W, 0);
  int64_t edges = 0;
  for (size_t x = 0; x < N; ++x)
    for (int32_t d : dag[x].deps) {
      if (d < 0 || (size_t)d >= x) return fail(STC_ERR_SCHEDULE, "kernel graph edge to a later node");
      ++edges;
      for (size_t w = 0; w < W; ++w) anc[x * W + w] |= anc[(size_t)d * W + w];
      anc[x * W + (size_t)d / 64] |= uint64_t(1) << (d % 64);
    }
  auto ordered = [&](int32_t a, int32_t b) {  // a < b
    return (anc[(size_t)b * W + (size_t)a / 64] >> (a % 64)) & 1;
  };
  std::sort(slot_use.begin(), slot_use.end(), [](const SlotUse& a, const SlotUse& b) {
    return std::tie(a.lo, a.hi, a.node, a.write) < std::tie(b.lo, b.hi, b.node, b.write);
  });
  slot_use.erase(std::unique(slot_use.begin(), slot_use.end(),
                             [](const SlotUse& a, const SlotUse& b) {
                               return a.lo == b.lo && a.hi == b.hi && a.node == b.node && a.write == b.write;
                             }),
                 slot_use.end());
  for (const SlotUse& g : slot_use)
    if (g.lo < 0 || g.hi > p.parts || g.lo >= g.hi) return fail(STC_ERR_SCHEDULE, "partial slot outside the slot memory");
  // every two uses of overlapping slot memory, one writing, are ordered
  int64_t slot_pairs = 0;
  for (size_t i = 0; i < slot_use.size(); ++i)
    for (size_t j = i + 1; j < slot_use.size() && slot_use[j].lo < slot_use[i].hi; ++j) {
      const SlotUse &g = slot_use[i], &k = slot_use[j];
      if ((!g.write && !k.write) || g.node == k.node) {
        if (g.node == k.node && (g.write || k.write))
          return fail(STC_ERR_SCHEDULE, "one kernel writes and reads overlapping partial slots");
        continue;
      }
      ++slot_pairs;
      const int32_t a = std::min(g.node, k.node), b = std::max(g.node, k.node);
      if (!ordered(a, b))
        return fail(STC_ERR_SCHEDULE, "unordered kernels (level " + std::to_string(dag[(size_t)a].level) + ", kind " +
                                          std::to_string(dag[(size_t)a].kind) + ") and (level " +
                                          std::to_string(dag[(size_t)b].level) + ", kind " +
                                          std::to_string(dag[(size_t)b].kind) + ") share partial-slot memory");
    }
  for (const auto& kv : touch) {
    const auto& v = kv.second;
    for (size_t i = 0; i < v.size(); ++i)
      for (size_t j = i + 1; j < v.size(); ++j) {
        if (!v[i].second && !v[j].second) continue;
        const int32_t a = std::min(v[i].first, v[j].first), b = std::max(v[i].first, v[j].first);
        if (a == b) continue;
        if (dag[(size_t)a].level == dag[(size_t)b].level)
          return fail(STC_ERR_SCHEDULE, "kernels of level " + std::to_string(dag[(size_t)a].level) +
                                            " touch one object, one of them writing it");
        if (!ordered(a, b))
          return fail(STC_ERR_SCHEDULE, "unordered kernels (level " + std::to_string(dag[(size_t)a].level) +
                                            ", kind " + std::to_string(dag[(size_t)a].kind) + ") and (level " +
                                            std::to_string(dag[(size_t)b].level) + ", kind " +
                                            std::to_string(dag[(size_t)b].kind) + ") share an object");
      }
  }
  int64_t unordered = 0;
  for (size_t b = 0; b < N; ++b)
    for (size_t a = 0; a < b; ++a) unordered += ordered((int32_t)a, (int32_t)b) ? 0 : 1;
  stats[0] = (int64_t)N;
  stats[1] = edges;
  stats[2] = unordered;
  stats[3] = (int64_t)touch.size();
  stats[4] = slot_pairs;
  return 0;
}

int stc_get_plan_stats(const stc_handle* h, int64_t* st) {
  if (!h || !st) return fail(STC_ERR_ARG, "null argument");
  const Plan& p = h->plan;
  int64_t split = 0, sep = 0;
  for (const UpdTask& u : p.upd) split += u.nsplit > 1 ? 1 : 0;
  for (const LevelOffsets& L : h->lv) {
    const bool early = L.g_cnt > L.g_last || L.u_cnt > L.u_last;
    sep += (L.g_last + L.u_last > 0 && early) ? 1 : 0;
  }
  std::vector<KernelNode> dag;
  kernel_dag(p, &dag);
  int64_t unshared = 0;
  for (const UpdTask& u : p.upd) unshared += u.nsplit > 1 ? (int64_t)(u.nsplit - 1) * u.c_rows * p.nb : 0;
  st[0] = split;
  st[1] = p.parts;
  st[2] = sep;
  st[3] = (int64_t)dag.size();
  st[4] = unshared;
  return 0;
}

int stc_get_work(const stc_handle* h, double* w) {
  if (!h || !w) return fail(STC_ERR_ARG, "null argument");
  const Plan& p = h->plan;
  const double q = (double)h->sym.qnz;
  w[0] = p.flops_update;
  w[1] = p.flops_potrf;
  w[2] = p.flops_trsm;
  w[3] = p.flops_tile;
  w[4] = p.flops_exact;
  w[5] = p.bytes_update;
  w[6] = 16.0 * q + 8.0 * (double)p.store;  // values and their block entries read, the store written once
  w[7] = (double)h->lv.size();
  w[8] = h->back.flops;
  w[9] = (double)(h->back_level_ptr.size() - 1);
  return 0;
}

int stc_profile_factorize(stc_handle* h, const double* d_values, void* stream, double* kind_ms,
                          int64_t* kind_launches, double* kind_flops) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!d_values || !kind_ms || !kind_launches || !kind_flops) return fail(STC_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  Prof prof;
  rc = run_factor(h, d_values, 1, st, &prof);
  if (rc == 0) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(STC_ERR_HIP, hipGetErrorString(e));
  }
  for (int k = 0; k < kKinds; ++k) {
    kind_ms[k] = 0.0;
    kind_launches[k] = 0;
    kind_flops[k] = 0.0;
  }
  for (auto& m : prof.marks) {
    float t = 0.f;
    if (rc == 0 && hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
      kind_ms[m.kind] += t;
      kind_launches[m.kind] += 1;
      kind_flops[m.kind] += m.flops;
    }
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  if (rc) return rc;
  h->last_stream = st;
  h->factored = true;
  h->zs_ready = false;
  h->fact_members = std::max<int32_t>(h->fact_members, 1);
  return 0;
}

int stc_fp64_mfma_peak(void* stream, double* tflops) {
  if (!tflops) return fail(STC_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = cus * 8;
  const int32_t iters = 2000;
  double* sink = nullptr;  // never written (the guard in the kernel is false)
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  hipLaunchKernelGGL(k_mfma_issue, dim3(blocks), dim3(256), 0, st, sink, iters, 1.0);
  HIPCHK(hipEventRecord(a, st));
  hipLaunchKernelGGL(k_mfma_issue, dim3(blocks), dim3(256), 0, st, sink, iters, 1.0);
  HIPCHK(hipEventRecord(b, st));
  HIPCHK(hipEventSynchronize(b));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  const double flops = (double)blocks * 4 /* waves */ * iters * 16 * (16.0 * 16 * 4 * 2);
  *tflops = flops / (ms * 1e-3) / 1e12;
  return 0;
}

int stc_save(const stc_handle* h, const char* path) {
  if (!h || !path) return fail(STC_ERR_ARG, "null argument");
  try {
    std::vector<char> buf;
    stc_handle* m = const_cast<stc_handle*>(h);  // serialization only reads the fields it visits
    serialize_plan(m->sym, m->plan, m->back, &buf);
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(STC_ERR_ARG, std::string("cannot open ") + path + " for writing");
    const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
    const int cl = std::fclose(f);
    if (w != buf.size() || cl != 0) return fail(STC_ERR_ARG, std::string("short write to ") + path);
    return 0;
  } catch (const std::bad_alloc&) {
    return fail(STC_ERR_ALLOC, "host allocation failed while saving the analysis");
  }
}

int stc_load(const char* path, stc_handle** out) {
  if (!path || !out) return fail(STC_ERR_ARG, "null argument");
  *out = nullptr;
  try {
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(STC_ERR_ARG, std::string("cannot open ") + path);
    std::vector<char> buf;
    long sz = -1;
    if (std::fseek(f, 0, SEEK_END) == 0) sz = std::ftell(f);
    if (sz < 0 || std::fseek(f, 0, SEEK_SET) != 0) {
      std::fclose(f);
      return fail(STC_ERR_ARG, std::string("cannot read ") + path);
    }
    buf.resize((size_t)sz);
    const size_t got = sz ? std::fread(buf.data(), 1, (size_t)sz, f) : 0;
    std::fclose(f);
    if (got != (size_t)sz) return fail(STC_ERR_ARG, std::string("short read from ") + path);
    auto* h = new stc_handle();
    std::string why;
    const int rc = deserialize_plan(buf.data(), buf.size(), &h->sym, &h->plan, &h->back, &why);
    if (rc) {
      delete h;
      return fail(rc, why);
    }
    finish_handle(h);
    *out = h;
    return 0;
  } catch (const std::bad_alloc&) {
    return fail(STC_ERR_ALLOC, "host allocation failed while loading the analysis");
  }
}

void stc_destroy(stc_handle* h) { delete h; }

}  // extern "C"
