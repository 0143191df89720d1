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

// ---------------------------------------------------------------------------
// fused update: C -= sum_c A_c B_c^T on one 64 x 64 block of an output tile
// ---------------------------------------------------------------------------

constexpr int UB = 64;   // output block
constexpr int UKT = 16;  // K chunk staged in LDS
constexpr int ULD = UKT + 1;

constexpr int UPD_LDS = 2 * UB * ULD + UB;  // doubles: As, Bs, two int maps

template <int NB>
__device__ __forceinline__ void dev_update(int32_t it, const int32_t* __restrict__ items,
                                           const UpdTaskD* __restrict__ tasks,
                                           const ContribD* __restrict__ contribs,
                                           const int32_t* __restrict__ maps,
                                           double* __restrict__ S, double* smem) {
  double* As = smem;
  double* Bs = smem + UB * ULD;
  int32_t* arow = reinterpret_cast<int32_t*>(smem + 2 * UB * ULD);
  int32_t* bcol = arow + UB;
  const int32_t task = items[3 * it], bx = items[3 * it + 1], by = items[3 * it + 2];
  const UpdTaskD u = tasks[task];
  const int32_t r0 = bx * UB, c0 = by * UB;
  const int32_t ncols = u.diag ? u.c_rows : NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  for (int32_t ci = u.c_begin; ci < u.c_end; ++ci) {
    const ContribD c = contribs[ci];
    int32_t src = -1;
    if (tid < UB) {
      int32_t r = r0 + tid;
      if (r < u.c_rows) src = c.rowmap < 0 ? (r < c.a_rows ? r : -1) : maps[c.rowmap + r];
      arow[tid] = src;
    } else if (tid < 2 * UB) {
      int32_t cc = c0 + tid - UB;
      if (cc < ncols) src = c.colmap < 0 ? (cc < c.b_rows ? cc : -1) : maps[c.colmap + cc];
      bcol[tid - UB] = src;
    }
    // block-wide: does any gathered A row and any gathered B row land here?
    const int anyA = __syncthreads_or(tid < UB && src >= 0);
    const int anyB = __syncthreads_or(tid >= UB && tid < 2 * UB && src >= 0);
    if (!(anyA && anyB)) continue;
    const double* A = S + c.a_off;
    const double* B = S + c.b_off;
    for (int k0 = 0; k0 < NB; k0 += UKT) {
      // 64 rows x 16 columns per operand: 4 consecutive doubles per thread
      {
        const int row = tid >> 2, kq = (tid & 3) * 4;
        const int32_t sa = arow[row], sb = bcol[row];
        double2 a0 = make_double2(0.0, 0.0), a1 = a0, b0 = a0, b1 = a0;
        if (sa >= 0) {
          const double2* pa = reinterpret_cast<const double2*>(A + (int64_t)sa * NB + k0 + kq);
          a0 = pa[0];
          a1 = pa[1];
        }
        if (sb >= 0) {
          const double2* pb = reinterpret_cast<const double2*>(B + (int64_t)sb * NB + k0 + kq);
          b0 = pb[0];
          b1 = pb[1];
        }
        double* da = As + row * ULD + kq;
        double* db = Bs + row * ULD + kq;
        da[0] = a0.x; da[1] = a0.y; da[2] = a1.x; da[3] = a1.y;
        db[0] = b0.x; db[1] = b0.y; db[2] = b1.x; db[3] = b1.y;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < UKT; kk += 4) {
        // A fragment: lane holds A[i = lane % 16][k = lane / 16]
        // B fragment: lane holds B[k = lane / 16][j = lane % 16] = Bop[j][k]
        double af[2], bf[2];
        for (int a = 0; a < 2; ++a) af[a] = As[(wr + a * 16 + (lane & 15)) * ULD + kk + (lane >> 4)];
        for (int b = 0; b < 2; ++b) bf[b] = Bs[(wc + b * 16 + (lane & 15)) * ULD + kk + (lane >> 4)];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  // epilogue: lane holds D[i][j] with j = lane % 16, i = lane / 16 + 4 e
  double* C = S + u.c_off;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) {
        const int32_t i = r0 + wr + a * 16 + (lane >> 4) + 4 * e;
        const int32_t j = c0 + wc + b * 16 + (lane & 15);
        if (i < u.c_rows && j < ncols && (!u.diag || j <= i)) C[(int64_t)i * NB + j] -= acc[a][b][e];
      }
}

// ---------------------------------------------------------------------------
// POTRF of diagonal tiles: right-looking over 32-column panels held in LDS;
// the trailing update runs on FP64 MFMA from the LDS panel.  As a by-product
// the inverse of every 32 x 32 diagonal block of L is written to dinv
// (row-major, block J at dinv + J*32*32), for the blocked TRSM.
// ---------------------------------------------------------------------------

constexpr int PW = 32;
constexpr int PLD = PW + 1;

// broadcast a double from a fixed lane of the wave (readlane on both halves)
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Cholesky of the 32 x 32 block held in P's first 32 rows, by the 32 low
// lanes of one wave, row r in lane r's registers; then the inverse of the
// factor, column c in lane c's registers.  Writes L (lower, diagonal
// included) back to P, the inverse to Z (row-major 32 x 32, stride PLD).
// Returns the pivot that failed first as a 0-based column, or -1.
__device__ __forceinline__ int chol32_wave(double* P, double* Z, int lane) {
  double a[PW];
  const int r = lane & 31;
#pragma unroll
  for (int j = 0; j < PW; ++j) a[j] = (j <= r) ? P[r * PLD + j] : 0.0;
  int bad = -1;
#pragma unroll
  for (int c = 0; c < PW; ++c) {
    const double d = lane_bcast(a[c], c);
    if (bad < 0 && (!(d > 0.0) || !isfinite(d))) bad = c;
    const double ljj = sqrt(d);
    a[c] = (r > c) ? a[c] / ljj : ((r == c) ? ljj : 0.0);
#pragma unroll
    for (int j = c + 1; j < PW; ++j) {
      const double ljc = lane_bcast(a[c], j);
      a[j] -= a[c] * ljc;
    }
  }
  // inverse: lane c solves L z = e_c
  double z[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) {
    double v = (i == r) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < i; ++q) v -= lane_bcast(a[q], i) * z[q];
    z[i] = v / lane_bcast(a[i], i);
  }
  if (lane < PW) {
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      P[r * PLD + j] = (j <= r) ? a[j] : 0.0;
      Z[j * PLD + r] = z[j];
    }
  }
  return bad;
}

template <int NB>
constexpr int potrf_lds() { return NB * PLD + PW * PLD; }

template <int NB>
__device__ __forceinline__ void dev_potrf(int32_t k, double* __restrict__ S,
                                          double* __restrict__ dinv_m, int32_t* __restrict__ inf,
                                          int32_t nreal, double* smem) {
  double* P = smem;
  double* Z = smem + NB * PLD;
  double* A = S + (int64_t)k * NB * NB;
  double* dinv = dinv_m + (int64_t)k * NB * PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j0 = 0; j0 < NB; j0 += PW) {
    const int pr = NB - j0;  // panel rows j0..NB-1
    for (int x = tid; x < pr * PW; x += 256) {
      const int r = x / PW, c = x % PW;
      P[r * PLD + c] = A[(int64_t)(j0 + r) * NB + j0 + c];
    }
    __syncthreads();
    if (wave == 0) {
      const int bad = chol32_wave(P, Z, lane);
      if (lane == 0 && bad >= 0 && k * NB + j0 + bad < nreal) atomicMin(inf, k * NB + j0 + bad + 1);
    }
    __syncthreads();
    // rows below the diagonal block: P_below <- P_below inv(L_top)^T on MFMA;
    // each wave owns whole 16-row blocks, reads them fully, then overwrites
    const int rb = (pr - PW) / 16;
    for (int t = wave; t < rb; t += 4) {
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
    // write the panel back (lower part of its diagonal block)
    for (int x = tid; x < pr * PW; x += 256) {
      const int r = x / PW, c = x % PW;
      if (c <= r || r >= PW) A[(int64_t)(j0 + r) * NB + j0 + c] = P[r * PLD + c];
    }
    // trailing update A[j0+32:, j0+32:] -= P[32:] P[32:]^T, lower 16 x 16
    // tiles distributed over the four waves
    const int tr = (NB - j0 - PW) / 16;
    const int ntile = tr * (tr + 1) / 2;
    for (int t = wave; t < ntile; t += 4) {
      int ti = 0, rem = t;
      while (rem > ti) {
        rem -= ti + 1;
        ++ti;
      }
      const int tj = rem;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      const double* pa = P + (PW + ti * 16 + (lane & 15)) * PLD + (lane >> 4);
      const double* pb = P + (PW + tj * 16 + (lane & 15)) * PLD + (lane >> 4);
#pragma unroll
      for (int kk = 0; kk < PW; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb[kk], acc, 0, 0, 0);
      const int gi = j0 + PW + ti * 16 + (lane >> 4), gj = j0 + PW + tj * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (ti != tj || gj <= gi + 4 * e) A[(int64_t)(gi + 4 * e) * NB + gj] -= acc[e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// TRSM: rows of a panel tile times L_kk^-T, 32 rows per work item, blocked by
// 32 columns: X_J <- (X_J - X_<J L_J,<J^T) inv(L_JJ)^T, both products on MFMA
// ---------------------------------------------------------------------------

constexpr int TR = 32;
constexpr int TLD = 4;  // row padding of the LDS copy

template <int NB>
constexpr int trsm_lds() { return TR * (NB + TLD); }

template <int NB>
__device__ __forceinline__ void dev_trsm(int32_t it, const int32_t* __restrict__ items,
                                         const TrsmTaskD* __restrict__ tasks,
                                         double* __restrict__ S,
                                         const double* __restrict__ dinv_m, double* smem) {
  constexpr int XLD = NB + TLD;
  double* X = smem;
  const TrsmTaskD t = tasks[items[2 * it]];
  const int32_t rb = items[2 * it + 1];
  const int32_t r0 = rb * TR;
  const int32_t nr = min(TR, t.rows - r0);
  double* Xg = S + t.x_off + (int64_t)r0 * NB;
  const double* L = S + t.l_off;
  const double* dinv = dinv_m + (int64_t)t.k * NB * PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int x = tid; x < TR * NB; x += 256) {
    const int r = x / NB, c = x % NB;
    X[r * XLD + c] = r < nr ? Xg[x] : 0.0;
  }
  __syncthreads();
  // each wave owns one 16 x 16 tile of the 32 x 32 block column
  const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
  for (int j0 = 0; j0 < NB; j0 += PW) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double* xa = X + (wr + (lane & 15)) * XLD + (lane >> 4);
    const double* lb = L + (int64_t)(j0 + wc + (lane & 15)) * NB + (lane >> 4);
    for (int kk = 0; kk < j0; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[kk], lb[kk], acc, 0, 0, 0);
    // Y = X_J - acc, kept in registers until every wave has read X_<J
    double y[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      y[e] = X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] - acc[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] = y[e];
    __syncthreads();
    // X_J = Y inv(L_JJ)^T
    d4 z = {0.0, 0.0, 0.0, 0.0};
    const double* ya = X + (wr + (lane & 15)) * XLD + j0 + (lane >> 4);
    const double* db = dinv + (j0 / PW) * PW * PW + (wc + (lane & 15)) * PW + (lane >> 4);
#pragma unroll
    for (int kk = 0; kk < PW; kk += 4)
      z = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[kk], db[kk], z, 0, 0, 0);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) X[(wr + (lane >> 4) + 4 * e) * XLD + j0 + wc + (lane & 15)] = z[e];
    __syncthreads();
  }
  for (int x = tid; x < nr * NB; x += 256) Xg[x] = X[(x / NB) * XLD + x % NB];
}

// ---------------------------------------------------------------------------
// one level of the schedule in one launch: work-groups [0, np) factor
// diagonal tiles, [np, np+nu) apply fused updates, the rest solve panel rows.
// POTRF work-groups come first so that the latency-bound factorizations start
// before the update work that fills the rest of the chip.
// ---------------------------------------------------------------------------

struct LevelArgs {
  const int32_t* potrf;   // block columns
  const int32_t* upd;     // triples
  const int32_t* trsm;    // pairs
  int32_t np, nu, nt;
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

template <int NB>
__global__ __launch_bounds__(256) void k_level(LevelArgs a) {
  extern __shared__ double smem[];
  const int32_t member = blockIdx.y;
  double* S = a.store + (int64_t)member * a.mstride;
  int32_t b = blockIdx.x;
  if (b < a.np) {
    dev_potrf<NB>(a.potrf[b], S, a.dinv + (int64_t)member * a.dstride, a.info + member, a.nreal,
                  smem);
    return;
  }
  b -= a.np;
  if (b < a.nu) {
    dev_update<NB>(b, a.upd, a.utasks, a.contribs, a.maps, S, smem);
    return;
  }
  b -= a.nu;
  dev_trsm<NB>(b, a.trsm, a.ttasks, S, a.dinv + (int64_t)member * a.dstride, smem);
}

// ---------------------------------------------------------------------------
// log-determinant: 2 sum log L_ii over the real rows, fixed summation order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_logdet(const double* __restrict__ store, int64_t mstride,
                                                int32_t nb, int64_t n,
                                                const int32_t* __restrict__ info,
                                                double* __restrict__ out) {
  __shared__ double part[256];
  const double* S = store + (int64_t)blockIdx.x * mstride;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
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

// turn "no failure" (still the sentinel) into 0
__global__ void k_info_finish(int32_t* info, int32_t count, int32_t big, int32_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    int32_t v = info[i] == big ? 0 : info[i];
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

__global__ void k_perm_in(const double* __restrict__ b, const int32_t* __restrict__ perm,
                          int64_t n, int64_t np, int32_t nrhs, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np * nrhs) return;
  int64_t r = i / np, a = i % np;
  y[i] = a < n ? b[r * n + perm[a]] : 0.0;
}

__global__ void k_perm_out(const double* __restrict__ y, const int32_t* __restrict__ perm,
                           int64_t n, int64_t np, int32_t nrhs, double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t r = i / n, a = i % n;
  b[r * n + perm[a]] = y[r * np + a];
}

// forward: block row m owns y_m: y_m -= sum_k L_mk y_k, then y_m <- L_mm^-1 y_m
template <int NB>
__global__ __launch_bounds__(256) void k_fwd(const int32_t* __restrict__ blks,
                                             const int32_t* __restrict__ row_ptr,
                                             const int32_t* __restrict__ row_tiles,
                                             const TileD* __restrict__ tiles,
                                             const int32_t* __restrict__ rows,
                                             const double* __restrict__ S, double* __restrict__ y,
                                             int64_t np, int32_t nrhs) {
  __shared__ double ys[NB];
  const int32_t m = blks[blockIdx.x];
  const int tid = threadIdx.x;
  const double* Lmm = S + (int64_t)m * NB * NB;
  for (int32_t r = 0; r < nrhs; ++r) {
    double* yr = y + (int64_t)r * np;
    for (int i = tid; i < NB; i += 256) ys[i] = yr[(int64_t)m * NB + i];
    __syncthreads();
    for (int32_t x = row_ptr[m]; x < row_ptr[m + 1]; ++x) {
      const TileD t = tiles[row_tiles[x]];
      const double* yk = yr + (int64_t)t.k * NB;
      for (int q = tid; q < t.cnt; q += 256) {
        const double* pr = S + t.off + (int64_t)q * NB;
        double v = 0.0;
        for (int c = 0; c < NB; ++c) v += pr[c] * yk[c];
        ys[rows[t.roff + q]] -= v;
      }
      __syncthreads();
    }
    for (int c = 0; c < NB; ++c) {
      if (tid == 0) ys[c] /= Lmm[(int64_t)c * NB + c];
      __syncthreads();
      for (int i = c + 1 + tid; i < NB; i += 256) ys[i] -= Lmm[(int64_t)i * NB + c] * ys[c];
      __syncthreads();
    }
    for (int i = tid; i < NB; i += 256) yr[(int64_t)m * NB + i] = ys[i];
    __syncthreads();
  }
}

// backward: block column k owns x_k: x_k -= sum_m L_mk^T x_m, then x_k <- L_kk^-T x_k
template <int NB>
__global__ __launch_bounds__(256) void k_bwd(const int32_t* __restrict__ blks,
                                             const int32_t* __restrict__ col_ptr,
                                             const int32_t* __restrict__ col_tiles,
                                             const TileD* __restrict__ tiles,
                                             const int32_t* __restrict__ rows,
                                             const double* __restrict__ S, double* __restrict__ y,
                                             int64_t np, int32_t nrhs) {
  __shared__ double ys[NB];
  const int32_t k = blks[blockIdx.x];
  const int tid = threadIdx.x;
  const double* Lkk = S + (int64_t)k * NB * NB;
  for (int32_t r = 0; r < nrhs; ++r) {
    double* yr = y + (int64_t)r * np;
    for (int i = tid; i < NB; i += 256) ys[i] = yr[(int64_t)k * NB + i];
    __syncthreads();
    for (int32_t x = col_ptr[k]; x < col_ptr[k + 1]; ++x) {
      const TileD t = tiles[col_tiles[x]];
      const double* ym = yr + (int64_t)t.m * NB;
      const double* P = S + t.off;
      for (int c = tid; c < NB; c += 256) {
        double v = 0.0;
        for (int q = 0; q < t.cnt; ++q) v += P[(int64_t)q * NB + c] * ym[rows[t.roff + q]];
        ys[c] -= v;
      }
      __syncthreads();
    }
    for (int c = NB - 1; c >= 0; --c) {
      if (tid == 0) ys[c] /= Lkk[(int64_t)c * NB + c];
      __syncthreads();
      for (int i = tid; i < c; i += 256) ys[i] -= Lkk[(int64_t)c * NB + i] * ys[c];
      __syncthreads();
    }
    for (int i = tid; i < NB; i += 256) yr[(int64_t)k * NB + i] = ys[i];
    __syncthreads();
  }
}

}  // namespace stc
