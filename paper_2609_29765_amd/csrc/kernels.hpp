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

template <int NB>
__global__ __launch_bounds__(256) void k_update(const int32_t* __restrict__ items,
                                                const UpdTaskD* __restrict__ tasks,
                                                const ContribD* __restrict__ contribs,
                                                const int32_t* __restrict__ maps,
                                                double* __restrict__ store, int64_t mstride) {
  __shared__ double As[UB * ULD];
  __shared__ double Bs[UB * ULD];
  __shared__ int32_t arow[UB], bcol[UB];
  double* S = store + (int64_t)blockIdx.y * mstride;
  const int32_t it = blockIdx.x;
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
// POTRF of diagonal tiles: right-looking over 32-column panels held in LDS
// ---------------------------------------------------------------------------

constexpr int PW = 32;

template <int NB>
__global__ __launch_bounds__(256) void k_potrf(const int32_t* __restrict__ ks,
                                               double* __restrict__ store, int64_t mstride,
                                               int32_t* __restrict__ info, int32_t nreal) {
  __shared__ double P[NB * (PW + 1)];
  __shared__ double dg[PW];
  double* S = store + (int64_t)blockIdx.y * mstride;
  const int32_t k = ks[blockIdx.x];
  double* A = S + (int64_t)k * NB * NB;
  const int tid = threadIdx.x;
  int32_t* inf = info + blockIdx.y;
  for (int j0 = 0; j0 < NB; j0 += PW) {
    const int pr = NB - j0;  // panel rows j0..NB-1
    for (int x = tid; x < pr * PW; x += 256) {
      int r = x / PW, c = x % PW;
      P[r * (PW + 1) + c] = A[(int64_t)(j0 + r) * NB + j0 + c];
    }
    __syncthreads();
    // left-looking inside the panel, one column at a time; the pivot's square
    // root goes to dg[] so that P's diagonal is never rewritten while read
    for (int c = 0; c < PW; ++c) {
      for (int r = c + tid; r < pr; r += 256) {
        double v = P[r * (PW + 1) + c];
        for (int p = 0; p < c; ++p) v -= P[r * (PW + 1) + p] * P[c * (PW + 1) + p];
        P[r * (PW + 1) + c] = v;
      }
      __syncthreads();
      const double d = P[c * (PW + 1) + c];
      const double ljj = sqrt(d);
      for (int r = c + 1 + tid; r < pr; r += 256) P[r * (PW + 1) + c] /= ljj;
      if (tid == 0) {
        dg[c] = ljj;
        const int32_t col = k * NB + j0 + c;
        if ((!(d > 0.0) || !isfinite(d)) && col < nreal) atomicMin(inf, col + 1);
      }
      __syncthreads();
    }
    for (int x = tid; x < pr * PW; x += 256) {
      int r = x / PW, c = x % PW;
      if (c < r) A[(int64_t)(j0 + r) * NB + j0 + c] = P[r * (PW + 1) + c];
      if (c == r) A[(int64_t)(j0 + r) * NB + j0 + c] = dg[c];
    }
    // trailing update of the lower part below/right of the panel
    const int tr = NB - j0 - PW;
    for (int x = tid; x < tr * tr; x += 256) {
      int i = x / tr, j = x % tr;
      if (j > i) continue;
      double v = 0.0;
      const double* pi = P + (PW + i) * (PW + 1);
      const double* pj = P + (PW + j) * (PW + 1);
#pragma unroll 8
      for (int p = 0; p < PW; ++p) v += pi[p] * pj[p];
      A[(int64_t)(j0 + PW + i) * NB + j0 + PW + j] -= v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// TRSM: rows of a panel tile times L_kk^-T, 32 rows per work item
// ---------------------------------------------------------------------------

constexpr int TR = 32;
constexpr int TCB = 16;

template <int NB>
__global__ __launch_bounds__(256) void k_trsm(const int32_t* __restrict__ items,
                                              const TrsmTaskD* __restrict__ tasks,
                                              double* __restrict__ store, int64_t mstride) {
  __shared__ double X[TR * (NB + 1)];
  __shared__ double Ld[TCB * (TCB + 1)];
  double* S = store + (int64_t)blockIdx.y * mstride;
  const TrsmTaskD t = tasks[items[2 * blockIdx.x]];
  const int32_t rb = items[2 * blockIdx.x + 1];
  const int32_t r0 = rb * TR;
  const int32_t nr = min(TR, t.rows - r0);
  double* Xg = S + t.x_off + (int64_t)r0 * NB;
  const double* L = S + t.l_off;
  const int tid = threadIdx.x;
  for (int x = tid; x < nr * NB; x += 256) X[(x / NB) * (NB + 1) + x % NB] = Xg[x];
  __syncthreads();
  for (int j0 = 0; j0 < NB; j0 += TCB) {
    // X[:, J] -= X[:, <J] L[J, <J]^T
    for (int x = tid; x < nr * TCB; x += 256) {
      int r = x / TCB, c = x % TCB;
      const double* lrow = L + (int64_t)(j0 + c) * NB;
      const double* xr = X + r * (NB + 1);
      double v = 0.0;
      for (int p = 0; p < j0; ++p) v += xr[p] * lrow[p];
      X[r * (NB + 1) + j0 + c] -= v;
    }
    for (int x = tid; x < TCB * TCB; x += 256) {
      int i = x / TCB, j = x % TCB;
      Ld[i * (TCB + 1) + j] = (j <= i) ? L[(int64_t)(j0 + i) * NB + j0 + j] : 0.0;
    }
    __syncthreads();
    // X[:, J] <- X[:, J] L_JJ^-T, one row per thread
    if (tid < nr) {
      double* xr = X + tid * (NB + 1) + j0;
      for (int c = 0; c < TCB; ++c) {
        double v = xr[c];
        for (int p = 0; p < c; ++p) v -= xr[p] * Ld[c * (TCB + 1) + p];
        xr[c] = v / Ld[c * (TCB + 1) + c];
      }
    }
    __syncthreads();
  }
  for (int x = tid; x < nr * NB; x += 256) Xg[x] = X[(x / NB) * (NB + 1) + x % NB];
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
