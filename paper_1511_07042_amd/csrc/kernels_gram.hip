// Tall-skinny FP64 products of the Rayleigh-Ritz step.
//
// Gram: G = Z^T Y over all n rows, Z = [z1 | z2] (nz columns), Y = [y1 | y2]
// (ny columns), interleaved row-major blocks.  This is the dense contraction
// of the enriched pencil (eq. pb-c-aux-mat: the blocks P_H A_h U^h, (U^h)^T
// A_h U^h and their M counterparts, here evaluated on the finest level), and it
// runs on the FP64 matrix cores: v_mfma_f64_16x16x4f64 takes a 16x4 slice of
// Z^T and a 4x16 slice of Y, i.e. four rows of both blocks per instruction.
// The FP64 16x16x4 result layout: lane l holds column l % 16 of rows
// (l / 16) + 4 v, v = 0..3.  Each 256-thread block owns a contiguous range of rows; its four wavefronts
// split the 16x16 output tiles by tile column.  Per-block results go to a
// partial buffer that a second kernel sums in a fixed order (deterministic).
//
// Update: U = Z Y for a small Y (the new Ritz vectors U <- [W_c, U'] Y).
#include <algorithm>
#include <cstdlib>

#include <mutex>
#include <vector>

#include "bmg_internal.h"

namespace bmg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

__device__ __forceinline__ double zcol(const double* __restrict__ z1, int w1,
                                       const double* __restrict__ z2, int w2, int64_t r, int c) {
  if (c < w1) return z1[r * w1 + c];
  c -= w1;
  if (c < w2) return z2[r * w2 + c];
  return 0.0;
}

// TI: tiles along nz (<= 6), TJW: tile columns per wavefront (<= 3).
// Rows advance 16 at a time: the fragments of four 4-row steps are loaded
// before their MFMAs are issued, so several loads are in flight per wavefront.
template <int TI, int TJW>
__global__ void __launch_bounds__(256) k_gram(int64_t n, int64_t rows_per_block, int nzp, int nyp,
                                              const double* __restrict__ z1, int w1,
                                              const double* __restrict__ z2, int w2,
                                              const double* __restrict__ y1, int v1,
                                              const double* __restrict__ y2, int v2,
                                              double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int TJ = nyp / 16;
  const int li = lane & 15;   // row of A / column of B / column of D
  const int lk = lane >> 4;   // k index of the fragment
  d4 acc[TI][TJW];
  for (int i = 0; i < TI; ++i)
    for (int t = 0; t < TJW; ++t) acc[i][t] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t rb = int64_t(blockIdx.x) * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  for (int64_t r0 = rb; r0 < re; r0 += 16) {
    double a[4][TI], b[4][TJW];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + 4 * u + lk;
      const bool ok = r < re;
#pragma unroll
      for (int i = 0; i < TI; ++i) a[u][i] = ok ? zcol(z1, w1, z2, w2, r, 16 * i + li) : 0.0;
#pragma unroll
      for (int t = 0; t < TJW; ++t) {
        const int tj = wave + 4 * t;
        b[u][t] = (ok && tj < TJ) ? zcol(y1, v1, y2, v2, r, 16 * tj + li) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < TJW; ++t) {
        if (wave + 4 * t >= TJ) continue;
#pragma unroll
        for (int i = 0; i < TI; ++i)
          acc[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][i], b[u][t], acc[i][t], 0, 0, 0);
      }
  }
  double* out = part + int64_t(blockIdx.x) * nzp * nyp;
  for (int t = 0; t < TJW; ++t) {
    const int tj = wave + 4 * t;
    if (tj >= TJ) break;
    for (int i = 0; i < TI; ++i)
      for (int v = 0; v < 4; ++v) out[(16 * i + lk + 4 * v) * nyp + 16 * tj + li] = acc[i][t][v];
  }
}

constexpr int kGramAmChunk = 16;  // rows whose products share one LDS pass
static_assert(kGramAmChunk == 16, "the levels' chunk order (DevLevel::chunk_order) is built over 16-row chunks");

// One (row, column pair) item of the products: rows r of A U and M U at
// columns 2 ch, 2 ch + 1 (FP64), the ELL row gathered against U.  With a
// compile-time width the item is straight-line code, so the items a thread
// takes in one pass have their loads in flight together.  An invalid item
// reads row r (a valid row) and returns zeros.
template <int WT>
__device__ __forceinline__ double4 am_item(int64_t r, bool valid, int W, const int* __restrict__ cols,
                                           const double* __restrict__ a, const double* __restrict__ mm,
                                           const double* __restrict__ u, int ldu, int ch,
                                           double2* diag = nullptr, const int* __restrict__ uperm = nullptr) {
  double a0 = 0.0, a1 = 0.0, m0 = 0.0, m1 = 0.0;
  const int64_t base = r * W;
  if (WT > 0) {
    int j[WT > 0 ? WT : 1];
    double av[WT > 0 ? WT : 1], mv[WT > 0 ? WT : 1];
    double2 xv[WT > 0 ? WT : 1];
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      j[k] = cols[base + k];
      av[k] = a[base + k];
      mv[k] = mm[base + k];
    }
    if (uperm != nullptr)
#pragma unroll
      for (int k = 0; k < WT; ++k) j[k] = uperm[j[k]];
#pragma unroll
    for (int k = 0; k < WT; ++k) xv[k] = *reinterpret_cast<const double2*>(u + int64_t(j[k]) * ldu + 2 * ch);
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      a0 += av[k] * xv[k].x;
      a1 += av[k] * xv[k].y;
      m0 += mv[k] * xv[k].x;
      m1 += mv[k] * xv[k].y;
    }
    if (diag) *diag = valid ? xv[0] : double2{0.0, 0.0};
  } else {
    for (int k = 0; k < W; ++k) {
      const int jj = uperm != nullptr ? uperm[cols[base + k]] : cols[base + k];
      const double av = a[base + k], mv = mm[base + k];
      const double2 xv = *reinterpret_cast<const double2*>(u + int64_t(jj) * ldu + 2 * ch);
      if (k == 0 && diag) *diag = valid ? xv : double2{0.0, 0.0};
      a0 += av * xv.x;
      a1 += av * xv.y;
      m0 += mv * xv.x;
      m1 += mv * xv.y;
    }
  }
  return valid ? double4{a0, a1, m0, m1} : double4{0.0, 0.0, 0.0, 0.0};
}

// Fused SpMM and Gram with the symmetric blocks computed once.  The Gram
// blocks of Z = [W | U] are W^T [A U | M U] and the symmetric U^T A U, U^T M U;
// the kernel computes W^T [A U | M U] and only the upper tiles of the two
// symmetric blocks.  Columns are laid out in 16-wide tiles: the chunk's rows of
// Z as [W padded to 16 TW | U padded to 16 TU] and of Y = [A U | M U] as
// [A U padded to 16 TU | M U padded to 16 TU], both staged in LDS.  The tile
// list (host-built) is split evenly over the four wavefronts, so each
// wavefront holds few accumulators; two LDS buffers alternate between chunks,
// so one barrier per chunk separates the products of a chunk from the MFMAs
// that read it, and the registers leave room for two blocks per CU (the
// gathers of one overlap the MFMAs of the other).  Partial sums per block, by
// tile, reduced in a fixed order by k_gram_sym_reduce.  uperm (nullable):
// the blocks W and U are in vertex order while the level is stored permuted;
// storage row r then reads row uperm[r].
constexpr int kSymMaxTiles = 72;
struct SymTiles {
  int T;                                         // tiles in the list
  unsigned char ti[kSymMaxTiles], tj[kSymMaxTiles];  // Z tile, Y tile
};

// LDS row strides (doubles): an odd number of 16-double groups, so the four
// rows a fragment load touches fall on alternating halves of the banks.
__host__ __device__ constexpr int sym_zp(int TW, int TU) { return 16 * ((TW + TU) | 1); }
__host__ __device__ constexpr int sym_yp(int TU) { return 16 * (2 * TU + 1); }

template <int TPW, int NB, int WT>
__global__ void __launch_bounds__(256) k_gram_sym(int64_t n, int64_t rows_per_block, SymTiles tl, int TW,
                                                  int TU, const int* __restrict__ cols,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ mm, int W,
                                                  const double* __restrict__ z1, int w1,
                                                  const double* __restrict__ u, int m, int ldu,
                                                  double* __restrict__ part,
                                                  const int* __restrict__ corder,
                                                  const int* __restrict__ uperm, int64_t part_stride) {
  constexpr int CH = kGramAmChunk;
  extern __shared__ double lds[];
  // a batch of equal-width requests: blockIdx.y picks the request, whose
  // columns start m further along each row and whose partials follow the last
  u += int64_t(blockIdx.y) * m;
  part += int64_t(blockIdx.y) * part_stride;
  const int ZP = sym_zp(TW, TU), YP = sym_yp(TU);
  double* const zs0 = lds;                 // [2][CH][ZP]
  double* const ys0 = lds + 2 * CH * ZP;   // [2][CH][YP]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int lk = lane >> 4;
  const int cpr = m / 2;
  const int items = CH * cpr;
  const int uoff = 16 * TW;   // first U column of a Z row
  const int moff = 16 * TU;   // first M U column of a Y row
  d4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  // padding columns stay zero for the whole kernel
  for (int e = threadIdx.x; e < 2 * CH * (ZP + YP); e += blockDim.x) lds[e] = 0.0;
  __syncthreads();
  const int64_t rb = int64_t(blockIdx.x) * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  int buf = 0;
  for (int64_t c0 = rb; c0 < re; c0 += CH, buf ^= 1) {
    const int64_t r0 = corder != nullptr ? int64_t(corder[c0 / CH]) * CH : c0;
    const int64_t r1 = r0 + CH < n ? r0 + CH : n;
    double* const zs = zs0 + buf * CH * ZP;
    double* const ys = ys0 + buf * CH * YP;
    // rows of W (rows past the end are zero)
    for (int e = threadIdx.x; e < CH * w1; e += blockDim.x) {
      const int rl = e / w1, c = e - (e / w1) * w1;
      const int64_t r = r0 + rl;
      const int64_t rz = uperm != nullptr && r < r1 ? int64_t(uperm[r]) : r;
      zs[rl * ZP + c] = r < r1 ? z1[rz * w1 + c] : 0.0;
    }
    // rows of A U and M U; the U row itself is the gather of the diagonal
    // slot (slot 0 of every ELL row is the row)
    for (int e0 = threadIdx.x; e0 < items; e0 += NB * 256) {
      double4 y[NB];
      double2 d[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int e = e0 + k * 256;
        const int rl = e / cpr, ch = e - (e / cpr) * cpr;
        const int64_t r = r0 + rl;
        const bool valid = e < items && r < r1;
        y[k] = am_item<WT>(valid ? r : r0, valid, W, cols, a, mm, u, ldu, ch, &d[k], uperm);
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int e = e0 + k * 256;
        if (e < items) {
          const int rl = e / cpr, ch = e - (e / cpr) * cpr;
          double* yr = ys + rl * YP;
          yr[2 * ch] = y[k].x;
          yr[2 * ch + 1] = y[k].y;
          yr[moff + 2 * ch] = y[k].z;
          yr[moff + 2 * ch + 1] = y[k].w;
          double* zr = zs + rl * ZP + uoff;
          zr[2 * ch] = d[k].x;
          zr[2 * ch + 1] = d[k].y;
        }
      }
    }
    __syncthreads();  // this buffer's rows are complete (and the other buffer is free)
#pragma unroll
    for (int q = 0; q < CH / 4; ++q) {
      const double* zq = zs + (4 * q + lk) * ZP + li;
      const double* yq = ys + (4 * q + lk) * YP + li;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wave * TPW + t;
        if (tile < tl.T)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(zq[16 * tl.ti[tile]], yq[16 * tl.tj[tile]], acc[t],
                                                        0, 0, 0);
      }
    }
  }
  double* out = part + int64_t(blockIdx.x) * tl.T * 256;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave * TPW + t;
    if (tile < tl.T)
      for (int v = 0; v < 4; ++v) out[tile * 256 + (lk + 4 * v) * 16 + li] = acc[t][v];
  }
}

// The same products and tiles with one (row, column pair) item per thread:
// a block is 16 rows x m/2 column pairs rounded up to whole wavefronts, so
// each thread forms one item per chunk with all seven gathers in flight at
// once, and the tiles are split over all of the block's wavefronts (few
// accumulators each).  The chunk's ELL rows (columns and both value arrays)
// are staged in LDS one chunk ahead: their loads are issued at the start of
// the previous chunk and stored before its barrier, so a chunk costs one
// round trip to memory (the gathers) plus its MFMAs.  The MFMA fragment
// offsets are kept in registers for the whole kernel.  Needs 16 W <= the
// block size.  Partial sums as in k_gram_sym (same tiles, same order).
template <int TPW, int WT>
__global__ void __launch_bounds__(1024) k_gram_sym1(int64_t n, int64_t rows_per_block, SymTiles tl, int TW,
                                                   int TU, const int* __restrict__ cols,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ mm, int W,
                                                   const double* __restrict__ z1, int w1,
                                                   const double* __restrict__ u, int m, int ldu,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ corder,
                                                   const int* __restrict__ uperm, int64_t part_stride) {
  constexpr int CH = kGramAmChunk;
  extern __shared__ double lds[];
  u += int64_t(blockIdx.y) * m;  // batch of equal-width requests, as in k_gram_sym
  part += int64_t(blockIdx.y) * part_stride;
  const int ZP = sym_zp(TW, TU), YP = sym_yp(TU);
  const int CW = CH * W;
  double* const zs0 = lds;                                     // [2][CH][ZP]
  double* const ys0 = zs0 + 2 * CH * ZP;                       // [2][CH][YP]
  double* const ma0 = ys0 + 2 * CH * YP;                       // [2][CH W] values of A
  double* const mm0 = ma0 + 2 * CW;                            // [2][CH W] values of M
  int* const mc0 = reinterpret_cast<int*>(mm0 + 2 * CW);       // [2][CH W] columns
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int cpr = m / 2, items = CH * cpr;
  const int uoff = 16 * TW, moff = 16 * TU;
  d4 acc[TPW];
  int zo[TPW], yo[TPW];
  bool live[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const int tile = wave * TPW + t;
    live[t] = tile < tl.T;
    zo[t] = live[t] ? 16 * tl.ti[tile] : 0;
    yo[t] = live[t] ? 16 * tl.tj[tile] : 0;
  }
  for (int e = tid; e < 2 * CH * (ZP + YP); e += nthr) lds[e] = 0.0;  // padding stays zero
  const int64_t rb = int64_t(blockIdx.x) * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  auto first_row = [&](int64_t c0) -> int64_t {
    return corder != nullptr ? int64_t(corder[c0 / CH]) * CH : c0;
  };
  // one entry (row r0 + tid / W, slot tid % W) of a chunk's ELL rows
  auto mload = [&](int64_t r0, int& pc, double& pa, double& pm) {
    const int64_t g = r0 * W + tid;
    const bool ok = g < n * W;
    pc = ok ? cols[g] : int(r0);
    pa = ok ? a[g] : 0.0;
    pm = ok ? mm[g] : 0.0;
  };
  const bool mt = tid < CW;
  if (rb < re && mt) {
    int pc;
    double pa, pm;
    mload(first_row(rb), pc, pa, pm);
    mc0[tid] = pc;
    ma0[tid] = pa;
    mm0[tid] = pm;
  }
  __syncthreads();
  const int rl = tid / cpr, ch = tid - (tid / cpr) * cpr;
  const bool wl = tid < CH * w1;
  const int wrl = wl ? tid / w1 : 0, wc = wl ? tid - (tid / w1) * w1 : 0;
  int buf = 0;
  for (int64_t c0 = rb; c0 < re; c0 += CH, buf ^= 1) {
    const int64_t r0 = first_row(c0);
    const int64_t r1 = r0 + CH < n ? r0 + CH : n;
    double* const zs = zs0 + buf * CH * ZP;
    double* const ys = ys0 + buf * CH * YP;
    // the next chunk's ELL rows: loads in flight during this chunk
    const bool more = c0 + CH < re;
    int pc = 0;
    double pa = 0.0, pm = 0.0;
    if (more && mt) mload(first_row(c0 + CH), pc, pa, pm);
    double wv = 0.0;
    if (wl) {
      const int64_t r = r0 + wrl;
      if (r < r1) wv = z1[(uperm != nullptr ? int64_t(uperm[r]) : r) * w1 + wc];
    }
    if (tid < items) {
      const int* mc = mc0 + buf * CW + rl * W;
      const double* ma = ma0 + buf * CW + rl * W;
      const double* mv = mm0 + buf * CW + rl * W;
      double a0 = 0.0, a1 = 0.0, m0 = 0.0, m1 = 0.0;
      double2 x0;
      if (WT > 0) {
        int j[WT > 0 ? WT : 1];
        double2 xv[WT > 0 ? WT : 1];
#pragma unroll
        for (int k = 0; k < WT; ++k) j[k] = uperm != nullptr ? uperm[mc[k]] : mc[k];
#pragma unroll
        for (int k = 0; k < WT; ++k) xv[k] = *reinterpret_cast<const double2*>(u + int64_t(j[k]) * ldu + 2 * ch);
#pragma unroll
        for (int k = 0; k < WT; ++k) {
          const double av = ma[k], mw = mv[k];
          a0 += av * xv[k].x;
          a1 += av * xv[k].y;
          m0 += mw * xv[k].x;
          m1 += mw * xv[k].y;
        }
        x0 = xv[0];
      } else {
        x0 = double2{0.0, 0.0};
        for (int k = 0; k < W; ++k) {
          const int jj = uperm != nullptr ? uperm[mc[k]] : mc[k];
          const double2 xv = *reinterpret_cast<const double2*>(u + int64_t(jj) * ldu + 2 * ch);
          if (k == 0) x0 = xv;  // slot 0 of every ELL row is the row itself
          a0 += ma[k] * xv.x;
          a1 += ma[k] * xv.y;
          m0 += mv[k] * xv.x;
          m1 += mv[k] * xv.y;
        }
      }
      const bool valid = r0 + rl < r1;
      double* yr = ys + rl * YP;
      double* zr = zs + rl * ZP + uoff;
      yr[2 * ch] = valid ? a0 : 0.0;
      yr[2 * ch + 1] = valid ? a1 : 0.0;
      yr[moff + 2 * ch] = valid ? m0 : 0.0;
      yr[moff + 2 * ch + 1] = valid ? m1 : 0.0;
      zr[2 * ch] = valid ? x0.x : 0.0;
      zr[2 * ch + 1] = valid ? x0.y : 0.0;
    }
    if (wl) zs[wrl * ZP + wc] = wv;
    for (int e = tid + nthr; e < CH * w1; e += nthr) {  // W wider than the block covers at once
      const int rw = e / w1, cw = e - (e / w1) * w1;
      const int64_t r = r0 + rw;
      zs[rw * ZP + cw] = r < r1 ? z1[(uperm != nullptr ? int64_t(uperm[r]) : r) * w1 + cw] : 0.0;
    }
    if (more && mt) {
      mc0[(buf ^ 1) * CW + tid] = pc;
      ma0[(buf ^ 1) * CW + tid] = pa;
      mm0[(buf ^ 1) * CW + tid] = pm;
    }
    __syncthreads();  // this chunk's rows and the next chunk's ELL rows are in LDS
#pragma unroll
    for (int q = 0; q < CH / 4; ++q) {
      const double* zq = zs + (4 * q + lk) * ZP + li;
      const double* yq = ys + (4 * q + lk) * YP + li;
      double af[TPW], bf[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        af[t] = zq[zo[t]];
        bf[t] = yq[yo[t]];
      }
#pragma unroll
      for (int t = 0; t < TPW; ++t)
        if (live[t]) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[t], bf[t], acc[t], 0, 0, 0);
    }
  }
  double* out = part + int64_t(blockIdx.x) * tl.T * 256;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave * TPW + t;
    if (live[t])
      for (int v = 0; v < 4; ++v) out[tile * 256 + (lk + 4 * v) * 16 + li] = acc[t][v];
  }
}

// G from the tile partials of k_gram_sym: each output element summed over the
// blocks in the same fixed order as k_gram_reduce, then placed in G [nz][2 m]
// (rows [W | U], columns [A U | M U]).  An element (a, b) of a symmetric block
// is computed for a <= b only and written to (a, b) and (b, a).
__global__ void __launch_bounds__(1024) k_gram_sym_reduce(const double* __restrict__ part, int nblk,
                                                          SymTiles tl, int TW, int TU, int w1, int m,
                                                          double* __restrict__ G, int64_t part_stride,
                                                          int64_t g_stride) {
  constexpr int kOut = 16, kSeg = 64;
  part += int64_t(blockIdx.y) * part_stride;  // request blockIdx.y of a batch
  G += int64_t(blockIdx.y) * g_stride;
  __shared__ double red[kSeg][kOut];
  const int el = threadIdx.x & (kOut - 1), seg = threadIdx.x / kOut;
  const int e = blockIdx.x * kOut + el;
  const int tot = tl.T * 256;
  double s = 0.0;
  if (e < tot) {
    const int64_t stride = int64_t(tot);
    constexpr int kU = 8;
    for (int b0 = seg; b0 < nblk; b0 += kSeg * kU) {
      double v[kU];
#pragma unroll
      for (int q = 0; q < kU; ++q) {
        const int b = b0 + kSeg * q;
        v[q] = b < nblk ? part[b * stride + e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kU; ++q)
        if (b0 + kSeg * q < nblk) s += v[q];
    }
  }
  red[seg][el] = s;
  __syncthreads();
  double g = 0.0;
  if (threadIdx.x < kOut * (kSeg / 4)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) g += red[4 * seg + q][el];
  }
  __syncthreads();
  if (threadIdx.x < kOut * (kSeg / 4)) red[seg][el] = g;
  __syncthreads();
  if (threadIdx.x < kOut && e < tot) {
    double t = 0.0;
    for (int q = 0; q < kSeg / 4; ++q) t += red[q][el];
    const int tile = e / 256, rr = (e / 16) & 15, cc = e & 15;
    const int ti = tl.ti[tile], tj = tl.tj[tile];
    const int ny = 2 * m;
    const int yj = 16 * tj + cc;
    const int b = tj < TU ? yj : yj - 16 * TU;   // column of U
    const int off = tj < TU ? 0 : m;             // A U or M U
    if (b >= m) return;
    if (ti < TW) {
      const int zi = 16 * ti + rr;
      if (zi < w1) G[zi * ny + off + b] = t;
    } else {
      const int ua = 16 * (ti - TW) + rr;
      if (ua >= m || ua > b) return;
      G[(w1 + ua) * ny + off + b] = t;
      if (ua != b) G[(w1 + b) * ny + off + ua] = t;
    }
  }
}

// G[i][j] = sum_b part[b][i][j] in a fixed order.  A block covers 16
// consecutive outputs with 64 segments of the partials (segment q takes
// b = q, q + 64, ...; a wavefront reads four 128-byte runs per load); the
// segment sums are then added in groups of four (q = 4g .. 4g + 3) and the 16
// group sums in order.
__global__ void __launch_bounds__(1024) k_gram_reduce(const double* __restrict__ part, int nblk,
                                                      int nzp, int nyp, int nz, int ny,
                                                      double* __restrict__ G) {
  constexpr int kOut = 16, kSeg = 64;
  __shared__ double red[kSeg][kOut];
  const int el = threadIdx.x & (kOut - 1), seg = threadIdx.x / kOut;
  const int e = blockIdx.x * kOut + el;
  const int tot = nz * ny;
  double s = 0.0;
  if (e < tot) {
    const int i = e / ny, j = e - (e / ny) * ny;
    const int64_t off = int64_t(i) * nyp + j;
    const int64_t stride = int64_t(nzp) * nyp;
    // eight loads in flight, added in the order b = seg, seg + 64, ...
    constexpr int kU = 8;
    for (int b0 = seg; b0 < nblk; b0 += kSeg * kU) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int b = b0 + kSeg * u;
        v[u] = b < nblk ? part[b * stride + off] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (b0 + kSeg * u < nblk) s += v[u];
    }
  }
  red[seg][el] = s;
  __syncthreads();
  double g = 0.0;
  if (threadIdx.x < kOut * (kSeg / 4)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) g += red[4 * seg + q][el];
  }
  __syncthreads();
  if (threadIdx.x < kOut * (kSeg / 4)) red[seg][el] = g;
  __syncthreads();
  if (threadIdx.x < kOut && e < tot) {
    double t = 0.0;
    for (int q = 0; q < kSeg / 4; ++q) t += red[q][el];
    G[e] = t;
  }
}

// U[r][c] = sum_i Z[r][i] Y[i][c], Z = [z1 | z2] (nz <= 96 columns), on the
// FP64 matrix cores.  Y (zero-padded to KS*4 rows, KS even, and TJ*16 columns)
// is staged in LDS once per block; each wavefront owns 16-row tiles of Z.  For
// one tile a lane loads its A fragments for every k step into registers (row
// l % 16; steps 2 s' and 2 s' + 1 take columns 8 s' + 2 (l / 16) and the next
// one, read together), the wavefront runs KS x TJ MFMAs with B fragments read
// from LDS in the same row order, and then writes the tile's 16 x m outputs;
// the next tile's fragments are loaded meanwhile.  A tile is read completely
// before any of its outputs is written and no other wavefront touches its rows,
// so U may alias z2 (the update is done in place).  The fragment registers
// hold KM k steps, a template parameter: 12 when nz <= 48, else 24, so a
// narrow block keeps fewer registers and more wavefronts per SIMD.
constexpr int kUpdKMax = 24;  // k steps of 4: nz <= 96

template <int TJ, int KM>
__global__ void __launch_bounds__(256) k_update_zy(int64_t n, const double* z1, int w1,
                                                   const double* z2, int w2, int ldz2,
                                                   const double* __restrict__ Y, int m, int ks,
                                                   double* U, int ldu, int64_t y_stride) {
  // a batch of equal-width requests: blockIdx.y picks the request (its
  // columns m further along each row, its Y after the previous one's)
  z2 += int64_t(blockIdx.y) * w2;
  U += int64_t(blockIdx.y) * m;
  Y += int64_t(blockIdx.y) * y_stride;
  extern __shared__ double ys[];  // [ks * 4][TJ * 16]
  constexpr int MP = TJ * 16;
  const int nz = w1 + w2;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t tiles = (n + 15) / 16;
  const int64_t wstride = int64_t(gridDim.x) * (blockDim.x >> 6);
  // this lane's A fragments of a tile: row l % 16 of the tile; k steps 2 s'
  // and 2 s' + 1 take columns 8 s' + 2 j and 8 s' + 2 j + 1 of Z (j = l / 16),
  // so a lane reads two adjacent columns with one 16-byte load (with w1 even;
  // the B rows follow the same order)
  auto load_a = [&](int64_t tile, double* a) {
    const int64_t r = tile * 16 + li;
    const bool live = tile < tiles && r < n;
    const double* p1 = z1 + (live ? r : 0) * w1;
    const double* p2 = z2 + (live ? r : 0) * ldz2 - w1;
    if ((w1 & 1) == 0) {
#pragma unroll
      for (int s2 = 0; s2 < KM / 2; ++s2) {
        const int c = 8 * s2 + 2 * lk;
        double2 v{0.0, 0.0};
        if (live && c < nz)
          v = c < w1 ? *reinterpret_cast<const double2*>(p1 + c) : *reinterpret_cast<const double2*>(p2 + c);
        a[2 * s2] = v.x;
        a[2 * s2 + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int s = 0; s < KM; ++s) {
        const int c = 8 * (s >> 1) + 2 * lk + (s & 1);
        a[s] = (live && c < w1) ? p1[c] : ((live && c >= w1 && c < nz) ? p2[c] : 0.0);
      }
    }
  };
  int64_t tile = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  double a[KM], an[KM];
  load_a(tile, a);  // in flight while Y is staged
#pragma unroll 8
  for (int e = threadIdx.x; e < ks * 4 * MP; e += blockDim.x) {
    const int i = e / MP, c = e - (e / MP) * MP;
    ys[e] = (i < nz && c < m) ? Y[i * m + c] : 0.0;
  }
  __syncthreads();
  for (; tile < tiles; tile += wstride) {
    // the next tile's fragments are loaded while this tile's MFMAs run (its
    // rows are not written by this tile: tiles are disjoint)
    load_a(tile + wstride, an);
    d4 acc[TJ];
#pragma unroll
    for (int t = 0; t < TJ; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KM; ++s) {
      if (s < ks) {
        const double* yrow = ys + (8 * (s >> 1) + 2 * lk + (s & 1)) * MP + li;
#pragma unroll
        for (int t = 0; t < TJ; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], yrow[16 * t], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < TJ; ++t) {
      const int c = 16 * t + li;
      if (c >= m) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = tile * 16 + lk + 4 * v;
        if (row < n) U[row * ldu + c] = acc[t][v];
      }
    }
#pragma unroll
    for (int s = 0; s < KM; ++s) a[s] = an[s];
  }
}

template <int TI, int TJW>
void gram_dispatch_launch(const GramPlan& p, int64_t n, int64_t rpb, const double* z1, int w1,
                          const double* z2, int w2, const double* y1, int v1, const double* y2,
                          int v2, double* part, hipStream_t s) {
  {
    const LaunchEvents ev = g_launch_events;
    g_launch_events = LaunchEvents{ev.start, nullptr};
    BMG_LAUNCH((k_gram<TI, TJW>), p.nblk, 256, 0, s, n, rpb, p.nzp, p.nyp, z1, w1, z2, w2, y1, v1, y2, v2, part);
    g_launch_events = LaunchEvents{nullptr, ev.stop};
  }
}

}  // namespace

GramPlan gram_plan(int64_t n, int nz, int ny) {
  GramPlan p;
  p.nz = nz;
  p.ny = ny;
  p.nzp = (nz + 15) / 16 * 16;
  p.nyp = (ny + 15) / 16 * 16;
  // at least 64 rows per block, at most 1024 blocks, and partial sums of at
  // most half the bytes the kernel reads (more blocks hide more of the
  // gathers' latency; the partials cost a second pass)
  int64_t blocks = (n + 63) / 64;
  const int64_t cap = int64_t(0.5 * double(n) * (nz + ny) / (double(p.nzp) * p.nyp));
  blocks = std::min<int64_t>(blocks, std::max<int64_t>(cap, 1));
  p.nblk = int(std::max<int64_t>(1, std::min<int64_t>(blocks, 1024)));
  // partial sums per block: the dense tile layout, or the symmetric one of
  // the fused kernel when nz = w1 + m and ny = 2 m
  p.per_block = int64_t(p.nzp) * p.nyp;
  if (ny % 2 == 0 && nz >= ny / 2) p.per_block = std::max(p.per_block, sym_tile_doubles(nz - ny / 2, ny / 2));
  return p;
}

int launch_gram(const GramPlan& p, int64_t n, const double* z1, int w1, const double* z2, int w2,
                const double* y1, int v1, const double* y2, int v2, double* part, double* G,
                hipStream_t s) {
  const int TI = p.nzp / 16;
  const int TJ = p.nyp / 16;
  const int TJW = (TJ + 3) / 4;
  if (TI < 1 || TI > 6 || TJW < 1 || TJW > 3) {
    set_error("gram: unsupported shape nz=%d ny=%d", p.nz, p.ny);
    return BMG_EINVAL;
  }
  int64_t rpb = (n + p.nblk - 1) / p.nblk;
  rpb = (rpb + 15) / 16 * 16;
#define GL(a, b) \
  gram_dispatch_launch<a, b>(p, n, rpb, z1, w1, z2, w2, y1, v1, y2, v2, part, s)
  switch (TI * 4 + TJW) {
    case 1 * 4 + 1: GL(1, 1); break;
    case 1 * 4 + 2: GL(1, 2); break;
    case 1 * 4 + 3: GL(1, 3); break;
    case 2 * 4 + 1: GL(2, 1); break;
    case 2 * 4 + 2: GL(2, 2); break;
    case 2 * 4 + 3: GL(2, 3); break;
    case 3 * 4 + 1: GL(3, 1); break;
    case 3 * 4 + 2: GL(3, 2); break;
    case 3 * 4 + 3: GL(3, 3); break;
    case 4 * 4 + 1: GL(4, 1); break;
    case 4 * 4 + 2: GL(4, 2); break;
    case 4 * 4 + 3: GL(4, 3); break;
    case 5 * 4 + 1: GL(5, 1); break;
    case 5 * 4 + 2: GL(5, 2); break;
    case 5 * 4 + 3: GL(5, 3); break;
    case 6 * 4 + 1: GL(6, 1); break;
    case 6 * 4 + 2: GL(6, 2); break;
    case 6 * 4 + 3: GL(6, 3); break;
  }
#undef GL
  int st = check_launch();
  if (st != BMG_OK) return st;
  const int tot = p.nz * p.ny;
  BMG_LAUNCH((k_gram_reduce), (tot + 15) / 16, 1024, 0, s, part, p.nblk, p.nzp, p.nyp, p.nz, p.ny, G);
  return check_launch();
}

namespace {

// Tiles of the symmetric fused Gram: W rows against every Y tile, then the
// upper tiles (ti <= tj) of U^T A U and of U^T M U.
SymTiles sym_tiles(int w1, int m) {
  SymTiles tl{};
  const int TW = (w1 + 15) / 16, TU = (m + 15) / 16;
  int T = 0;
  for (int ti = 0; ti < TW; ++ti)
    for (int tj = 0; tj < 2 * TU; ++tj) {
      tl.ti[T] = (unsigned char)ti;
      tl.tj[T] = (unsigned char)tj;
      ++T;
    }
  for (int half = 0; half < 2; ++half)
    for (int i = 0; i < TU; ++i)
      for (int j = i; j < TU; ++j) {
        tl.ti[T] = (unsigned char)(TW + i);
        tl.tj[T] = (unsigned char)(half * TU + j);
        ++T;
      }
  tl.T = T;
  return tl;
}

template <int TPW, int NB, int WT>
void sym_attr() {
  (void)hipFuncSetAttribute((const void*)k_gram_sym<TPW, NB, WT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int TPW>
void sym_attr_all() {
  sym_attr<TPW, 1, 7>();
  sym_attr<TPW, 1, 0>();
  sym_attr<TPW, 2, 7>();
  sym_attr<TPW, 2, 0>();
  sym_attr<TPW, 3, 7>();
  sym_attr<TPW, 3, 0>();
}

template <int TPW>
void sym_launch(const GramPlan& p, const DevLevel& L, const SymTiles& tl, int TW, int TU, const double* w,
                int w1, const double* u, int m, int ldu, int64_t rpb, size_t shm, double* part, hipStream_t s,
                const int* uperm, int nreq, int64_t part_stride) {
  const int64_t n = L.n;
  static const int nbenv = std::getenv("BMG_GRAM_NB") ? std::atoi(std::getenv("BMG_GRAM_NB")) : 0;
  const int nb = nbenv ? nbenv : (kGramAmChunk * (m / 2) > 256 ? 2 : 1);
#define GS(nb_, wt_)                                                                                   \
  BMG_LAUNCH((k_gram_sym<TPW, nb_, wt_>), dim3(p.nblk, nreq), 256, shm, s, n, rpb, tl, TW, TU, L.cols,  \
             L.a64, L.m64, L.W, w, w1, u, m, ldu, part, L.chunk_order, uperm, part_stride)
  if (L.W == 7) {
    if (nb == 3) GS(3, 7);
    else if (nb == 2) GS(2, 7);
    else GS(1, 7);
  } else {
    if (nb == 3) GS(3, 0);
    else if (nb == 2) GS(2, 0);
    else GS(1, 0);
  }
#undef GS
}

template <int TPW>
void sym1_attr() {
  (void)hipFuncSetAttribute((const void*)k_gram_sym1<TPW, 7>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_gram_sym1<TPW, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

template <int TPW>
void sym1_launch(const GramPlan& p, const DevLevel& L, const SymTiles& tl, int TW, int TU, const double* w,
                 int w1, const double* u, int m, int ldu, int64_t rpb, int nthr, size_t shm, double* part,
                 hipStream_t s, const int* uperm, int nreq, int64_t part_stride) {
  if (L.W == 7)
    BMG_LAUNCH((k_gram_sym1<TPW, 7>), dim3(p.nblk, nreq), nthr, shm, s, L.n, rpb, tl, TW, TU, L.cols, L.a64,
               L.m64, L.W, w, w1, u, m, ldu, part, L.chunk_order, uperm, part_stride);
  else
    BMG_LAUNCH((k_gram_sym1<TPW, 0>), dim3(p.nblk, nreq), nthr, shm, s, L.n, rpb, tl, TW, TU, L.cols, L.a64,
               L.m64, L.W, w, w1, u, m, ldu, part, L.chunk_order, uperm, part_stride);
}

}  // namespace

int64_t sym_tile_doubles(int w1, int m) { return int64_t(sym_tiles(w1, m).T) * 256; }

int launch_gram_am(const GramPlan& p, const DevLevel& L, const double* w, int w1, const double* u,
                   int m, double* part, double* G, hipStream_t s, const int* uperm, int ldu, int nreq,
                   int64_t part_stride, int64_t g_stride) {
  if (ldu <= 0) ldu = m;
  if (nreq < 1 || nreq > 65535 || (nreq > 1 && (uperm != nullptr || int64_t(nreq) * m > ldu))) {
    set_error("gram_am: batch of %d requests of width %d in rows of %d", nreq, m, ldu);
    return BMG_EINVAL;
  }
  if (ldu < m || (ldu & 1) != 0) {
    set_error("gram_am: row stride %d of u must be even and at least m = %d", ldu, m);
    return BMG_EINVAL;
  }
  {
    const int TW = (w1 + 15) / 16, TU = (m + 15) / 16;
    if (TW > 2 || TU > 6 || p.ny != 2 * m || p.nz != w1 + m || m % 2 != 0 || m < 2) {
      set_error("gram_am: unsupported shape w1=%d m=%d", w1, m);
      return BMG_EINVAL;
    }
    const SymTiles tl = sym_tiles(w1, m);
    if (int64_t(tl.T) * 256 > p.per_block) {
      set_error("gram_am: partial buffer of %lld doubles per block is too small", (long long)p.per_block);
      return BMG_EINVAL;
    }
    static std::once_flag once;
    std::call_once(once, [] {
      sym_attr_all<1>();
      sym_attr_all<2>();
      sym_attr_all<3>();
      sym_attr_all<4>();
      sym_attr_all<6>();
      sym_attr_all<8>();
      sym_attr_all<10>();
      sym_attr_all<12>();
      sym_attr_all<17>();
    });
    const int64_t n = L.n;
    // a block of 512 or more threads (16 rows x m/2 column pairs) fills a CU
    // by its registers, so 256 of them make one round (measured on the sphere
    // refined 8 times, m = 80: 545 against 555 us with 512); narrower blocks
    // share a CU, and 512 of them are used
    const bool wide = (kGramAmChunk * (m / 2) + 63) / 64 * 64 >= 512;
    static const int cap_env = std::getenv("BMG_GRAM_BLOCKS") ? std::atoi(std::getenv("BMG_GRAM_BLOCKS")) : 0;
    const int cap = cap_env > 0 ? cap_env : (wide ? 256 : 512);
    GramPlan q = p;
    q.nblk = std::max(1, std::min(p.nblk, cap));
    int64_t rpb = (n + q.nblk - 1) / q.nblk;
    rpb = (rpb + kGramAmChunk - 1) / kGramAmChunk * kGramAmChunk;
    q.nblk = int((n + rpb - 1) / rpb);
    const size_t shm = size_t(2) * kGramAmChunk * (sym_zp(TW, TU) + sym_yp(TU)) * sizeof(double);
    // one item per thread when the block (16 rows x m/2 column pairs, whole
    // wavefronts) can stage a chunk's ELL rows
    const int nthr = (kGramAmChunk * (m / 2) + 63) / 64 * 64;
    const int tpw1 = (tl.T + nthr / 64 - 1) / (nthr / 64);
    if (kGramAmChunk * L.W <= nthr && nthr <= 1024 && tpw1 <= 8) {
      static std::once_flag once1;
      std::call_once(once1, [] {
        sym1_attr<1>();
        sym1_attr<2>();
        sym1_attr<3>();
        sym1_attr<4>();
        sym1_attr<5>();
        sym1_attr<6>();
        sym1_attr<8>();
      });
      const size_t shm1 = shm + size_t(2) * kGramAmChunk * L.W * (2 * sizeof(double) + sizeof(int));
      const LaunchEvents ev = g_launch_events;
      g_launch_events = LaunchEvents{ev.start, nullptr};
#define G1(t_) sym1_launch<t_>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, nthr, shm1, part, s, uperm, nreq, part_stride)
      if (tpw1 <= 1) G1(1);
      else if (tpw1 <= 2) G1(2);
      else if (tpw1 <= 3) G1(3);
      else if (tpw1 <= 4) G1(4);
      else if (tpw1 <= 5) G1(5);
      else if (tpw1 <= 6) G1(6);
      else G1(8);
#undef G1
      g_launch_events = LaunchEvents{nullptr, ev.stop};
      int st = check_launch();
      if (st != BMG_OK) return st;
      BMG_LAUNCH((k_gram_sym_reduce), dim3((tl.T * 256 + 15) / 16, nreq), 1024, 0, s, part, q.nblk, tl, TW,
               TU, w1, m, G, part_stride, g_stride);
      return check_launch();
    }
    const int tpw = (tl.T + 3) / 4;
    {
      const LaunchEvents ev = g_launch_events;
      g_launch_events = LaunchEvents{ev.start, nullptr};
      if (tpw <= 1) sym_launch<1>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 2) sym_launch<2>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 3) sym_launch<3>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 4) sym_launch<4>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 6) sym_launch<6>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 8) sym_launch<8>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 10) sym_launch<10>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else if (tpw <= 12) sym_launch<12>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      else sym_launch<17>(q, L, tl, TW, TU, w, w1, u, m, ldu, rpb, shm, part, s, uperm, nreq, part_stride);
      g_launch_events = LaunchEvents{nullptr, ev.stop};
    }
    int st = check_launch();
    if (st != BMG_OK) return st;
    BMG_LAUNCH((k_gram_sym_reduce), dim3((tl.T * 256 + 15) / 16, nreq), 1024, 0, s, part, q.nblk, tl, TW,
               TU, w1, m, G, part_stride, g_stride);
    return check_launch();
  }
}

// ------------------------------------------- allocation-free fused Gram --
// bmg_gram_am_noalloc keeps the Gram kernel's partial sums in this array
// instead of a buffer from hipMalloc.  Each device holds its own copy until
// the process ends; its address on the current device comes from
// hipGetSymbolAddress (the name itself is a host-side stand-in, not a device
// address) and is kept per device.  Every partial sum is written before it is
// read, so nothing needs clearing between calls; calls that overlap on one
// device share the array and race.
constexpr size_t kNoallocScratchDoubles = size_t(2) << 20;  // 16 MiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // by device ordinal

int noalloc_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (int(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                hipGetErrorString(e));
      return BMG_EDEVICE;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return BMG_OK;
}
}  // namespace

int launch_update_zy(int64_t n, const double* z1, int w1, const double* z2, int w2,
                     const double* Y, double* U, int m, hipStream_t s, int ldz2, int ldu, int nreq) {
  const int nz = w1 + w2;
  if (ldz2 <= 0) ldz2 = w2;
  if (ldu <= 0) ldu = m;
  if (nreq < 1 || nreq > 65535 || (nreq > 1 && (int64_t(nreq) * w2 > ldz2 || int64_t(nreq) * m > ldu))) {
    set_error("update: batch of %d requests too wide for rows of %d / %d", nreq, ldz2, ldu);
    return BMG_EINVAL;
  }
  const int64_t y_stride = int64_t(nz) * m;
  if (ldz2 < w2 || ldu < m || (ldz2 & 1) != 0) {
    set_error("update: row strides %d, %d too small for w2 = %d, m = %d (or odd)", ldz2, ldu, w2, m);
    return BMG_EINVAL;
  }
  const int ks = (nz + 7) / 8 * 2;  // k steps of 4, in pairs (see the kernel's A fragments)
  const int TJ = (m + 15) / 16;
  if (ks < 1 || ks > kUpdKMax || TJ < 1 || TJ > 6 || m % 4 != 0) {
    set_error("update: unsupported shape nz=%d m=%d", nz, m);
    return BMG_EINVAL;
  }
  const size_t shm = size_t(ks) * 4 * TJ * 16 * sizeof(double);
  const int64_t tiles = (n + 15) / 16;
  // up to 1024 blocks (each stages Y in LDS once)
  const int grid = int(std::min<int64_t>((tiles + 3) / 4, 1024));
  static std::once_flag once;  // solves on several threads may arrive together
  std::call_once(once, [] {
    (void)hipFuncSetAttribute((const void*)k_update_zy<5, 24>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              96 * 1024);
    (void)hipFuncSetAttribute((const void*)k_update_zy<6, 24>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              96 * 1024);
  });
  // fragment registers for 12 k steps when they suffice (nz <= 48), else 24
#define UL(tj)                                                                                    \
  do {                                                                                            \
    if (ks <= 12)                                                                                 \
      BMG_LAUNCH((k_update_zy<tj, 12>), dim3(grid, nreq), 256, shm, s, n, z1, w1, z2, w2, ldz2, Y, m, ks, U, \
                 ldu, y_stride);                                                                         \
    else                                                                                                 \
      BMG_LAUNCH((k_update_zy<tj, 24>), dim3(grid, nreq), 256, shm, s, n, z1, w1, z2, w2, ldz2, Y, m, ks, U, \
                 ldu, y_stride);                                                                         \
  } while (0)
  switch (TJ) {
    case 1: UL(1); break;
    case 2: UL(2); break;
    case 3: UL(3); break;
    case 4: UL(4); break;
    case 5: UL(5); break;
    default: UL(6); break;
  }
#undef UL
  return check_launch();
}

}  // namespace bmg

extern "C" int bmg_gram_am_noalloc(const bmg_hierarchy* h, int32_t level, const double* w, int32_t m2,
                                   const double* u, int32_t m, double* G, void* stream) {
  using namespace bmg;
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy with device data required");
  BMG_CHECK(level >= 0 && level < int(h->dev.size()), "level %d out of range", level);
  BMG_CHECK(u != nullptr && G != nullptr, "u and G must be non-NULL");
  BMG_CHECK(m >= 2 && m % 2 == 0 && m2 >= 0 && m2 + m <= 96 && (m2 == 0 || w != nullptr),
            "gram_am_noalloc needs even m >= 2, 0 <= m2, m2 + m <= 96, and w when m2 > 0");
  BMG_HIP(hipSetDevice(h->device));
  double* part = nullptr;
  BMG_TRY(noalloc_scratch(h->device, &part));
  const DevLevel& D = h->dev[level];
  GramPlan p = gram_plan(D.n, m2 + m, 2 * m);
  // as many row blocks as the planner asks for, while their partial sums fit
  const size_t per_block = size_t(p.per_block);
  if (per_block > kNoallocScratchDoubles) {
    set_error("gram_am_noalloc: one block's partial sums (%zu doubles) exceed the %zu-double scratch",
              per_block, kNoallocScratchDoubles);
    return BMG_EINVAL;
  }
  p.nblk = int(std::min<size_t>(size_t(p.nblk), kNoallocScratchDoubles / per_block));
  // the blocks come in vertex order; a permuted level reads them through perm
  return launch_gram_am(p, D, w, m2, u, m, part, G, static_cast<hipStream_t>(stream), D.perm);
}
