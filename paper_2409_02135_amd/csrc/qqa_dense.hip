// Dense coupling product on the matrix cores: C = W f(P) for a dense symmetric coupling
// matrix W (n x n, row-major) and the replica state P (n x stride), with f(p) = 2p - 1
// (max-cut) or f(p) = p (MIS).  FP32 inputs, FP32 accumulation (v_mfma_f32_32x32x2_f32).
//
// A workgroup owns a 128 x 128 tile of C (128 variables x 128 replica columns) and one of
// `splits` contiguous parts of the k range; 16 wavefronts in a 4 x 4 grid each own a 32 x 32
// block of the tile.  The k range is walked in chunks of kBK rows whose W and P tiles are
// staged through LDS (double-buffered); the next chunk is fetched into registers while the
// matrix cores work on the current one.  A chunk moves 64 KB for 2 x 128 x 128 x kBK flops
// (32 flops per byte); a 64 x 64 tile would move half as many flops per byte, more than the
// L2-to-CU bandwidth can feed at the matrix cores' rate.  The k split (split-K) gives every
// CU a workgroup: part s writes its partial product to its own array and dense_reduce_kernel
// adds the parts in part order, so the product is deterministic.
//
// Because W is symmetric, the A operand W[i][k] is read as W[k][i]: for fixed k the 128
// rows of a tile are 128 consecutive floats, so both operand tiles are coalesced row reads.
// Workgroups are numbered so that the column tiles sharing one band of W rows land on the
// same XCD (dispatch assigns consecutive workgroup ids to XCDs round-robin): the band is
// then fetched into that XCD's L2 once and re-read there.
#include <algorithm>

#include "qqa_internal.h"

namespace qqa {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kXcds = 8;
constexpr int kTile = 128;          // rows and columns of C per workgroup
constexpr int kBK = 64;             // k rows per chunk
constexpr int kDenseThreads = 1024; // 16 wavefronts, one 32 x 32 block each

template <bool MAXCUT, bool AVEC>
__global__ __launch_bounds__(kDenseThreads) void dense_tile128_kernel(const float* __restrict__ W,
                                                                       const float* __restrict__ P,
                                                                       float* __restrict__ Cp, int n, int stride,
                                                                       int tiles_m, int tiles_n, int splits,
                                                                       int chunks_per_split) {
  extern __shared__ float4 smem4[];
  float* smem = reinterpret_cast<float*>(smem4);
  constexpr int NT = kDenseThreads;
  constexpr int kStage = 2 * kBK * kTile;  // floats per buffer: A chunk then B chunk
  constexpr int kV = kBK * kTile / 4 / NT;  // float4 of each operand per thread and chunk
  static_assert(kV >= 1 && kBK * kTile / 4 == kV * NT, "whole float4 per thread and chunk");

  // XCD-aware order: logical tiles [x * nb / 8, (x + 1) * nb / 8) run on XCD x; the column
  // tiles of one (part, row band) are consecutive, so they share their W band in one L2
  const int nb = gridDim.x;
  int t = blockIdx.x;
  if (nb % kXcds == 0) t = (blockIdx.x % kXcds) * (nb / kXcds) + blockIdx.x / kXcds;
  const int ct = t % tiles_n, rt = (t / tiles_n) % tiles_m, part = t / (tiles_n * tiles_m);
  const int row0 = rt * kTile, col0 = ct * kTile;
  const int total_chunks = (n + kBK - 1) / kBK;
  const int c_begin = part * chunks_per_split, c_end = min(total_chunks, c_begin + chunks_per_split);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 2) * 32, wc = (wave & 3) * 32;
  const int li = lane & 31, lk = lane >> 5;
  // float4 v of this thread's share of a chunk: chunk row fr(v), columns fc .. fc + 3
  const int fc = (tid & 31) * 4;
  auto fr = [&](int v) { return (tid >> 5) + v * (NT / 32); };

  float4 ra[kV], rb[kV];
  float rs[kV][4];
  // raw loads only: any arithmetic on them here would wait for each load in turn
  auto fetch = [&](int k0) {
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const int k = k0 + fr(v);
      if constexpr (AVEC) {
        const int r = row0 + fc;
        ra[v] = (k < n && r < n) ? *reinterpret_cast<const float4*>(W + (size_t)k * n + r) : make_float4(0, 0, 0, 0);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          rs[v][c] = (k < n && row0 + fc + c < n) ? W[(size_t)k * n + row0 + fc + c] : 0.f;
      }
      const int col = col0 + fc;
      rb[v] = (k < n && col < stride) ? *reinterpret_cast<const float4*>(P + (size_t)k * stride + col)
                                      : make_float4(0, 0, 0, 0);
    }
  };
  // f(P) is applied when the chunk is written to LDS, after the matrix-core loop
  auto stash = [&](int buf, int k0) {
    float* As = smem + buf * kStage;
    float* Bs = As + kBK * kTile;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      if constexpr (AVEC) {
        *reinterpret_cast<float4*>(As + fr(v) * kTile + fc) = ra[v];
      } else {
        *reinterpret_cast<float4*>(As + fr(v) * kTile + fc) = make_float4(rs[v][0], rs[v][1], rs[v][2], rs[v][3]);
      }
      float4 b = rb[v];
      if (MAXCUT) {
        const bool ok = k0 + fr(v) < n && col0 + fc < stride;
        b = ok ? make_float4(2.f * b.x - 1.f, 2.f * b.y - 1.f, 2.f * b.z - 1.f, 2.f * b.w - 1.f)
               : make_float4(0, 0, 0, 0);
      }
      *reinterpret_cast<float4*>(Bs + fr(v) * kTile + fc) = b;
    }
  };

  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;

  if (c_begin < c_end) {
    fetch(c_begin * kBK);
    stash(0, c_begin * kBK);
    __syncthreads();
  }
  for (int s = c_begin; s < c_end; ++s) {
    const int buf = (s - c_begin) & 1;
    if (s + 1 < c_end) fetch((s + 1) * kBK);
    const float* As = smem + buf * kStage;
    const float* Bs = As + kBK * kTile;
    // the next chunk goes to the other buffer halfway through this one's matrix-core work:
    // that buffer's last readers passed the barrier that ended the previous chunk, and by
    // then its global loads have returned (measured: 78.0 against 79.4 us when written after
    // the loop, n = 4,096, S = 256)
#pragma unroll
    for (int jj = 0; jj < kBK / 2; ++jj) {
      if (jj == kBK / 4 && s + 1 < c_end) stash(buf ^ 1, (s + 1) * kBK);
      const int j = 2 * jj + lk;
      const float a = As[j * kTile + wr + li];  // A[wr + li][k0 + j] = W[k0 + j][row0 + wr + li]
      const float b = Bs[j * kTile + wc + li];  // B[k0 + j][wc + li]
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  // accumulator r of lane l holds C[wr + 8 (r / 4) + 4 (l / 32) + r % 4][wc + l % 32]
  float* C = Cp + (size_t)part * n * stride;
  const int col = col0 + wc + li;
  if (col >= stride) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + wr + 8 * (r >> 2) + 4 * lk + (r & 3);
    if (row < n) C[(size_t)row * stride + col] = acc[r];
  }
}

// C = sum of the `parts` partial products, added in part order
__global__ __launch_bounds__(kBlock) void dense_reduce_kernel(const float* __restrict__ Cp, int parts, size_t count4,
                                                              float* __restrict__ C) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count4) return;
  float4 s = reinterpret_cast<const float4*>(Cp)[i];
  for (int q = 1; q < parts; ++q) {
    const float4 x = reinterpret_cast<const float4*>(Cp + (size_t)q * count4 * 4)[i];
    s.x += x.x;
    s.y += x.y;
    s.z += x.z;
    s.w += x.w;
  }
  reinterpret_cast<float4*>(C)[i] = s;
}

int dense_splits(int n, int stride) {
  const int tiles = ((n + kTile - 1) / kTile) * ((stride + kTile - 1) / kTile);
  const int chunks = (n + kBK - 1) / kBK;
  // enough parts that every CU has a workgroup, each part at least 8 chunks long
  int splits = 1;
  while (splits < 8 && tiles * splits * 2 <= 256 && chunks / (splits * 2) >= 8) splits *= 2;
  return splits;
}

size_t dense_workspace_bytes(int n, int stride) {
  const int splits = dense_splits(n, stride);
  return splits > 1 ? (size_t)splits * n * stride * sizeof(float) : 0;
}

hipError_t launch_dense_parts(const float* W, const float* P, float* out, int n, int stride, int problem,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int tiles_m = (n + kTile - 1) / kTile, tiles_n = (stride + kTile - 1) / kTile;
  const int splits = dense_splits(n, stride);
  const int chunks = (n + kBK - 1) / kBK;
  const int per = (chunks + splits - 1) / splits;
  const dim3 grid(tiles_m * tiles_n * splits), block(kDenseThreads);
  const size_t lds = 2 * (size_t)(2 * kBK * kTile) * sizeof(float);
  const bool avec = n % 4 == 0;
#define LAUNCH(MC, AV)                                                                                        \
  hipLaunchKernelGGL((dense_tile128_kernel<MC, AV>), grid, block, lds, st, W, P, out, n, stride, tiles_m, tiles_n, \
                     splits, per)
  if (problem == kMAXCUT) {
    if (avec) LAUNCH(true, true);
    else LAUNCH(true, false);
  } else {
    if (avec) LAUNCH(false, true);
    else LAUNCH(false, false);
  }
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_dense_coupling(const float* W, const float* P, float* C, int n, int stride, int problem,
                                 float* work, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int splits = dense_splits(n, stride);
  if (splits > 1 && !work) return hipErrorInvalidValue;
  hipError_t e = launch_dense_parts(W, P, splits > 1 ? work : C, n, stride, problem, st);
  if (e != hipSuccess || splits == 1) return e;
  const size_t count4 = (size_t)n * stride / 4;
  hipLaunchKernelGGL(dense_reduce_kernel, dim3((unsigned)((count4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, work,
                     splits, count4, C);
  return hipGetLastError();
}

}  // namespace qqa
