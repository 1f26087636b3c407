// Dense coupling product on the matrix cores: C = W f(P) for a dense symmetric coupling
// matrix W (n x n, row-major) and the replica state P (n x stride), with f(p) = 2p - 1
// (max-cut) or f(p) = p (MIS).  FP32 inputs, FP32 accumulation (v_mfma_f32_32x32x2_f32).
//
// A workgroup owns a 64 x 64 tile of C (64 variables x 64 replica columns) and walks the k
// range in chunks of BK.  The chunk's W and P tiles are staged through LDS (double-
// buffered); the next chunk is fetched into registers while the matrix cores work on the
// current one.  Sixteen wavefronts share the tile: wavefront w owns the 32 x 32 quarter
// w % 4 and the k slice w / 4 of every chunk, so each SIMD runs four independent MFMA
// chains; at the end the four k-slice partial sums of a quarter are added in slice order
// through LDS.  The number of output tiles of the main workload (4096 x 256) equals the
// number of CUs, so splitting k inside the workgroup is what keeps every SIMD busy.
//
// Because W is symmetric, the A operand W[i][k] is read as W[k][i]: for fixed k the 64
// rows of a tile are 64 consecutive floats, so both tiles are coalesced row reads.
// Workgroups are numbered so that the column tiles sharing one band of W rows land on the
// same XCD (dispatch assigns consecutive workgroup ids to XCDs round-robin): the band is
// then fetched into that XCD's L2 once and re-read there.  The k order within a slice and
// the order of the slice sums are fixed, so the product is deterministic.
#include <algorithm>

#include "qqa_internal.h"

namespace qqa {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 64;        // rows and columns of C per workgroup
constexpr int kXcds = 8;
constexpr int kSlices = 4;       // k slices per chunk (wavefronts per quarter)
constexpr int kDenseThreads = 64 * 4 * kSlices;
constexpr int kDenseBK = 64;     // k rows per chunk

template <int BK, bool MAXCUT, bool AVEC>
__global__ __launch_bounds__(kDenseThreads) void dense_coupling_kernel(const float* __restrict__ W,
                                                                       const float* __restrict__ P,
                                                                       float* __restrict__ C, int n, int stride,
                                                                       int tiles_n) {
  extern __shared__ float4 smem4[];
  float* smem = reinterpret_cast<float*>(smem4);
  constexpr int NT = kDenseThreads;
  constexpr int kStage = 2 * BK * kTile;     // floats per buffer: A chunk then B chunk
  constexpr int kVec = BK * kTile / 4 / NT;  // float4 per thread per operand chunk
  constexpr int kScal = BK * kTile / NT;     // floats per thread (scalar A path)
  constexpr int kPairs = BK / kSlices / 2;   // k pairs per wavefront per chunk
  static_assert(kVec >= 1 && BK % (2 * kSlices) == 0, "chunk too small for the workgroup");

  // XCD-aware tile order: logical tiles [x * nb / 8, (x + 1) * nb / 8) run on XCD x
  const int nb = gridDim.x;
  int tile = blockIdx.x;
  if (nb % kXcds == 0) tile = (blockIdx.x % kXcds) * (nb / kXcds) + blockIdx.x / kXcds;
  const int row0 = (tile / tiles_n) * kTile, col0 = (tile % tiles_n) * kTile;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int quarter = wave & 3, slice = wave >> 2;
  const int wr = (quarter >> 1) * 32, wc = (quarter & 1) * 32;
  const int li = lane & 31, lk = lane >> 5;

  // register staging of one chunk
  float4 ra[AVEC ? kVec : 1];
  float rs[AVEC ? 1 : kScal];
  float4 rb[kVec];

  // raw loads only: any arithmetic on them here would wait for each load in turn
  auto fetch = [&](int k0) {
    if constexpr (AVEC) {
#pragma unroll
      for (int i = 0; i < kVec; ++i) {
        const int idx = tid + NT * i, kr = idx >> 4, c = (idx & 15) * 4;
        const int k = k0 + kr, r = row0 + c;
        ra[i] = (k < n && r < n) ? *reinterpret_cast<const float4*>(W + (size_t)k * n + r) : make_float4(0, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < kScal; ++i) {
        const int idx = tid + NT * i, kr = idx >> 6, c = idx & 63;
        const int k = k0 + kr, r = row0 + c;
        rs[i] = (k < n && r < n) ? W[(size_t)k * n + r] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < kVec; ++i) {
      const int idx = tid + NT * i, kr = idx >> 4, c = (idx & 15) * 4;
      const int k = k0 + kr, col = col0 + c;
      rb[i] = (k < n && col < stride) ? *reinterpret_cast<const float4*>(P + (size_t)k * stride + col)
                                      : make_float4(0, 0, 0, 0);
    }
  };
  // f(P) is applied when the chunk is written to LDS, after the matrix-core loop
  auto stash = [&](int buf, int k0) {
    float* As = smem + buf * kStage;
    float* Bs = As + BK * kTile;
    if constexpr (AVEC) {
#pragma unroll
      for (int i = 0; i < kVec; ++i) {
        const int idx = tid + NT * i;
        *reinterpret_cast<float4*>(As + (idx >> 4) * kTile + (idx & 15) * 4) = ra[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < kScal; ++i) {
        const int idx = tid + NT * i;
        As[(idx >> 6) * kTile + (idx & 63)] = rs[i];
      }
    }
#pragma unroll
    for (int i = 0; i < kVec; ++i) {
      const int idx = tid + NT * i;
      float4 b = rb[i];
      if (MAXCUT) {
        const bool ok = k0 + (idx >> 4) < n && col0 + (idx & 15) * 4 < stride;
        b = ok ? make_float4(2.f * b.x - 1.f, 2.f * b.y - 1.f, 2.f * b.z - 1.f, 2.f * b.w - 1.f)
               : make_float4(0, 0, 0, 0);
      }
      *reinterpret_cast<float4*>(Bs + (idx >> 4) * kTile + (idx & 15) * 4) = b;
    }
  };

  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;

  const int chunks = (n + BK - 1) / BK;
  if (chunks > 0) {
    fetch(0);
    stash(0, 0);
    __syncthreads();
  }
  for (int s = 0; s < chunks; ++s) {
    if (s + 1 < chunks) fetch((s + 1) * BK);
    const float* As = smem + (s & 1) * kStage;
    const float* Bs = As + BK * kTile;
#pragma unroll
    for (int jj = 0; jj < kPairs; ++jj) {
      const int j = 2 * (slice * kPairs + jj) + lk;
      const float a = As[j * kTile + wr + li];  // A[wr + li][k0 + j]
      const float b = Bs[j * kTile + wc + li];  // B[k0 + j][wc + li]
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    if (s + 1 < chunks) stash((s + 1) & 1, (s + 1) * BK);
    __syncthreads();
  }

  // slices 1..3 hand their partial quarters to slice 0 through LDS (free after the loop)
  float* red = smem;
  if (slice > 0)
#pragma unroll
    for (int r = 0; r < 16; ++r) red[(((slice - 1) * 4 + quarter) * 16 + r) * 64 + lane] = acc[r];
  __syncthreads();
  if (slice > 0) return;
#pragma unroll
  for (int h = 0; h < kSlices - 1; ++h)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += red[((h * 4 + quarter) * 16 + r) * 64 + lane];

  // accumulator r of lane l holds C[wr + 8 (r / 4) + 4 (l / 32) + r % 4][wc + l % 32]
  const int col = col0 + wc + li;
  if (col >= stride) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + wr + 8 * (r >> 2) + 4 * lk + (r & 3);
    if (row < n) C[(size_t)row * stride + col] = acc[r];
  }
}

hipError_t launch_dense_coupling(const float* W, const float* P, float* C, int n, int stride, int problem,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  constexpr int BK = kDenseBK;
  const int tiles_m = (n + kTile - 1) / kTile, tiles_n = (stride + kTile - 1) / kTile;
  const dim3 grid(tiles_m * tiles_n), block(kDenseThreads);
  // two chunk buffers; the end-of-kernel slice reduction reuses them
  const size_t lds = std::max(2 * 2 * (size_t)BK * kTile, (size_t)(kSlices - 1) * 4 * 16 * 64) * sizeof(float);
  const bool avec = n % 4 == 0;
  if (problem == kMAXCUT) {
    if (avec)
      hipLaunchKernelGGL((dense_coupling_kernel<BK, true, true>), grid, block, lds, st, W, P, C, n, stride, tiles_n);
    else
      hipLaunchKernelGGL((dense_coupling_kernel<BK, true, false>), grid, block, lds, st, W, P, C, n, stride, tiles_n);
  } else {
    if (avec)
      hipLaunchKernelGGL((dense_coupling_kernel<BK, false, true>), grid, block, lds, st, W, P, C, n, stride, tiles_n);
    else
      hipLaunchKernelGGL((dense_coupling_kernel<BK, false, false>), grid, block, lds, st, W, P, C, n, stride, tiles_n);
  }
  return hipGetLastError();
}

}  // namespace qqa
