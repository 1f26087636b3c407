// Dense coupling product on the matrix cores: C = W f(P) for a dense symmetric coupling
// matrix W (n x n, row-major) and the replica state P (n x stride), with f(p) = 2p - 1
// (max-cut) or f(p) = p (MIS).  FP32 inputs, FP32 accumulation (v_mfma_f32_32x32x2_f32).
//
// Each wavefront owns a 32 x 32 tile of C and walks the whole k range two at a time; a
// workgroup of four wavefronts covers 64 rows x 64 replica columns.  Because W is
// symmetric, the A operand W[i][k] is read as W[k][i]: for fixed k the 32 rows of a tile
// are 32 consecutive floats, so both operand fragments are coalesced row reads.  The
// k order is fixed, so the product is deterministic.
#include "qqa_internal.h"

namespace qqa {

typedef float floatx16 __attribute__((ext_vector_type(16)));

template <bool MAXCUT>
__global__ __launch_bounds__(256) void dense_coupling_kernel(const float* __restrict__ W, const float* __restrict__ P,
                                                             float* __restrict__ C, int n, int stride) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = blockIdx.x * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.y * 64 + (wave & 1) * 32;
  const int li = lane & 31, lk = lane >> 5;
  const int arow = row0 + li;  // A fragment: A[arow][k + lk] = W[k + lk][arow]
  const int bcol = col0 + li;  // B fragment: B[k + lk][bcol] = f(P[k + lk][bcol])
  const bool aok = arow < n, bok = bcol < stride;
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int kfull = n & ~1;
  for (int k = 0; k < kfull; k += 2) {
    const int kk = k + lk;
    const float a = aok ? W[(size_t)kk * n + arow] : 0.f;
    float b = bok ? P[(size_t)kk * stride + bcol] : 0.f;
    if (MAXCUT) b = bok ? 2.f * b - 1.f : 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
  if (kfull < n) {  // odd n: the last k pairs with a zero row
    const int kk = kfull + lk;
    const bool kok = kk < n;
    const float a = (aok && kok) ? W[(size_t)kk * n + arow] : 0.f;
    float b = (bok && kok) ? P[(size_t)kk * stride + bcol] : 0.f;
    if (MAXCUT) b = (bok && kok) ? 2.f * b - 1.f : 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
  // accumulator r of lane l holds C[row0 + 8 (r / 4) + 4 (l / 32) + r % 4][col0 + l % 32]
  const int col = col0 + li;
  if (col >= stride) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + 8 * (r >> 2) + 4 * lk + (r & 3);
    if (row < n) C[(size_t)row * stride + col] = acc[r];
  }
}

hipError_t launch_dense_coupling(const float* W, const float* P, float* C, int n, int stride, int problem,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid((n + 63) / 64, (stride + 63) / 64), block(256);
  if (problem == kMAXCUT)
    hipLaunchKernelGGL(dense_coupling_kernel<true>, grid, block, 0, st, W, P, C, n, stride);
  else
    hipLaunchKernelGGL(dense_coupling_kernel<false>, grid, block, 0, st, W, P, C, n, stride);
  return hipGetLastError();
}

}  // namespace qqa
