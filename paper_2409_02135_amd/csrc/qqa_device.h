// Device functions shared by every kernel that updates replica rows (single-instance,
// split-row, persistent and multi-instance slot kernels), so that all of them perform the
// same floating-point operations in the same order for a given row.
#pragma once

#include "qqa_internal.h"

namespace qqa {

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the uniform / normal transforms.
// ---------------------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // 32x32 -> 64-bit products: one v_mad_u64_u32 each gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// odd multiples of 2^-24 in (0,1): exact in binary32
__device__ __forceinline__ float u01(uint32_t r) { return (float)((r >> 8) | 1u) * 0x1.0p-24f; }

// Box-Muller on (u0,u1), (u2,u3) with the hardware transcendental units:
// R = sqrt(-2 ln u) = sqrt(-2 ln2 * log2 u) (v_log_f32, v_sqrt_f32); the angle 2 pi u is
// passed to v_sin_f32 / v_cos_f32 in revolutions (their argument is scaled by 2 pi).
__device__ __forceinline__ float4 normals4(U4 r) {
  const float m2ln2 = -1.38629436111989061883f;  // -2 ln 2
  const float R1 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01(r.x)));
  const float R2 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01(r.z)));
  const float a1 = u01(r.y), a2 = u01(r.w);
  return make_float4(R1 * __builtin_amdgcn_cosf(a1), R1 * __builtin_amdgcn_sinf(a1), R2 * __builtin_amdgcn_cosf(a2),
                     R2 * __builtin_amdgcn_sinf(a2));
}

// ---------------------------------------------------------------------------------------
// Fused update of one row (all S replicas of variable `row`), lanes gl = 0..LPR-1.
// ---------------------------------------------------------------------------------------
template <int LPR>
__device__ __forceinline__ float group_sum(float x) {
  // butterfly inside the LPR-lane group: a fixed tree determined by LPR alone, and
  // every lane ends with the same bits (IEEE addition is commutative)
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, LPR);
  return x;
}

__device__ __forceinline__ float comp(const float4& v, int c) {
  return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}
__device__ __forceinline__ void set_comp(float4& v, int c, float x) {
  if (c == 0) v.x = x; else if (c == 1) v.y = x; else if (c == 2) v.z = x; else v.w = x;
}

// z^E for a compile-time E: the multiplications of ipow_odd(z, E), in its order
template <int E>
__device__ __forceinline__ float ipow_fixed(float z) {
  float r = z;
#pragma unroll
  for (int i = 1; i < E; ++i) r *= z;
  return r;
}

__device__ __forceinline__ float ipow_odd(float z, int e) {
  float r = z;
  for (int i = 1; i < e; ++i) r *= z;
  return r;
}

// Device-coherent float4 access for state that other workgroups of a running kernel read:
// two 64-bit agent-scope relaxed atomic accesses, which the compiler emits as L2-bypassing
// (write-through) memory instructions, so no cache write-back or invalidation is needed to
// share the values across the chip.
__device__ __forceinline__ float4 load_coherent(const float* p) {
  const unsigned long long lo =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long hi =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p) + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_float4(__uint_as_float((unsigned)lo), __uint_as_float((unsigned)(lo >> 32)), __uint_as_float((unsigned)hi),
                     __uint_as_float((unsigned)(hi >> 32)));
}
__device__ __forceinline__ void store_coherent(float* p, const float4 v) {
  const unsigned long long lo = (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
  const unsigned long long hi = (unsigned long long)__float_as_uint(v.z) | ((unsigned long long)__float_as_uint(v.w) << 32);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p) + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Neighbour quads loaded per batch of the coupling loop: a batch issues all its loads before
// the first one is used, so a row's gathers cost one memory round trip per batch.
constexpr int kGatherQuads = 8;

// acc += sum over edges e in [e_begin, e_end) of w_e * f(p_col(e)), with f(p) = p (MIS or
// max clique) or 2p - 1 (max-cut), accumulated in edge order.  Each batch takes
// kGatherQuads / QPL edges (at least one): their column indices and weights, then all their
// neighbour loads, then the fused multiply-adds.  The loads are unconditional (an edge past
// the row's end loads the row's last neighbour again, and its product is discarded by a
// select), so no branch separates them and they are all in flight together.
// Normally every lane of the group walks all edges in edge order for its own quads.  Edge
// split: when the row has fewer quads than the group has lanes (nq divides LPR, one quad
// per lane), the LPR / nq lane slices take every (LPR / nq)-th edge for quad gl % nq, and a
// butterfly over the slices adds their partial sums, so every lane ends with its quad's
// sum (identical bits in each slice).  Both orders are fixed by the layout alone.  SPLIT =
// false keeps plain edge order whatever the shape (idle lanes instead).
template <int LPR, int QPL, bool FULL, bool COHERENT = false, bool SPLIT = true, int QUADS = kGatherQuads>
__device__ __forceinline__ void gather_coupling(const StepParams& a, const int e_begin, const int e_end, const int gl,
                                                const int nq, const bool maxcut, float4 (&acc)[QPL]) {
  // the persistent engines (COHERENT) keep one edge per batch: their registers hold state
  constexpr int U = COHERENT ? 1 : (QUADS / QPL > 0 ? QUADS / QPL : 1);
  const int slices = (SPLIT && !FULL && QPL == 1 && nq < LPR && LPR % nq == 0) ? LPR / nq : 1;
  const int lane_q = slices > 1 ? gl % nq : gl;  // the quad this lane gathers
  const int first = e_begin + (slices > 1 ? gl / nq : 0);
  for (int e0 = first; e0 < e_end; e0 += U * slices) {
    const float* pj[U];
    float w[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * slices;
      ok[u] = e < e_end;
      const int ec = ok[u] ? e : e_end - 1;  // a valid edge of this row
      pj[u] = a.P_in + (size_t)a.col[ec] * a.stride;
      w[u] = a.w ? a.w[ec] : 1.f;
    }
    // a lane past the row's last quad loads that quad again (unconditional loads, no join);
    // its sums are never used
    float4 x[U][QPL];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const int q = lane_q + LPR * k;
        const float* src = pj[u] + 4 * ((FULL || q < nq) ? q : nq - 1);
        x[u][k] = COHERENT ? load_coherent(src) : *reinterpret_cast<const float4*>(src);
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float xc = comp(x[u][k], c);
          const float f = maxcut ? 2.f * xc - 1.f : xc;
          const float r = fmaf(w[u], f, comp(acc[k], c));
          set_comp(acc[k], c, ok[u] ? r : comp(acc[k], c));
        }
      }
  }
  if (SPLIT && !FULL && QPL == 1 && slices > 1) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      if (off < nq) break;  // lanes differing in the slice bits only
      acc[0].x += __shfl_xor(acc[0].x, off, LPR);
      acc[0].y += __shfl_xor(acc[0].y, off, LPR);
      acc[0].z += __shfl_xor(acc[0].z, off, LPR);
      acc[0].w += __shfl_xor(acc[0].w, off, LPR);
    }
  }
}

// FULL: S == 4 * LPR * QPL, every lane owns whole, valid quads (no replica masks).

// A row's own replica values (p, and the AdamW moments when used) for lane gl.
template <int LPR, int QPL, bool FULL>
__device__ __forceinline__ void load_row(const StepParams& a, const float* P, const int row, const int gl,
                                         float4 (&p)[QPL], float4 (&mm)[QPL], float4 (&vv)[QPL]) {
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  const size_t base = (size_t)row * a.stride;
  const bool adam = a.rule == kADAMW;
  // Unconditional loads, so that no branch joins them (a join makes the compiler copy the
  // loaded registers, which waits for the loads): a lane past the row's last quad reads
  // that quad again, and its values are masked wherever they are used; without moments the
  // row itself stands in for m and v, whose values are then not used.
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    const size_t off = base + 4 * (size_t)((FULL || q < nq) ? q : nq - 1);
    p[k] = *reinterpret_cast<const float4*>(P + off);
    mm[k] = *reinterpret_cast<const float4*>((adam ? a.m : P) + off);
    vv[k] = *reinterpret_cast<const float4*>((adam ? a.v : P) + off);
  }
}

// Where a row's coupling terms come from: its CSR range and, for a split row, its first
// chunk (-1 otherwise).  Loaded before the row's own state, so that waiting for these few
// words does not also wait for the state loads (vector loads complete in order).
struct RowMeta {
  int e0, e1, hub;
};
__device__ __forceinline__ RowMeta row_meta(const StepParams& a, const int row) {
  RowMeta m{0, 0, -1};
  if (a.hub_first) m.hub = a.hub_first[row];
  m.e0 = a.row_ptr[row];
  m.e1 = a.row_ptr[row + 1];
  return m;
}

// Coupling product of one row: C_i = sum_j A_ij p_j (MIS) or sum_j A_ij (2 p_j - 1)
// (max-cut), accumulated in CSR order (or chunk order for split rows) so that the
// rounding sequence depends on the graph only.  DENSE: read from the precomputed product
// a.coupling instead (a compile-time choice: a runtime branch around that load would join
// the sparse path and make it wait for every load in flight).
template <int LPR, int QPL, bool FULL, bool COHERENT = false, bool SPLIT = true, bool DENSE = false,
          int QUADS = kGatherQuads, int SPEC = 0>
__device__ __forceinline__ void row_coupling(const StepParams& a, const int row, const RowMeta& rm, const int gl,
                                             float4 (&acc)[QPL]) {
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  if (DENSE) {
    const size_t pitch = (size_t)a.n * a.stride;  // between partial products
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      const int q = gl + LPR * k;
      const size_t off = (size_t)row * a.stride + 4 * (size_t)((FULL || q < nq) ? q : nq - 1);
      acc[k] = *reinterpret_cast<const float4*>(a.coupling + off);
      for (int part = 1; part < a.coupling_parts; ++part) {
        const float4 x = *reinterpret_cast<const float4*>(a.coupling + part * pitch + off);
        acc[k].x += x.x;
        acc[k].y += x.y;
        acc[k].z += x.z;
        acc[k].w += x.w;
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (rm.hub >= 0) {
    const int nch = (rm.e1 - rm.e0 + kHubChunk - 1) / kHubChunk;
    for (int c = 0; c < nch; ++c) {
      const float* part = a.hub_partial + (size_t)(rm.hub + c) * a.stride;
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const int q = gl + LPR * k;
        if (FULL || q < nq) {
          const float4 x = *reinterpret_cast<const float4*>(part + 4 * q);
          acc[k].x += x.x;
          acc[k].y += x.y;
          acc[k].z += x.z;
          acc[k].w += x.w;
        }
      }
    }
  } else {
    const bool maxcut = SPEC ? spec_problem(SPEC) == kMAXCUT : a.problem == kMAXCUT;
    gather_coupling<LPR, QPL, FULL, COHERENT, SPLIT, QUADS>(a, rm.e0, rm.e1, gl, nq, maxcut, acc);
  }
}

// Replica statistics of one row (Eq. 10): mu_i and the communication coefficient
// cg_i = -alpha_c / sigma_i (0 when sigma_i = 0), two passes, population STD.  The sums run
// over lane gl's quads, then the group's butterfly: the rounding depends on the layout only.
template <int LPR, int QPL, bool FULL>
__device__ __forceinline__ void row_stats(const StepParams& a, const int gl, const float4 (&p)[QPL], float& mu,
                                          float& cg) {
  float sum = 0.f;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < a.S) sum += comp(p[k], c);
  }
  sum = group_sum<LPR>(sum);
  mu = sum * a.inv_S;
  float sq = 0.f;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < a.S) {
        const float d = comp(p[k], c) - mu;
        sq = fmaf(d, d, sq);
      }
  }
  sq = group_sum<LPR>(sq);
  const float sigma = __builtin_amdgcn_sqrtf(sq * a.inv_S);
  cg = sigma > 0.f ? -a.comm_alpha * __builtin_amdgcn_rcpf(sigma) : 0.f;
}

// Everything after the coupling product and the row statistics: gradient, AdamW or plain
// step, noise, clamp.  Writes the new values of lane gl's replicas to po / mo / vo (padding
// replicas 0).  Quad indices are local to `a` (whose pointers and S may describe a slice of
// the row); q_off is the slice's first quad in the row, for the noise counter.  SUMS: the
// kernel may run max clique (per-replica sums in a.colsum); kernels that never do leave it
// out and keep their registers.  NOISE_IN: the quads' normals come in xi_in (formed
// beforehand with the same generator and counters), not from the generator here.
template <int LPR, int QPL, bool FULL, bool SUMS = true, bool NOISE_IN = false, int SPEC = 0>
__device__ __forceinline__ void finish_elems(const StepParams& a, const int row, const int gl, const int q_off,
                                             const float mu, const float cg, const float4 (&p)[QPL],
                                             const float4 (&mm)[QPL], const float4 (&vv)[QPL],
                                             const float4 (&acc)[QPL], float4 (&po)[QPL], float4 (&mo)[QPL],
                                             float4 (&vo)[QPL], const float4* xi_in = nullptr) {
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  const bool maxcut = SPEC ? spec_problem(SPEC) == kMAXCUT : a.problem == kMAXCUT;
  const bool clique = SUMS && (SPEC ? spec_problem(SPEC) == kMAXCLIQUE : a.problem == kMAXCLIQUE);
  const bool adam = SPEC ? spec_rule(SPEC) == kADAMW : a.rule == kADAMW;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    po[k] = mo[k] = vo[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!FULL && q >= nq) continue;
    const float4 xi = NOISE_IN ? xi_in[k]
                               : normals4(philox4x32_10((uint32_t)row, (uint32_t)(q_off + q), a.k, kStreamNoise,
                                                        a.key0, a.key1));
    float4 T = make_float4(0.f, 0.f, 0.f, 0.f);  // max clique: 1^T p of the quad's replicas
    if (clique) {
#pragma unroll
      for (int c = 0; c < 4; ++c) set_comp(T, c, (float)((double)a.colsum[4 * q + c] * 0x1p-32));
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float pc = comp(p[k], c);
      const float C = comp(acc[k], c);
      // MIS: -1 + lambda C;  max-cut: C;  max clique: -1 + lambda (1^T p - 1/2 - C)
      const float gf = maxcut ? C : fmaf(a.lambda, clique ? (comp(T, c) - 0.5f) - C : C, -1.f);
      const float z = 2.f * pc - 1.f;
      const float ge = a.ce * (SPEC ? ipow_fixed<spec_alpha(SPEC) - 1>(z) : ipow_odd(z, a.alpha_e - 1));
      const float gc = cg * (pc - mu);
      const float g = gf + ge + gc;
      float pn, mn = 0.f, vn = 0.f;
      if (adam) {
        mn = fmaf(a.beta1, comp(mm[k], c), a.omb1 * g);
        vn = fmaf(a.beta2, comp(vv[k], c), a.omb2 * (g * g));
        const float den = __builtin_amdgcn_sqrtf(vn * a.inv_bc2) + a.eps;
        pn = pc * a.wd_factor - a.lr * (mn * a.inv_bc1) * __builtin_amdgcn_rcpf(den);
      } else {
        pn = pc - a.lr * g;
      }
      pn = fmaf(a.noise_scale, comp(xi, c), pn);
      pn = fminf(fmaxf(pn, 0.f), 1.f);
      const bool valid = FULL || 4 * q + c < a.S;
      set_comp(po[k], c, valid ? pn : 0.f);
      set_comp(mo[k], c, valid ? mn : 0.f);
      set_comp(vo[k], c, valid ? vn : 0.f);
    }
  }
}

// Statistics, then the element update, of one whole row.
template <int LPR, int QPL, bool FULL, bool SUMS = true, int SPEC = 0>
__device__ __forceinline__ void finish_row(const StepParams& a, const int row, const int gl, const float4 (&p)[QPL],
                                           const float4 (&mm)[QPL], const float4 (&vv)[QPL],
                                           const float4 (&acc)[QPL], float4 (&po)[QPL], float4 (&mo)[QPL],
                                           float4 (&vo)[QPL]) {
  float mu, cg;
  row_stats<LPR, QPL, FULL>(a, gl, p, mu, cg);
  finish_elems<LPR, QPL, FULL, SUMS, false, SPEC>(a, row, gl, 0, mu, cg, p, mm, vv, acc, po, mo, vo);
}

template <int LPR, int QPL, bool FULL, bool COHERENT = false>
__device__ __forceinline__ void store_row(const StepParams& a, float* P, const int row, const int gl,
                                          const float4 (&po)[QPL], const float4 (&mo)[QPL], const float4 (&vo)[QPL],
                                          const bool moments) {
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  const size_t base = (size_t)row * a.stride;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    if (!FULL && q >= nq) continue;
    if (COHERENT) store_coherent(P + base + 4 * q, po[k]);
    else *reinterpret_cast<float4*>(P + base + 4 * q) = po[k];
    if (moments && a.rule == kADAMW) {
      *reinterpret_cast<float4*>(a.m + base + 4 * q) = mo[k];
      *reinterpret_cast<float4*>(a.v + base + 4 * q) = vo[k];
    }
  }
}

// One update of one row, state streamed from and to memory.  DENSE: the coupling product
// was computed beforehand into a.coupling.
template <int LPR, int QPL, bool FULL, bool SUMS = true, bool DENSE = false, int SPEC = 0>
__device__ __forceinline__ void update_row(const StepParams& a, const int row, const int gl) {
  float4 p[QPL], mm[QPL], vv[QPL], acc[QPL], po[QPL], mo[QPL], vo[QPL];
  const RowMeta rm = DENSE ? RowMeta{0, 0, -1} : row_meta(a, row);
  load_row<LPR, QPL, FULL>(a, a.P_in, row, gl, p, mm, vv);  // issued before the gathers
  row_coupling<LPR, QPL, FULL, false, true, DENSE, kGatherQuads, SPEC>(a, row, rm, gl, acc);
  finish_row<LPR, QPL, FULL, SUMS, SPEC>(a, row, gl, p, mm, vv, acc, po, mo, vo);
  store_row<LPR, QPL, FULL>(a, a.P_out, row, gl, po, mo, vo, true);
}

}  // namespace qqa
