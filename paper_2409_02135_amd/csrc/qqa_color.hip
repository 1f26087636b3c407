// Categorical K-state QQA for graph coloring (the paper's generalisation to discrete
// variables): state V in [0,1]^(N x K) per replica, sigma = Clamp-normalised rows
// (sigma_ik = V_ik / Z_i, Z_i = sum_k V_ik; an all-zero row reads as uniform 1/K, with
// Z_i taken as 1 in the chain rule), expected-conflict objective
//   l(sigma) = sum_{(i,j) in E, i<j} sum_k sigma_ik sigma_jk,
// categorical alpha-entropy s_K = sum_i {1 - c sum_k (K sigma_ik - 1)^alpha},
// c = 1 / ((K-1)((K-1)^(alpha-1) + 1)), and the replica STD term per (variable, colour).
//
// Layout: the (variable i, colour k) pairs are rows r = i*K + k of the usual replica layout
// (row-major, replicas contiguous, stride = S rounded up to 4), for V, m, v, sigma and the
// objective gradient G = dR/dsigma.  One update is two launches:
//   cat_grad_kernel    per row (i, k): sum_j A_ij sigma_jk (gathered through the graph's CSR
//                      with the row pitch K * stride), + the entropy and STD terms -> G
//   cat_update_*       per variable i: dR/dV_ik = (G_ik - sum_k' sigma_ik' G_ik') / Z_i,
//                      AdamW, sqrt(2 eta T) xi (Philox row i*K + k), clamp -> V; then sigma
//                      of the new V, in place.  K <= 8 keeps the variable's K rows in
//                      registers (one read of V, G, m, v); larger K takes three passes.
// Rounding: x_i = argmax_k V_ik (first maximum); cost = edges whose ends share a colour.
#include "qqa_device.h"

namespace qqa {

// sigma from V for variable i, quad q (all K colours); padding replicas 0
__global__ __launch_bounds__(kBlock) void cat_sigma_kernel(const float* __restrict__ V, float* __restrict__ sig,
                                                           int n, int K, int stride, int S) {
  const int nq = stride >> 2;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)n * nq) return;
  const int i = (int)(t / nq), q = (int)(t % nq);
  float4 Z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < K; ++k) {
    const float4 x = *reinterpret_cast<const float4*>(V + ((size_t)i * K + k) * stride + 4 * q);
    Z.x += x.x;
    Z.y += x.y;
    Z.z += x.z;
    Z.w += x.w;
  }
  const float u = 1.f / (float)K;
  for (int k = 0; k < K; ++k) {
    const size_t off = ((size_t)i * K + k) * stride + 4 * q;
    const float4 x = *reinterpret_cast<const float4*>(V + off);
    float4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float z = comp(Z, c);
      set_comp(o, c, 4 * q + c < S ? (z > 0.f ? comp(x, c) / z : u) : 0.f);
    }
    *reinterpret_cast<float4*>(sig + off) = o;
  }
}

// G_ik = sum_j A_ij sigma_jk + ce (K sigma_ik - 1)^(alpha-1) - alpha_c (sigma_ik - mu_ik) / std_ik
// a.P_in = sigma, a.n = N * K rows, a.ce = -gamma c alpha K
template <int LPR, int QPL, bool FULL>
__global__ __launch_bounds__(kBlock) void cat_grad_kernel(StepParams a, int K, float* __restrict__ G) {
  int r = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  if (LPR == 64) r = __builtin_amdgcn_readfirstlane(r);
  if (r >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LPR - 1);
  const int i = r / K, k = r % K;
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  // neighbours' sigma of colour k: rows j*K + k, i.e. pitch K*stride from sigma + k*stride
  StepParams b = a;
  b.P_in = a.P_in + (size_t)k * a.stride;
  b.stride = K * a.stride;
  b.w = nullptr;
  float4 acc[QPL];
#pragma unroll
  for (int q = 0; q < QPL; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  gather_coupling<LPR, QPL, FULL>(b, a.row_ptr[i], a.row_ptr[i + 1], gl, nq, false, acc);
  float4 p[QPL];
  float sum = 0.f;
#pragma unroll
  for (int kk = 0; kk < QPL; ++kk) {
    const int q = gl + LPR * kk;
    p[kk] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (FULL || q < nq) p[kk] = *reinterpret_cast<const float4*>(a.P_in + (size_t)r * a.stride + 4 * q);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < a.S) sum += comp(p[kk], c);
  }
  sum = group_sum<LPR>(sum);
  const float mu = sum * a.inv_S;
  float sq = 0.f;
#pragma unroll
  for (int kk = 0; kk < QPL; ++kk) {
    const int q = gl + LPR * kk;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < a.S) {
        const float d = comp(p[kk], c) - mu;
        sq = fmaf(d, d, sq);
      }
  }
  sq = group_sum<LPR>(sq);
  const float sd = __builtin_amdgcn_sqrtf(sq * a.inv_S);
  const float cg = sd > 0.f ? -a.comm_alpha * __builtin_amdgcn_rcpf(sd) : 0.f;
  const float Kf = (float)K;
#pragma unroll
  for (int kk = 0; kk < QPL; ++kk) {
    const int q = gl + LPR * kk;
    if (!FULL && q >= nq) continue;
    float4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float s = comp(p[kk], c);
      const float g = comp(acc[kk], c) + a.ce * ipow_odd(fmaf(Kf, s, -1.f), a.alpha_e - 1) + cg * (s - mu);
      set_comp(o, c, (FULL || 4 * q + c < a.S) ? g : 0.f);
    }
    *reinterpret_cast<float4*>(G + (size_t)r * a.stride + 4 * q) = o;
  }
}

// One pass over the K colour rows of variable i, quad q: V, G and the moments are read once
// and kept in registers (K <= KMAX), then the step, then sigma of the new V from the same
// registers.
// sum_k sigma_k G_k is formed as (sum_k V_k G_k) / Z, which is the same quantity as the
// generic kernel's (rounded differently).
template <int KMAX>
__global__ __launch_bounds__(kBlock) void cat_update_regs_kernel(StepParams a, int K, const float* __restrict__ G,
                                                                 float* __restrict__ sig) {
  const int nq = a.stride >> 2;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)a.n * nq) return;
  const int i = (int)(t / nq), q = (int)(t % nq);
  const bool adam = a.rule == kADAMW;
  const size_t base = (size_t)i * K * a.stride + 4 * q;
  float4 x[KMAX], g[KMAX], mm[KMAX], vv[KMAX];
  float4 Z = make_float4(0.f, 0.f, 0.f, 0.f), XG = make_float4(0.f, 0.f, 0.f, 0.f), GS = XG;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= K) break;
    const size_t off = base + (size_t)k * a.stride;
    x[k] = *reinterpret_cast<const float4*>(a.P_in + off);
    g[k] = *reinterpret_cast<const float4*>(G + off);
    mm[k] = vv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (adam) {
      mm[k] = *reinterpret_cast<const float4*>(a.m + off);
      vv[k] = *reinterpret_cast<const float4*>(a.v + off);
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= K) break;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      set_comp(Z, c, comp(Z, c) + comp(x[k], c));
      set_comp(XG, c, fmaf(comp(x[k], c), comp(g[k], c), comp(XG, c)));
      set_comp(GS, c, comp(GS, c) + comp(g[k], c));
    }
  }
  const float u = 1.f / (float)K;
  float4 D, Zc;  // sum_k sigma_k G_k and Z (Z := 1 for an all-zero row)
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float z = comp(Z, c);
    set_comp(D, c, z > 0.f ? comp(XG, c) / z : comp(GS, c) * u);
    set_comp(Zc, c, z > 0.f ? z : 1.f);
  }
  float4 Zo = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= K) break;
    const size_t off = base + (size_t)k * a.stride;
    const float4 xi =
        normals4(philox4x32_10((uint32_t)(i * K + k), (uint32_t)q, a.k, kStreamNoise, a.key0, a.key1));
    float4 po, mo, vo;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float grad = (comp(g[k], c) - comp(D, c)) / comp(Zc, c);
      const float pc = comp(x[k], c);
      float pn, mn = 0.f, vn = 0.f;
      if (adam) {
        mn = fmaf(a.beta1, comp(mm[k], c), a.omb1 * grad);
        vn = fmaf(a.beta2, comp(vv[k], c), a.omb2 * (grad * grad));
        const float den = __builtin_amdgcn_sqrtf(vn * a.inv_bc2) + a.eps;
        pn = pc * a.wd_factor - a.lr * (mn * a.inv_bc1) * __builtin_amdgcn_rcpf(den);
      } else {
        pn = pc - a.lr * grad;
      }
      pn = fmaf(a.noise_scale, comp(xi, c), pn);
      pn = fminf(fmaxf(pn, 0.f), 1.f);
      const bool valid = 4 * q + c < a.S;
      set_comp(po, c, valid ? pn : 0.f);
      set_comp(mo, c, valid ? mn : 0.f);
      set_comp(vo, c, valid ? vn : 0.f);
      set_comp(Zo, c, comp(Zo, c) + (valid ? pn : 0.f));
    }
    x[k] = po;
    *reinterpret_cast<float4*>(a.P_out + off) = po;
    if (adam) {
      *reinterpret_cast<float4*>(a.m + off) = mo;
      *reinterpret_cast<float4*>(a.v + off) = vo;
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= K) break;
    float4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float z = comp(Zo, c);
      set_comp(o, c, 4 * q + c < a.S ? (z > 0.f ? comp(x[k], c) / z : u) : 0.f);
    }
    *reinterpret_cast<float4*>(sig + base + (size_t)k * a.stride) = o;
  }
}

// per variable i and replica quad q: the chain rule through the normalisation, the step, and
// sigma of the new state.  a.P_in = V_in, a.P_out = V_out, a.m / a.v, a.n = N variables.
// Any K; three passes over the K colour rows.
__global__ __launch_bounds__(kBlock) void cat_update_kernel(StepParams a, int K, const float* __restrict__ G,
                                                            float* __restrict__ sig) {
  const int nq = a.stride >> 2;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)a.n * nq) return;
  const int i = (int)(t / nq), q = (int)(t % nq);
  const bool adam = a.rule == kADAMW;
  float4 Z = make_float4(0.f, 0.f, 0.f, 0.f), D = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < K; ++k) {
    const size_t off = ((size_t)i * K + k) * a.stride + 4 * q;
    const float4 x = *reinterpret_cast<const float4*>(a.P_in + off);
    const float4 s = *reinterpret_cast<const float4*>(sig + off);
    const float4 g = *reinterpret_cast<const float4*>(G + off);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      set_comp(Z, c, comp(Z, c) + comp(x, c));
      set_comp(D, c, fmaf(comp(s, c), comp(g, c), comp(D, c)));
    }
  }
  float4 Zo = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < K; ++k) {
    const size_t off = ((size_t)i * K + k) * a.stride + 4 * q;
    const float4 x = *reinterpret_cast<const float4*>(a.P_in + off);
    const float4 g = *reinterpret_cast<const float4*>(G + off);
    float4 mm = make_float4(0.f, 0.f, 0.f, 0.f), vv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (adam) {
      mm = *reinterpret_cast<const float4*>(a.m + off);
      vv = *reinterpret_cast<const float4*>(a.v + off);
    }
    const float4 xi =
        normals4(philox4x32_10((uint32_t)(i * K + k), (uint32_t)q, a.k, kStreamNoise, a.key0, a.key1));
    float4 po, mo, vo;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float z = comp(Z, c);
      const float grad = (comp(g, c) - comp(D, c)) / (z > 0.f ? z : 1.f);
      const float pc = comp(x, c);
      float pn, mn = 0.f, vn = 0.f;
      if (adam) {
        mn = fmaf(a.beta1, comp(mm, c), a.omb1 * grad);
        vn = fmaf(a.beta2, comp(vv, c), a.omb2 * (grad * grad));
        const float den = __builtin_amdgcn_sqrtf(vn * a.inv_bc2) + a.eps;
        pn = pc * a.wd_factor - a.lr * (mn * a.inv_bc1) * __builtin_amdgcn_rcpf(den);
      } else {
        pn = pc - a.lr * grad;
      }
      pn = fmaf(a.noise_scale, comp(xi, c), pn);
      pn = fminf(fmaxf(pn, 0.f), 1.f);
      const bool valid = 4 * q + c < a.S;
      set_comp(po, c, valid ? pn : 0.f);
      set_comp(mo, c, valid ? mn : 0.f);
      set_comp(vo, c, valid ? vn : 0.f);
      set_comp(Zo, c, comp(Zo, c) + (valid ? pn : 0.f));
    }
    *reinterpret_cast<float4*>(a.P_out + off) = po;
    if (adam) {
      *reinterpret_cast<float4*>(a.m + off) = mo;
      *reinterpret_cast<float4*>(a.v + off) = vo;
    }
  }
  // sigma of the new state (this thread wrote exactly these elements above)
  const float u = 1.f / (float)K;
  for (int k = 0; k < K; ++k) {
    const size_t off = ((size_t)i * K + k) * a.stride + 4 * q;
    const float4 x = *reinterpret_cast<const float4*>(a.P_out + off);
    float4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float z = comp(Zo, c);
      set_comp(o, c, 4 * q + c < a.S ? (z > 0.f ? comp(x, c) / z : u) : 0.f);
    }
    *reinterpret_cast<float4*>(sig + off) = o;
  }
}

// Gradient and update in one launch, for shapes where one variable's K colour rows of NQ
// replica quads fit a lane group: lane l = k NQ + q of an LG = KP NQ lane group serves colour
// k (KP: K rounded up to a power of two; lanes k >= K only take part in the exchanges) and
// quad q of variable i.  sigma is read from sig_in (the neighbours' rows and the own row) and
// the new sigma goes to sig_out, so the neighbours' rows are never overwritten while read.
// Per element the operations and their order are those of cat_grad_kernel at one quad per
// lane followed by cat_update_regs_kernel: the colour sums of a replica (Z, sum V G, sum G,
// and the new Z) are formed in colour order from values exchanged through LDS.  ce is the
// gradient kernel's entropy coefficient (-gamma c alpha K); a is the update's parameters.
template <int NQ, int KP, int GB>
__global__ __launch_bounds__(kBlock) void cat_fused_kernel(StepParams a, int K, float ce,
                                                           const float* __restrict__ sig_in,
                                                           float* __restrict__ sig_out) {
  constexpr int LG = NQ * KP;
  constexpr int GPB = kBlock / LG;  // variables per block
  __shared__ float4 xs[GPB][KP][NQ];
  __shared__ float4 gs[GPB][KP][NQ];
  const int grp = (int)threadIdx.x / LG, l = (int)threadIdx.x % LG;
  const int k = l / NQ, q = l % NQ;
  const int i = (int)blockIdx.x * GPB + grp;
  const bool live = i < a.n;
  const bool colour = live && k < K;
  // lanes past the last variable or colour load a valid row (unconditional loads) and store nothing
  const int ic = live ? i : a.n - 1, kc = k < K ? k : K - 1;
  const size_t off = ((size_t)ic * K + kc) * a.stride + 4 * q;
  const size_t pitch = (size_t)K * a.stride;  // between variables' colour-kc rows
  const bool adam = a.rule == kADAMW;
  const int e0 = a.row_ptr[ic], e1 = a.row_ptr[ic + 1];
  const float4 s_own = *reinterpret_cast<const float4*>(sig_in + off);
  const float4 x = *reinterpret_cast<const float4*>(a.P_in + off);
  const float4 mm = *reinterpret_cast<const float4*>((adam ? a.m : a.P_in) + off);
  const float4 vv = *reinterpret_cast<const float4*>((adam ? a.v : a.P_in) + off);

  // sum_j A_ij sigma_jk in edge order, neighbours' rows loaded in batches of GB (the batch
  // size changes no sum, only how many loads are in flight before the first is used)
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const float* sk = sig_in + (size_t)kc * a.stride + 4 * q;
  for (int b = e0; b < e1; b += GB) {
    float4 y[GB];
    bool ok[GB];
#pragma unroll
    for (int u = 0; u < GB; ++u) {
      const int e = b + u;
      ok[u] = e < e1;
      y[u] = *reinterpret_cast<const float4*>(sk + (size_t)a.col[ok[u] ? e : e1 - 1] * pitch);
    }
#pragma unroll
    for (int u = 0; u < GB; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float r = fmaf(1.f, comp(y[u], c), comp(acc, c));
        set_comp(acc, c, ok[u] ? r : comp(acc, c));
      }
  }
  // replica statistics of sigma_ik over the NQ lanes of colour k, then G = dR/dsigma_ik
  float sum = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (4 * q + c < a.S) sum += comp(s_own, c);
#pragma unroll
  for (int o = NQ / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, NQ);
  const float mu = sum * a.inv_S;
  float sq = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (4 * q + c < a.S) {
      const float d = comp(s_own, c) - mu;
      sq = fmaf(d, d, sq);
    }
#pragma unroll
  for (int o = NQ / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, NQ);
  const float sd = __builtin_amdgcn_sqrtf(sq * a.inv_S);
  const float cg = sd > 0.f ? -a.comm_alpha * __builtin_amdgcn_rcpf(sd) : 0.f;
  const float Kf = (float)K;
  float4 G;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float sv = comp(s_own, c);
    const float g = comp(acc, c) + ce * ipow_odd(fmaf(Kf, sv, -1.f), a.alpha_e - 1) + cg * (sv - mu);
    set_comp(G, c, 4 * q + c < a.S ? g : 0.f);
  }

  // the colour sums of each replica, in colour order
  xs[grp][k][q] = x;
  gs[grp][k][q] = G;
  __syncthreads();
  float4 Z = make_float4(0.f, 0.f, 0.f, 0.f), XG = Z, GS = Z;
  for (int kk = 0; kk < K; ++kk) {
    const float4 xv = xs[grp][kk][q], gv = gs[grp][kk][q];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      set_comp(Z, c, comp(Z, c) + comp(xv, c));
      set_comp(XG, c, fmaf(comp(xv, c), comp(gv, c), comp(XG, c)));
      set_comp(GS, c, comp(GS, c) + comp(gv, c));
    }
  }
  const float u = 1.f / Kf;
  const float4 xi = normals4(philox4x32_10((uint32_t)(ic * K + kc), (uint32_t)q, a.k, kStreamNoise, a.key0, a.key1));
  float4 po, mo, vo;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float z = comp(Z, c);
    const float D = z > 0.f ? comp(XG, c) / z : comp(GS, c) * u;
    const float grad = (comp(G, c) - D) / (z > 0.f ? z : 1.f);
    const float pc = comp(x, c);
    float pn, mn = 0.f, vn = 0.f;
    if (adam) {
      mn = fmaf(a.beta1, comp(mm, c), a.omb1 * grad);
      vn = fmaf(a.beta2, comp(vv, c), a.omb2 * (grad * grad));
      const float den = __builtin_amdgcn_sqrtf(vn * a.inv_bc2) + a.eps;
      pn = pc * a.wd_factor - a.lr * (mn * a.inv_bc1) * __builtin_amdgcn_rcpf(den);
    } else {
      pn = pc - a.lr * grad;
    }
    pn = fmaf(a.noise_scale, comp(xi, c), pn);
    pn = fminf(fmaxf(pn, 0.f), 1.f);
    const bool valid = 4 * q + c < a.S;
    set_comp(po, c, valid ? pn : 0.f);
    set_comp(mo, c, valid ? mn : 0.f);
    set_comp(vo, c, valid ? vn : 0.f);
  }
  // sigma of the new V: its colour sums, in colour order
  __syncthreads();
  xs[grp][k][q] = po;
  __syncthreads();
  float4 Zo = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int kk = 0; kk < K; ++kk) {
    const float4 pv = xs[grp][kk][q];
#pragma unroll
    for (int c = 0; c < 4; ++c) set_comp(Zo, c, comp(Zo, c) + comp(pv, c));
  }
  if (!colour) return;
  float4 so;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float z = comp(Zo, c);
    set_comp(so, c, 4 * q + c < a.S ? (z > 0.f ? comp(po, c) / z : u) : 0.f);
  }
  *reinterpret_cast<float4*>(a.P_out + off) = po;
  if (adam) {
    *reinterpret_cast<float4*>(a.m + off) = mo;
    *reinterpret_cast<float4*>(a.v + off) = vo;
  }
  *reinterpret_cast<float4*>(sig_out + off) = so;
}

// colours x_i = argmax_k V_ik (first maximum) per replica
__global__ __launch_bounds__(kBlock) void cat_color_kernel(const float* __restrict__ V, uint8_t* __restrict__ X,
                                                           int n, int K, int stride, int S) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)n * S) return;
  const int i = (int)(t / S), s = (int)(t % S);
  int arg = 0;
  float best = V[((size_t)i * K) * stride + s];
  for (int k = 1; k < K; ++k) {
    const float x = V[((size_t)i * K + k) * stride + s];
    if (x > best) {
      best = x;
      arg = k;
    }
  }
  X[(size_t)i * stride + s] = (uint8_t)arg;
}

// conflicts per replica: edges (i, j), j > i, whose ends share a colour; integer counts are
// folded in LDS, then one atomic per replica per block (order-free)
__global__ __launch_bounds__(kBlock) void cat_conflict_kernel(const int32_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const uint8_t* __restrict__ X, int n, int stride, int S,
                                                              unsigned long long* __restrict__ acc) {
  extern __shared__ unsigned long long cat_sh[];  // [stride]
  for (int s = threadIdx.x; s < stride; s += kBlock) cat_sh[s] = 0ull;
  __syncthreads();
  // block b covers rows b, b + gridDim.x, ...; threads over replicas
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    for (int s = threadIdx.x; s < S; s += kBlock) {
      const uint8_t xi = X[(size_t)i * stride + s];
      unsigned long long c = 0;
      for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int j = col[e];
        if (j > i && X[(size_t)j * stride + s] == xi) ++c;
      }
      if (c) atomicAdd(&cat_sh[s], c);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < S; s += kBlock)
    if (cat_sh[s]) atomicAdd(&acc[s], cat_sh[s]);
}

// the best replica's colouring
__global__ __launch_bounds__(kBlock) void cat_extract_kernel(const uint8_t* __restrict__ X, int n, int stride,
                                                             const int32_t* __restrict__ best, uint8_t* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = X[(size_t)i * stride + best[0]];
}

static unsigned blocks_for(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

hipError_t launch_cat_sigma(const float* V, float* sig, int n, int K, int stride, int S, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cat_sigma_kernel, dim3(blocks_for((long long)n * (stride >> 2))), dim3(kBlock), 0, st, V, sig, n,
                     K, stride, S);
  return hipGetLastError();
}

template <int LPR, int QPL>
static void launch_cat_grad_t(const StepParams& p, int K, float* G, hipStream_t st) {
  const dim3 grid(blocks_for((long long)p.n * LPR)), block(kBlock);
  if (p.S == 4 * LPR * QPL)
    hipLaunchKernelGGL((cat_grad_kernel<LPR, QPL, true>), grid, block, 0, st, p, K, G);
  else
    hipLaunchKernelGGL((cat_grad_kernel<LPR, QPL, false>), grid, block, 0, st, p, K, G);
}

hipError_t launch_cat_grad(const StepParams& p, int K, float* G, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(p.S, p.lanes_per_row);
#define X(L, Q)                        \
  if (r.lpr == L && r.qpl == Q) {      \
    launch_cat_grad_t<L, Q>(p, K, G, st); \
    return hipGetLastError();          \
  }
  QQA_FOR_EACH_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_cat_update(const StepParams& p, int K, const float* G, float* sig, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const dim3 grid(blocks_for((long long)p.n * (p.stride >> 2))), block(kBlock);
  if (K <= 4)
    hipLaunchKernelGGL((cat_update_regs_kernel<4>), grid, block, 0, st, p, K, G, sig);
  else if (K <= 8)
    hipLaunchKernelGGL((cat_update_regs_kernel<8>), grid, block, 0, st, p, K, G, sig);
  else  // more colours: the register footprint would leave too few loads in flight
    hipLaunchKernelGGL(cat_update_kernel, grid, block, 0, st, p, K, G, sig);
  return hipGetLastError();
}

bool cat_fused_shape(int S, int lanes_per_row, int K) {
  const int nq = (S + 3) / 4;
  if (K < 2 || K > 8 || (nq & (nq - 1)) != 0) return false;
  const ReplicaShape r = replica_shape(S, lanes_per_row);
  int kp = 2;
  while (kp < K) kp *= 2;
  return r.lpr == nq && r.qpl == 1 && kp * nq <= 64;
}

hipError_t launch_cat_fused(const StepParams& p, int K, float ce, const float* sig_in, float* sig_out, int64_t nnz,
                            hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  if (!cat_fused_shape(p.S, p.lanes_per_row, K)) return hipErrorInvalidValue;
  const int nq = (p.S + 3) / 4;
  int kp = 2;
  while (kp < K) kp *= 2;
  // neighbours loaded per batch: 16 above a mean degree of 8 (measured at ER n = 1e5, K = 8,
  // S = 32: 250 against 260 us per update at mean degree 10, but 205 against 194 at degree 5)
  const bool wide = nnz > 8 * (int64_t)p.n;
#define X(NQ, KP)                                                                                         \
  if (nq == NQ && kp == KP) {                                                                             \
    constexpr int gpb = kBlock / (NQ * KP);                                                               \
    const dim3 grid((unsigned)((p.n + gpb - 1) / gpb));                                                   \
    if (wide)                                                                                             \
      hipLaunchKernelGGL((cat_fused_kernel<NQ, KP, 16>), grid, dim3(kBlock), 0, st, p, K, ce, sig_in, sig_out); \
    else                                                                                                  \
      hipLaunchKernelGGL((cat_fused_kernel<NQ, KP, 8>), grid, dim3(kBlock), 0, st, p, K, ce, sig_in, sig_out); \
    return hipGetLastError();                                                                             \
  }
  X(1, 2) X(2, 2) X(4, 2) X(8, 2) X(16, 2) X(32, 2) X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(16, 4) X(1, 8) X(2, 8)
  X(4, 8) X(8, 8)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_cat_eval(const int32_t* row_ptr, const int32_t* col, const float* V, uint8_t* X, int n, int K,
                           int stride, int S, unsigned long long* acc, hipStream_t st) {
  hipError_t e = launch_fill_u64(acc, 2 * (size_t)stride, st);
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(cat_color_kernel, dim3(blocks_for((long long)n * S)), dim3(kBlock), 0, st, V, X, n, K, stride, S);
  const int blocks = std::max(1, std::min(n, 1024));
  hipLaunchKernelGGL(cat_conflict_kernel, dim3(blocks), dim3(kBlock), (size_t)stride * sizeof(unsigned long long), st,
                     row_ptr, col, X, n, stride, S, acc);
  return hipGetLastError();
}

hipError_t launch_cat_extract(const uint8_t* X, int n, int stride, const int32_t* best, uint8_t* x, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cat_extract_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, st, X, n, stride, best, x);
  return hipGetLastError();
}

}  // namespace qqa
