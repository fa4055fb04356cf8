// gfx950 kernels of batched CROWN-style bound propagation: the small kernels launched
// directly by the host side of the C-ABI (parameter-gradient contraction, concretization,
// layout of the fused spec rows, queue reset, weight copies and swizzles, final-row
// seeds, batch ordering, diagnostics export, the continuous-time flowpipe without a
// controller).
//   k_concretize   a6: FP64 box concretization with outward rounding.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "ct_flow.hpp"
#include "diffreach.h"

namespace dr {

// ---------------------------------------------------------------------------
// Parameter gradient: a contraction over the rows of the batch per layer,
//   dW_k[m][j] = sum_row A_k[row][m] E_{k-1}[row][j],   db_k[m] = sum_row A_k[row][m],
// with A the weighted multipliers and E the adjoints written by k_final<..., PGRAD>.
// ---------------------------------------------------------------------------
struct WgradArgs {
  const void* tape;         // column-major tapes, rows_pad entries per column
  size_t rows_pad;
  int rows;                 // valid rows (S R); later rows are read as zero
  int chunk_rows;           // rows per workgroup (multiple of 16)
  int n_chunks;
  size_t poff[kMaxL];       // partial sums of layer k at poff[k-1]: n_chunks x np_k x (np_{k-1} + 1)
  void* part;
  double* dW[kMaxL];        // outputs (natural n_k x n_{k-1}, FP64)
  double* db[kMaxL];
};

// One workgroup = (row chunk, 16-row tile m of dW_k, layer k).  Each wave owns the
// 16-column tiles j = wave, wave + 4, ... and runs the 16x16x4 MFMA over the chunk:
// a lane fetches four consecutive rows of one column with one vector load, and the
// four MFMA steps of a 16-row block take rows {v, 4 + v, 8 + v, 12 + v} in lane-group
// order (any bijection of the summation index is the same sum).
template <typename T>
__global__ void __launch_bounds__(256) k_wgrad(const NetDev* __restrict__ nets, int net_index, WgradArgs wa) {
  const NetDev& net = nets[net_index];
  const int k = blockIdx.z + 1, mt = blockIdx.y, chunk = blockIdx.x;
  const int L = net.L, NT = net.NT;
  const int npk = net.np[k], npj = net.np[k - 1];
  if (k > L || mt * 16 >= npk) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
  const int njt = npj / 16;
  const size_t rp = wa.rows_pad;
  gconst<T> tp = as_global((const T*)wa.tape);
  gconst<T> colA = tp + (size_t)(ptape_col_a(k, NT) + mt * 16 + n) * rp;
  const int cg0 = ptape_col_g(k - 1, L, NT, net.np[L]);
  const int row0 = chunk * wa.chunk_rows;
  const int row1 = min(row0 + wa.chunk_rows, (int)rp);
  V4<T> acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = V4<T>{0, 0, 0, 0};
  double bsum = 0.0;
  // the loads of block b + 16 are issued before the products of block b
  auto load = [&](int b, V4<T>& a4, V4<T> (&e4)[4]) {
    const int rb = b + 4 * g;
    a4 = *(gconst<V4<T>>)(colA + rb);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int jt = wave + 4 * u;
      if (jt < njt) e4[u] = *(gconst<V4<T>>)(tp + (size_t)(cg0 + jt * 16 + n) * rp + rb);
    }
  };
  V4<T> a_c, e_c[4], a_n, e_n[4];
  if (row0 < row1) load(row0, a_c, e_c);
  for (int b = row0; b < row1; b += 16) {
    if (b + 16 < row1) load(b + 16, a_n, e_n);
    const int rb = b + 4 * g;
    if (b + 16 > wa.rows) {   // the block holds rows past the last one: read them as zero
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rb + v >= wa.rows) {
          a_c[v] = (T)0;
#pragma unroll
          for (int u = 0; u < 4; ++u) e_c[u][v] = (T)0;
        }
    }
    if (wave == 0) bsum += (double)a_c[0] + (double)a_c[1] + (double)a_c[2] + (double)a_c[3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int jt = wave + 4 * u;
      if (jt < njt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u] = mfma16(a_c[v], e_c[u][v], acc[u]);
      }
    }
    a_c = a_n;
#pragma unroll
    for (int u = 0; u < 4; ++u) e_c[u] = e_n[u];
  }
  T* part = (T*)wa.part + wa.poff[k - 1] + (size_t)chunk * npk * (npj + 1);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int jt = wave + 4 * u;
    if (jt < njt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mt * 16 + nrn<T>(g, v);
        part[(size_t)m * (npj + 1) + jt * 16 + n] = acc[u][v];
      }
    }
  }
  if (wave == 0) {
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (g == 0) part[(size_t)(mt * 16 + n) * (npj + 1) + npj] = (T)bsum;
  }
}

// Sum of the per-chunk partials (FP64) into the natural-layout outputs.
template <typename T>
__global__ void k_wgrad_reduce(const NetDev* __restrict__ nets, int net_index, WgradArgs wa) {
  const NetDev& net = nets[net_index];
  const int k = blockIdx.y + 1;
  if (k > net.L) return;
  const int npk = net.np[k], npj = net.np[k - 1], nk = net.n[k], nj = net.n[k - 1];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * (nj + 1)) return;
  const int m = e / (nj + 1), jj = e % (nj + 1);
  const int j = jj < nj ? jj : npj;   // the last column holds the bias
  const T* part = (const T*)wa.part + wa.poff[k - 1];
  const size_t stride = (size_t)npk * (npj + 1);
  double sum = 0.0;
#pragma unroll 8
  for (int c = 0; c < wa.n_chunks; ++c) sum += (double)part[c * stride + (size_t)m * (npj + 1) + j];
  if (jj < nj) wa.dW[k - 1][(size_t)m * nj + jj] = sum;
  else wa.db[k - 1][m] = sum;
}

// ---------------------------------------------------------------------------
// a6: concretization of affine bounds over the boxes (FP64, outward rounding).
// ---------------------------------------------------------------------------
__global__ void k_concretize(int S, int q, int n0, int Q2, const double* __restrict__ xc, const double* __restrict__ xr,
                             const double* lam_lo, const double* acc_lo, const double* lam_hi,
                             const double* acc_hi, double* lb, double* ub, const uint32_t* ctx_st,
                             uint32_t* status) {
  // Q2 (a power of two >= q, <= 16) consecutive lanes per subdomain, one spec row each
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = e / Q2, r = e % Q2;
  const bool valid = s < S && r < q;
  const int sc_ = s < S ? s : 0, rc = r < q ? r : 0;
  const uint32_t cst = ctx_st ? ctx_st[sc_] : 0u;
  const bool dead = cst & (DR_RES_INFEASIBLE | DR_RES_BADSPLIT);
  uint32_t bits = 0;
  if (valid) {
    const size_t i = (size_t)sc_ * q + rc;
    double cl = acc_lo[i], ch = acc_hi[i], al = 0.0, ah = 0.0;
    for (int m = 0; m < n0; ++m) {
      double c = xc[(size_t)sc_ * n0 + m], rr = xr[(size_t)sc_ * n0 + m];
      double wl = lam_lo[i * n0 + m], wh = lam_hi[i * n0 + m];
      cl += wl * c - fabs(wl) * rr;
      ch += wh * c + fabs(wh) * rr;
      al += fabs(wl) * (fabs(c) + rr);
      ah += fabs(wh) * (fabs(c) + rr);
    }
    const double vl = cl - 0x1p-48 * (fabs(acc_lo[i]) + al);
    const double vh = ch + 0x1p-48 * (fabs(acc_hi[i]) + ah);
    lb[i] = dead ? INFINITY : vl;
    ub[i] = dead ? -INFINITY : vh;
    if (!dead && (!(fabs(vl) < INFINITY) || !(fabs(vh) < INFINITY))) bits = DR_RES_NONFINITE;
  }
  // OR of the row bits over the subdomain's lane group
  for (int o = 1; o < Q2; o <<= 1) bits |= (uint32_t)__shfl_xor((int)bits, o);
  if (status && s < S && r == 0) status[s] = cst | bits;
}

// a5 when fused into k_bound_init: lay the stored final rows out as the affine bounds.
__global__ void k_copy_final(int S, int q, int n0, const double* __restrict__ fin, const uint32_t* __restrict__ st,
                             double* lam_lo, double* acc_lo, double* lam_hi, double* acc_hi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int R = 2 * q;
  if (e >= S * R) return;
  const int s = e / R, r = e % R;
  const bool dead = st[s] & (DR_RES_INFEASIBLE | DR_RES_BADSPLIT);
  const double* f = fin + ((size_t)s * 16 + r) * 17;
  const bool lower = r < q;
  const int rr = lower ? r : r - q;
  double* lam = (lower ? lam_lo : lam_hi) + ((size_t)s * q + rr) * n0;
  for (int m = 0; m < n0; ++m) lam[m] = dead ? 0.0 : (lower ? f[m] : -f[m]);
  if (lower) acc_lo[(size_t)s * q + rr] = dead ? INFINITY : f[16];
  else acc_hi[(size_t)s * q + rr] = dead ? -INFINITY : -f[16];
}

// Work queue of a persistent launch, cleared by a kernel of its own just before the
// launch on the same stream (a kernel node, so graph replays need no memset node).
__global__ void k_reset_queue(unsigned* q) {
  if (threadIdx.x < 2) q[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------
// Natural padded copy of W_k (rows np_k, cols np_{k-1}) and b_k in the chain type.
template <typename T, typename S>
__global__ void k_copy_weights(const S* __restrict__ W, const S* __restrict__ b, int nk, int nkm1, int npk,
                               int npkm1, T* Wn, T* bn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npk * npkm1) {
    int r = i / npkm1, cc = i % npkm1;
    Wn[i] = (r < nk && cc < nkm1) ? (T)W[(size_t)r * nkm1 + cc] : (T)0;
  }
  if (i < npk) bn[i] = i < nk ? (T)b[i] : (T)0;
}

// Swizzle into MFMA A-operand order: block (mt, kt), lane l, sub-step i holds
// A[16 mt + l % 16][16 kt + nrn(l / 16, i)], with A[m][kk] = W[kk][m] (fwd) or W[m][kk] (adj).
template <typename T>
__global__ void k_swizzle(const T* __restrict__ Wn, int npk, int npkm1, int adjoint, T* out) {
  const int MT = (adjoint ? npk : npkm1) / 16, KT = (adjoint ? npkm1 : npk) / 16;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = MT * KT * 64 * 4;
  if (e >= total) return;
  const int i = e & 3, lane = (e >> 2) & 63, blk = e >> 8;
  const int mt = blk / KT, kt = blk % KT;
  const int m = mt * 16 + (lane & 15), kk = kt * 16 + nrn<T>(lane >> 4, i);
  out[e] = adjoint ? Wn[(size_t)m * npkm1 + kk] : Wn[(size_t)kk * npkm1 + m];
}

// Seeds of the final rows [c; -c]: a_L = c (or c B), g = a_L W_L, acc = a_L . b_L, skip = c A,
// and a priori bounds of their FP64 rounding (gamma_n = n u / (1 - n u), u = 2^-53, for a
// dot product of n terms: |fl(x.y) - x.y| <= gamma_n |x|.|y|):
//   |a_o - c.B_o| <= da_o = gamma_{n_target} sum_t |c_t| |B_to|,
//   seedWe_m = gamma_{n_L} sum_o |a_o| |W_om| + sum_o da_o |W_om|   (bounds |g_m - (cB) W_L[:, m]|),
//   seedBe   = gamma_{n_L} sum_o |a_o| |b_o|  + sum_o da_o |b_o|,
//   skipE_m  = gamma_{n_target} sum_t |c_t| |A_tm|.
// The sums of non-negative terms are inflated by 2^-40 relative to cover their own rounding.
__device__ __forceinline__ double gamma64(int n) {
  const double nu = n * 0x1p-53;
  return nu / (1.0 - nu);
}
template <typename T>
__global__ void k_seeds(const T* __restrict__ WL, const T* __restrict__ bL, int nL, int npLm1,
                        const double* __restrict__ C, int q, int n_target, const double* __restrict__ A,
                        const double* __restrict__ B, int n0, int npL, double* seedW, double* seedB, double* skip,
                        double* seedA, double* seedWe, double* seedBe, double* skipE, T* seedT, T* seedM) {
  const int R = 2 * q;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= R * npLm1) return;
  const int r = e / npLm1, m = e % npLm1;
  const int rr = r < q ? r : r - q;
  const double sg = r < q ? 1.0 : -1.0;
  const double ga = gamma64(n_target), gl = gamma64(nL);
  // multipliers on the network output
  double g = 0.0, acc = 0.0, eg = 0.0, eb = 0.0;
  for (int o = 0; o < nL; ++o) {
    double a = 0.0, aa = 0.0;
    if (B) {
      for (int t = 0; t < n_target; ++t) {
        a += C[(size_t)rr * n_target + t] * B[(size_t)t * nL + o];
        aa += fabs(C[(size_t)rr * n_target + t]) * fabs(B[(size_t)t * nL + o]);
      }
    } else {
      a = C[(size_t)rr * n_target + o];
    }
    a *= sg;
    const double da = B ? ga * aa : 0.0;
    if (m == 0) seedA[(size_t)r * npL + o] = a;
    const double w = (double)WL[(size_t)o * npLm1 + m], bo = (double)bL[o];
    g += a * w;
    acc += a * bo;
    eg += (gl * fabs(a) + da) * fabs(w);
    eb += (gl * fabs(a) + da) * fabs(bo);
  }
  seedW[(size_t)r * npLm1 + m] = g;
  seedWe[(size_t)r * npLm1 + m] = eg * (1.0 + 0x1p-40);
  const T gt = (T)g;
  seedT[(size_t)r * npLm1 + m] = gt;
  seedM[(size_t)r * npLm1 + m] = rup<T>((fabs(g - (double)gt) + 0x1p-50 * fabs(g) + eg * (1.0 + 0x1p-40)) * (1.0 + 0x1p-30));
  if (m == 0) {
    seedB[r] = acc;
    seedBe[r] = eb * (1.0 + 0x1p-40);
    for (int o = nL; o < npL; ++o) seedA[(size_t)r * npL + o] = 0.0;
  }
  if (m < 16) {
    double sk = 0.0, ske = 0.0;
    if (A && m < n0)
      for (int t = 0; t < n_target; ++t) {
        sk += C[(size_t)rr * n_target + t] * A[(size_t)t * n0 + m];
        ske += fabs(C[(size_t)rr * n_target + t]) * fabs(A[(size_t)t * n0 + m]);
      }
    skip[(size_t)r * 16 + m] = sg * sk;
    skipE[(size_t)r * 16 + m] = gamma64(n_target) * ske * (1.0 + 0x1p-40);
  }
}

// Natural (row-major, padded) copies of the step-boundary matrices of the unrolled
// closed loop, before their forward swizzle: Mn (16 x npLm1) = the seeds of the rows
// +e_r (B_r W_L in the chain type) for r < n_state, zero rows beyond; An (16 x 16) = A
// rounded to the chain type, rows r < n_state, columns m < n_0.
template <typename T>
__global__ void k_joint_mats(const T* __restrict__ seedT, int npLm1, const double* __restrict__ A, int ns, int n0,
                             T* Mn, T* An) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 16 * npLm1) {
    const int r = e / npLm1;
    Mn[e] = r < ns ? seedT[e] : (T)0;
  }
  if (e < 256) {
    const int r = e >> 4, m = e & 15;
    An[e] = (r < ns && m < n0) ? (T)A[(size_t)r * n0 + m] : (T)0;
  }
}

// Zero n doubles (a kernel, not a memset node, so that graph replays of a call that
// accumulates into a caller's buffer stay correct).
__global__ void k_zero(double* p, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) p[e] = 0.0;
}

// Sum of the per-workgroup weight-gradient regions of the reach gradient (chain type)
// in a fixed order (FP64, deterministic) into the natural-layout outputs.
struct ReachWreduceArgs {
  const void* wreg;
  size_t stride;            // chain-type elements per workgroup region
  size_t woff[kMaxL];
  int n_regions;
  double* dW[kMaxL];        // n_k x n_{k-1} FP64, or null
  double* db[kMaxL];        // n_k FP64, or null
};
template <typename T>
__global__ void k_reach_wreduce(const NetDev* __restrict__ nets, int net_index, ReachWreduceArgs ra) {
  const NetDev& net = nets[net_index];
  const int k = blockIdx.y + 1;
  if (k > net.L) return;
  const int nk = net.n[k], nj = net.n[k - 1], ld = net.np[k - 1] + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * (nj + 1)) return;
  const int i = e / (nj + 1), jj = e % (nj + 1);
  const int j = jj < nj ? jj : ld - 1;   // the last column holds the bias
  const T* reg = (const T*)ra.wreg + ra.woff[k - 1] + (size_t)i * ld + j;
  double sum = 0.0;
  for (int w = 0; w < ra.n_regions; ++w) sum += (double)reg[(size_t)w * ra.stride];
  if (jj < nj) {
    if (ra.dW[k - 1]) ra.dW[k - 1][(size_t)i * nj + jj] = sum;
  } else if (ra.db[k - 1]) {
    ra.db[k - 1][i] = sum;
  }
}

// Counting sort of the batch by network id (one workgroup).
__global__ void k_order(int S, const int* __restrict__ net_id, int n_nets, int* order, int* net_cnt,
                        int* net_off, uint32_t* st) {
  __shared__ int cnt[kMaxNets], cur[kMaxNets];
  const int tid = threadIdx.x;
  if (tid < kMaxNets) cnt[tid] = 0;
  __syncthreads();
  for (int s = tid; s < S; s += blockDim.x) {
    int id = net_id ? net_id[s] : 0;
    if (id >= 0 && id < n_nets) atomicAdd(&cnt[id], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int o = 0;
    for (int i = 0; i < kMaxNets; ++i) {
      net_off[i] = o;
      cur[i] = o;
      net_cnt[i] = i < n_nets ? cnt[i] : 0;
      o += i < n_nets ? cnt[i] : 0;
    }
  }
  __syncthreads();
  for (int s = tid; s < S; s += blockDim.x) {
    int id = net_id ? net_id[s] : 0;
    if (id >= 0 && id < n_nets) {
      order[atomicAdd(&cur[id], 1)] = s;
      st[s] = 0u;
    } else {
      st[s] = DR_RES_BADSPLIT;
    }
  }
}

// Pre-activation bounds of the batch in natural order (diagnostics).  A single-network
// context (direct) reads network 0 whatever net_id holds; a subdomain whose id is
// outside [0, n_nets) was processed by no launch and gets NaN rows.
__global__ void k_export_bounds(int S, int Hp_max, int H_max, const NetDev* __restrict__ nets, int n_nets,
                                int direct, const int* net_id, const double* bl, const double* bu, double* l,
                                double* u) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * H_max) return;
  const int s = e / H_max, h = e % H_max;
  const int id = (direct || !net_id) ? 0 : net_id[s];
  double lo = NAN, hi = NAN;
  if (id >= 0 && id < n_nets) {
    const NetDev& net = nets[id];
    if (h < net.H) {
      int k = 1, hh = h;
      while (k < net.L - 1 && hh >= net.n[k]) { hh -= net.n[k]; ++k; }
      const size_t p = (size_t)s * Hp_max + (size_t)(k - 1) * 16 * net.NT + hh;
      lo = bl[p];
      hi = bu[p];
    }
  }
  l[e] = lo;
  u[e] = hi;
}

// The flowpipe without a controller: one wavefront per box (Algorithm "Reachability of
// CT Dynamics with TM Flowpipe"); each workgroup is one wavefront and takes boxes
// round-robin.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_flowpipe_ct(CtArgs ca) {
  extern __shared__ __align__(16) char ct_raw[];
  CtLds C;
  C.carve((double*)ct_raw, 0);
  ct_pairs(C, ca.dyn);
  for (int b = blockIdx.x; b < ca.batch.n_sub; b += gridDim.x) {
    ct_seed(C, ca, b, ca.dyn.n);
    bool ok = true;
    for (int k = 0; k < ca.n_ctl; ++k) ok = ct_steps(C, ca, false, b, k * ca.K) && ok;
    if (threadIdx.x == 0 && ca.status) ca.status[b] = ok ? 0u : (uint32_t)DR_RES_NONFINITE;
    ct_sync();
  }
}

// K flowpipe steps of every box of the closed loop with its input held (interval
// `interval` of Algorithm "Reachability of CT NN Control Systems"): the box's state and
// the input's model come from the state buffer (written by k_ct_control) and go back
// there; one wavefront per box.
__global__ void __launch_bounds__(64) k_flowpipe_ct_held(CtArgs ca, int interval) {
  extern __shared__ __align__(16) char ct_raw[];
  CtLds C;
  C.carve((double*)ct_raw, ca.dyn.n_u);
  ct_pairs(C, ca.dyn);
  const int lane = threadIdx.x;
  for (int b = blockIdx.x; b < ca.batch.n_sub; b += gridDim.x) {
    double* st = ca.state + (size_t)b * kCtState;
    const int n_u = ca.dyn.n_u;
    if (lane < kCtMax) { C.c[lane] = st[lane]; C.lo[lane] = st[272 + lane]; C.hi[lane] = st[288 + lane]; }
    if (lane < n_u) {
      C.U.c[lane] = st[304 + lane]; C.U.lo[lane] = st[576 + lane]; C.U.hi[lane] = st[592 + lane];
      C.U.l[lane] = 0.0; C.U.w[lane] = 0.0;
    }
    for (int e = lane; e < kCtMax * kCtMax; e += 64) {
      const int r = e >> 4, z = e & 15;
      C.S[r * kCtLd + z] = st[16 + e];
      if (r < n_u) { C.U.L[r * kCtLd + z] = st[320 + e]; C.U.M[r * kCtLd + z] = 0.0; }
    }
    ct_sync();
    const bool ok = ct_steps(C, ca, true, b, interval * ca.K);
    if (lane < kCtMax) { st[lane] = C.c[lane]; st[272 + lane] = C.lo[lane]; st[288 + lane] = C.hi[lane]; }
    if (lane < n_u) { st[576 + lane] = C.U.lo[lane]; st[592 + lane] = C.U.hi[lane]; }
    for (int e = lane; e < kCtMax * kCtMax; e += 64) {
      const int r = e >> 4, z = e & 15;
      st[16 + e] = C.S[r * kCtLd + z];
      if (r < n_u) st[320 + e] = C.U.L[r * kCtLd + z];
    }
    if (lane == 0 && !ok && ca.status) ca.status[b] |= (uint32_t)DR_RES_NONFINITE;
    ct_sync();
  }
}

}  // namespace dr
