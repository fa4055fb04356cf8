// gfx950 kernels of batched CROWN-style bound propagation: the chain kernels.
//
// Steps (see the C-ABI header for the contract of each entry point):
//   k_bound_init   a1-a4: per-subdomain persistent workgroups: exact layer-1 bounds,
//                  IBP, CROWN intermediate bounds of IBP-unstable neurons on the
//                  matrix cores, split clamping, ReLU relaxation.
//   k_final        a5/a7: per-wave persistent tiles of final spec rows; plain CROWN
//                  (affine bounds out) or alpha/beta projected gradient ascent with a
//                  hand-written adjoint.
//   k_reach_dt     a8: per-box persistent workgroups, stepwise linear-TM closed loop
//                  with shared-slope CROWN.
// The templates are instantiated per chain type and tile count in instances.hip (one
// translation unit per instance set, compiled in parallel); the small set-up, layout
// and concretization kernels live in aux_kernels.hpp.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "diffreach.h"

namespace dr {

// Summation error of the offsets (bias and intercept terms) relative to sum |a'| (M + |b|):
// per 16-neuron tile a lane sums its 8 terms (two per neuron) in the chain type with fused
// multiply-adds (error <= gamma_8 sum |terms|, Higham's bound; gamma_8 < 2^-20 for FP32),
// then adds the tile's partial to an FP64 accumulator (error far below 2^-42).  The terms
// of a neuron are bounded by |a'| (M + |b|): |a' b| directly, and the intercept term
// |g t| = |a'| |l| <= |a'| M (a' = s g, t = -s l) up to the rounding of a'.
template <typename T> __host__ __device__ constexpr double acc_eps() { return sizeof(T) == 4 ? 0x1p-20 : 0x1p-42; }
constexpr double kMargInflate = 1.0 + 0x1p-12;

// ReLU relaxation of one neuron in the chain's arithmetic, with its margin
// coefficient mu: |a'| mu bounds the rounding introduced by this neuron's product
// a' W (a priori gamma_{2K} bound with v = |W| H) and by the relaxation product.
template <typename T>
__device__ V4<T> build_relax(double l, double u, double v, double bias, bool split, int K, bool shared,
                             int margin_on) {
  double M = fmax(fabs(l), fabs(u));
  T lo, up, t;
  bool inexact = split;
  if (!(u > 0.0)) {
    lo = 0; up = 0; t = 0;
  } else if (l >= 0.0) {
    lo = 1; up = 1; t = 0;
  } else {
    double s = u / (u - l);
    T sT = (T)s;
    double sd = (double)sT;
    double tt = fmax(-sd * l, u - sd * u);
    tt += fabs(tt) * 0x1p-50;
    up = sT;
    t = rup<T>(tt);
    lo = shared ? sT : ((u > -l) ? (T)1 : (T)0);
    inexact = true;
  }
  if (!(M < INFINITY)) M = 0.0;  // non-finite bounds are reported through status bits
  double mu = gamma_n<T>(2 * K) * v + (inexact ? 2.0 * unit_round<T>() * M : 0.0) +
              acc_eps<T>() * (fabs(bias) + M);
  mu *= 1.0 + 0x1p-40;
  if (!margin_on) mu = 0.0;
  V4<T> r;
  r[0] = lo; r[1] = up; r[2] = t; r[3] = rup<T>(mu);
  return r;
}

// Relaxation of one layer applied in place to the chain state st: the multipliers g
// over h_k become the row multipliers a' over z_k.  The offsets (a' b_k and the upper
// intercepts g t where g < 0; in the shared-slope form the lower offset takes g t for
// g < 0 and the upper one for g > 0) are summed per tile in the chain type and added to
// the FP64 accumulators once per tile; the margin accumulates |a'| mu per lane.
template <typename T, int NT, bool SHARED, typename RelPtr, typename Stage, typename BT>
__device__ __forceinline__ void relax_layer(Stage& st, RelPtr rel, lconst<BT> bias, int gq, double& acc,
                                            double& acc2, T& marg) {
  // the relaxation of tile t + 1 is loaded while tile t is processed
  V4<T> r_cur[4], r_nxt[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) r_cur[i] = rel[gq * 4 + i];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) r_nxt[i] = rel[(t + 1) * 16 + gq * 4 + i];
    }
    T pa = 0, pa2 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const V4<T> r = r_cur[i];
      const T gv = st.get(t, i);
      const bool neg = gv < (T)0;
      const T a = (neg ? r[1] : r[0]) * gv;
      const T bj = (T)bias[t * 16 + nrn<T>(gq, i)];
      pa = fma(a, bj, pa);
      pa = fma(gv, neg ? r[2] : (T)0, pa);
      if (SHARED) {
        pa2 = fma(a, bj, pa2);
        pa2 = fma(gv, neg ? (T)0 : r[2], pa2);
      }
      marg += fabs(a) * r[3];
      st.set(t, i, a);
    }
    acc += (double)pa;
    if (SHARED) acc2 += (double)pa2;
    tile_fence<T, NT>();
    if (t + 1 < NT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) r_cur[i] = r_nxt[i];
    }
  }
}

// st <- A st for NT x NT tiles of swizzled weights (the products finish before the
// state is overwritten).
template <typename T, int NT, typename P, typename Stage>
__device__ __forceinline__ void gemm_inplace(P Wsw, Stage& st, int lane) {
  T nxt[NT][4];
  gemm_k<T, NT, NT>(Wsw, st, nxt, lane);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) st.set(t, i, nxt[t][i]);
}

// Backward chain of one N-tile from hidden layer K-1 down to the input.  st holds
// the seed multipliers over h_{K-1} (in registers or in the wavefront's LDS stage,
// see stage_in_lds); on return w holds the input coefficients.  lds_b: the hidden
// biases staged in LDS (layer k at (k - 1) 16 NT).  With WL the products read the LDS
// copy lds_w of the forward-swizzled weights.
template <typename T, int NT, bool SHARED, bool WL = false, typename Stage, typename BT>
__device__ __forceinline__ void chain_to_input(const NetDev& net, int K, Stage& st, const V4<T>* rel_all,
                                               double& acc, double& acc2, T& marg, T (&w)[1][4], int lane,
                                               const BT* lds_b, const V4<T>* lds_w = nullptr) {
  const int gq = lane >> 4;
  for (int k = K - 1; k >= 1; --k) {
    relax_layer<T, NT, SHARED>(st, rel_all + (k - 1) * 16 * NT, (lconst<BT>)(lds_b + (k - 1) * 16 * NT), gq, acc,
                               acc2, marg);
    if constexpr (WL) {
      lconst<V4<T>> Wl = (lconst<V4<T>>)(lds_w + lds_w_offset(k, NT));
      if (k > 1)
        gemm_inplace<T, NT>(Wl, st, lane);
      else
        gemm_k<T, 1, NT>(Wl, st, w, lane);
    } else {
      gconst<V4<T>> Wg = as_global(uniform_ptr((const V4<T>*)net.Wf[k - 1]));
      if (k > 1)
        gemm_inplace<T, NT>(Wg, st, lane);
      else
        gemm_k<T, 1, NT>(Wg, st, w, lane);
    }
  }
}

// ---------------------------------------------------------------------------
// NR row tiles of one subdomain processed together by one wavefront (register chain
// states): the tiles share every load of the relaxation and of the weight tiles, and
// their independent products and relaxation steps interleave, which hides the latency
// of each tile's dependent chain behind the other's work.
// ---------------------------------------------------------------------------
template <typename T, int NT, int NR, typename RelPtr, typename BT>
__device__ __forceinline__ void relax_layer_n(T (&st)[NR][NT][4], RelPtr rel, lconst<BT> bias, int gq,
                                              double (&acc)[NR], T (&marg)[NR]) {
  V4<T> r_cur[4], r_nxt[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) r_cur[i] = rel[gq * 4 + i];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) r_nxt[i] = rel[(t + 1) * 16 + gq * 4 + i];
    }
    T bj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bj[i] = (T)bias[t * 16 + nrn<T>(gq, i)];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T pa = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const V4<T> rr = r_cur[i];
        const T gv = st[r][t][i];
        const bool neg = gv < (T)0;
        const T a = (neg ? rr[1] : rr[0]) * gv;
        pa = fma(a, bj[i], pa);
        pa = fma(gv, neg ? rr[2] : (T)0, pa);
        marg[r] += fabs(a) * rr[3];
        st[r][t][i] = a;
      }
      acc[r] += (double)pa;
    }
    if (t + 1 < NT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) r_cur[i] = r_nxt[i];
    }
  }
}

// out[r][mt] = sum_kt A(mt, kt) in[r][kt] for NR row tiles (A loaded once per tile pair).
template <typename T, int MT, int KT, int NR, typename P>
__device__ __forceinline__ void gemm_n(P Wsw, const T (&in)[NR][KT][4], T (&out)[NR][MT][4], int lane) {
  V4<T> acc[NR][MT];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[r][mt] = V4<T>{0, 0, 0, 0};
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const V4<T> a = Wsw[(mt * KT + kt) * 64 + lane];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r][mt] = mfma16(a[i], in[r][kt][i], acc[r][mt]);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[r][mt][i] = acc[r][mt][i];
}

// chain_to_input for NR register-held row tiles (plain relaxation, no shared slope).
template <typename T, int NT, int NR, bool WL, typename BT>
__device__ __forceinline__ void chain_to_input_n(const NetDev& net, int K, T (&st)[NR][NT][4], const V4<T>* rel_all,
                                                 double (&acc)[NR], T (&marg)[NR], T (&w)[NR][1][4], int lane,
                                                 const BT* lds_b, const V4<T>* lds_w) {
  const int gq = lane >> 4;
  for (int k = K - 1; k >= 1; --k) {
    relax_layer_n<T, NT, NR>(st, rel_all + (k - 1) * 16 * NT, (lconst<BT>)(lds_b + (k - 1) * 16 * NT), gq, acc,
                             marg);
    auto step = [&](auto Wp) {
      if (k > 1) {
        T nxt[NR][NT][4];
        gemm_n<T, NT, NT, NR>(Wp, st, nxt, lane);
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) st[r][t][i] = nxt[r][t][i];
      } else {
        gemm_n<T, 1, NT, NR>(Wp, st, w, lane);
      }
    };
    if constexpr (WL) step((lconst<V4<T>>)(lds_w + lds_w_offset(k, NT)));
    else step(as_global(uniform_ptr((const V4<T>*)net.Wf[k - 1])));
  }
}

// Stage the hidden biases (padded, layer k at (k - 1) 16 NT) into LDS, once per
// workgroup: in FP64 (BT = double, saves a conversion per relaxed multiplier, the
// offsets being summed in FP64) or in the chain type (less LDS and registers).
template <typename T, typename BT>
__device__ void stage_biases(const NetDev& net, BT* dst) {
  const int n16 = 16 * net.NT;
  for (int e = threadIdx.x; e < net.Hp; e += kWG) {
    const int k = e / n16;
    dst[e] = (BT)as_global((const T*)net.bn[k])[e - k * n16];
  }
}

// Element W_k[r][m] read from the LDS copy of the forward-swizzled weights of hidden
// layer k >= 2 (both widths 16 NT): the inverse of the forward swizzle.
template <typename T>
__device__ __forceinline__ T lds_weight(const V4<T>* lds_w, int k, int NT, int r, int m) {
  const int rr = r & 15;
  const int g = sizeof(T) == 4 ? rr >> 2 : rr & 3;    // lane group and component holding row rr
  const int c = sizeof(T) == 4 ? rr & 3 : rr >> 2;
  lconst<T> W = (lconst<T>)(lds_w + lds_w_offset(k, NT));
  return W[(((m >> 4) * NT + (r >> 4)) * 64 + g * 16 + (m & 15)) * 4 + c];
}

// Stage the forward-swizzled weights of layers 1..L-1 into LDS (once per workgroup):
// the layers are one contiguous range of the staged block, and each thread issues up to
// eight global loads before its LDS writes, so the copy costs few load round trips.
template <typename T>
__device__ void stage_weights(const NetDev& net, V4<T>* dst) {
  const int NT = net.NT, total = lds_w_count(net.L, NT);
  constexpr int kBatch = 8;
  for (int e0 = threadIdx.x; e0 < total; e0 += kBatch * kWG) {
    V4<T> v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * kWG;
      if (e < total) {
        const int k = e < NT * 64 ? 1 : 2 + (e - NT * 64) / (NT * NT * 64);   // layer of staged entry e
        v[u] = as_global((const V4<T>*)net.Wf[k - 1])[e - lds_w_offset(k, NT)];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * kWG;
      if (e < total) dst[e] = v[u];
    }
  }
}


// Synchronisation of the threads that share one subdomain: the whole workgroup
// (TPS = 256) or one wavefront (TPS = 64, where LDS operations of the wave are
// processed in order and only compiler reordering must be prevented).  Threads of a
// workgroup exchange data only through LDS inside these kernels (global results are
// written for later launches, or re-read only by the lane that wrote them), so the
// fences order LDS accesses alone: they never wait for global loads or stores in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
template <int TPS> __device__ __forceinline__ void sub_sync() {
  if (TPS == 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
  } else {
    lds_barrier();
  }
}

// Compact the flagged neurons j < n (flag(j) evaluated by the caller's lambda) into
// U; returns the count.  TPS threads take 16 NT neurons in chunks of TPS.
template <int TPS, typename F>
__device__ __forceinline__ int compact_flags(int n16, F flag_of, int* U, int* wcnt) {
  const int t = threadIdx.x & (TPS - 1), lane = threadIdx.x & 63;
  int total = 0;
  for (int c0 = 0; c0 < n16; c0 += TPS) {
    const int j = c0 + t;
    const bool flag = j < n16 && flag_of(j);
    unsigned long long m = __ballot(flag);
    int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (TPS == 64) {
      if (flag) U[total + pre] = j;
      total += __popcll(m);
    } else {
      const int wid = t >> 6;
      if (lane == 0) wcnt[wid] = __popcll(m);
      lds_barrier();
      int base = total, tot = 0;
      for (int w = 0; w < TPS / 64; ++w) {
        if (w < wid) base += wcnt[w];
        tot += wcnt[w];
      }
      if (flag) U[base + pre] = j;
      total += tot;
      lds_barrier();
    }
  }
  sub_sync<TPS>();
  return total;
}

// Interval (IBP) bound of neuron j of hidden layer k from the centre/radius of
// relu(h_{k-1}) (hc, hr, zero-padded to np_{k-1}), with v = |W_k| relu(u_{k-1}) for the
// margin coefficients; FP64 with outward rounding.  Four partial sums, vector loads.
template <typename T, int NT>
__device__ __forceinline__ void ibp_neuron(const NetDev& net, int k, int j, const double* hc, const double* hr,
                                           double& lo, double& hi, double& v) {
  constexpr int npk = 16 * NT;     // hidden layers k >= 2 take a padded hidden layer as input
  gconst<V4<T>> W = as_global((const V4<T>*)((const T*)net.Wn[k - 1] + (size_t)j * npk));
  double zc[4] = {0, 0, 0, 0}, zr[4] = {0, 0, 0, 0}, za[4] = {0, 0, 0, 0};
  // the whole weight row is in flight at once for narrow layers
  constexpr int kUnroll = NT <= 4 ? 4 * NT : 8;
#pragma unroll kUnroll
  for (int m4 = 0; m4 < npk / 4; ++m4) {
    V4<T> w4 = W[m4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double w = (double)w4[i], c = hc[m4 * 4 + i], r = hr[m4 * 4 + i];
      zc[i] += w * c;
      zr[i] += fabs(w) * r;
      za[i] += fabs(w) * c;
    }
  }
  const double zcs = (double)((const T*)net.bn[k - 1])[j] + ((zc[0] + zc[1]) + (zc[2] + zc[3]));
  const double zrs = (zr[0] + zr[1]) + (zr[2] + zr[3]);
  const double zas = (za[0] + za[1]) + (za[2] + za[3]);
  double e = 0x1p-44 * (zas + zrs + fabs(zcs));
  lo = zcs - zrs - e;
  hi = zcs + zrs + e;
  v = zas + zrs;
}

// relu(h) centre/radius of hidden layer k (for the next layer's IBP), zero-padded.
template <int TPS>
__device__ __forceinline__ void relu_box(const double* l, const double* u, int n16, double* hc, double* hr) {
  const int t = threadIdx.x & (TPS - 1);
  for (int m = t; m < n16; m += TPS) {
    const double a = fmax(l[m], 0.0), b = fmax(u[m], 0.0);
    hc[m] = 0.5 * (a + b);
    hr[m] = 0.5 * (b - a);
  }
}

// ---------------------------------------------------------------------------
// a1-a4: intermediate bounds, persistent.  TPS threads own one subdomain at a time:
// a whole workgroup (TPS = 256, wide networks: the chain tiles of a layer are spread
// over its four waves) or one wavefront (TPS = 64, narrow networks: four subdomains
// per workgroup progress independently, no workgroup barriers).  NR = 2 (a variant for
// narrow FP32 networks) processes the row tiles of a wavefront in pairs and asks for two
// waves per SIMD (a register budget of 256, which the paired tiles fill).
// ---------------------------------------------------------------------------
// NR: row tiles per chain step of a wavefront (1, or 2 for narrow FP32 networks).
template <int NR> constexpr int bound_min_waves() { return NR == 2 ? 2 : 1; }

template <typename T, int NT, bool WLDS, int TPS, int NR = 1>
__global__ void __launch_bounds__(kWG, (bound_min_waves<NR>()))
k_bound_init(const NetDev* __restrict__ nets, int net_index, BatchDev batch, Scratch sc, int inter_mode,
             int max_splits) {
  constexpr int kWaves = kWavesPerWG;
  extern __shared__ __align__(16) char lds_raw[];
  const NetDev& net = nets[net_index];
  const int L = net.L, Hp = net.Hp, HpS = sc.Hp_max;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int t = tid & (TPS - 1);                       // thread index within the subdomain's team
  const int n_team_waves = TPS / 64;
  const int wave_in_team = (TPS == 64) ? 0 : wid;
  const size_t sub_bytes = SubLds<T>::bytes(Hp, NT);
  // dynamic LDS: per-wave chain stages, the subdomain state(s), staged weights, biases
  char* stage = lds_raw + (size_t)wid * stage_bytes<T, NT>();
  char* lds_base = lds_raw + kWaves * stage_bytes<T, NT>();
  SubLds<T> S;
  S.carve(lds_base + (TPS == 64 ? (size_t)wid * sub_bytes : 0), Hp, NT);
  char* lds_tail = lds_base + (TPS == 64 ? kWaves : 1) * sub_bytes;
  V4<T>* lds_w = nullptr;
  if (WLDS) {
    lds_w = (V4<T>*)lds_tail;
    lds_tail += (size_t)lds_w_count(L, NT) * sizeof(V4<T>);
    stage_weights<T>(net, lds_w);
  }
  T* lds_b = (T*)lds_tail;
  stage_biases<T, T>(net, lds_b);
  lds_barrier();
  const int cnt = batch_count(sc, net_index);
  const int n0 = net.n[0];
  const int n16 = 16 * NT;

  // static round-robin assignment of the work items (item = worker + round * workers):
  // the per-subdomain costs are close to one another, and a shared queue counter would
  // serialise every worker's fetch at the same moment (measured: ~35 us of a 4096-item
  // launch whose items are short)
  const int n_workers = TPS == 64 ? (int)gridDim.x * kWaves : (int)gridDim.x;
  const int worker = TPS == 64 ? (int)blockIdx.x * kWaves + wid : (int)blockIdx.x;
  for (int item = worker;; item += n_workers) {
    if (item >= cnt) break;
    const int s = subdomain_of(sc, net_index, item);

    // ---- a1 ingest: box, splits
    if (t < 16) {
      S.xc[t] = t < n0 ? batch.xc[(size_t)s * n0 + t] : 0.0;
      S.xr[t] = t < n0 ? batch.xr[(size_t)s * n0 + t] : 0.0;
    }
    for (int p = t; p < Hp; p += TPS) {
      S.slot[p] = -1;
      S.l[p] = 0.0;
      S.u[p] = 0.0;
    }
    if (t == 0) S.misc[1] = 0;
    if (t < 8) sc.rows[(size_t)s * 8 + t] = 0;
    sub_sync<TPS>();
    if (t < n0) {
      double c = S.xc[t], r = S.xr[t];
      if (!(fabs(c) < INFINITY) || !(r < INFINITY) || !(r >= 0.0)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
    }
    if (batch.sptr) {
      int a = batch.sptr[s], b = batch.sptr[s + 1];
      if (b - a > max_splits || b < a) {
        if (t == 0) atomicOr(&S.misc[1], DR_RES_BADSPLIT);
      } else {
        for (int e = a + t; e < b; e += TPS) {
          uint32_t wd = batch.spk[e];
          int k = (int)(wd >> 24), j = (int)(wd & 0xFFFFu), pos = (int)((wd >> 16) & 1u);
          if (k < 1 || k > L - 1 || j >= net.n[k]) {
            atomicOr(&S.misc[1], DR_RES_BADSPLIT);
          } else {
            int p = (k - 1) * n16 + (j & ~15) + pos_of<T>(j & 15);
            S.slot[p] = ((e - a) << 1) | pos;
          }
        }
      }
    }
    sub_sync<TPS>();

    // ---- a2 layer 1: exact bounds of an affine map over the box
    {
      const int n1 = net.n[1];
      for (int j = t; j < n16; j += TPS) {
        const int p = (j & ~15) + pos_of<T>(j & 15);
        double lo = 0.0, hi = 0.0, v = 0.0, bj = 0.0;
        bool split = S.slot[p] >= 0;
        if (j < n1) {
          gconst<V4<T>> W = as_global((const V4<T>*)((const T*)net.Wn[0] + (size_t)j * net.np[0]));
          bj = (double)((const T*)net.bn[0])[j];
          double zc = bj, zr = 0.0, za = 0.0;
#pragma unroll
          for (int m4 = 0; m4 < 4; ++m4) {
            V4<T> w4 = W[m4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double w = (double)w4[i];
              zc += w * S.xc[m4 * 4 + i];
              zr += fabs(w) * S.xr[m4 * 4 + i];
              za += fabs(w) * fabs(S.xc[m4 * 4 + i]);
            }
          }
          double e = 0x1p-44 * (za + zr + fabs(zc));
          lo = zc - zr - e;
          hi = zc + zr + e;
          v = za + zr;
          if (split) {
            if (S.slot[p] & 1) lo = fmax(lo, 0.0); else hi = fmin(hi, 0.0);
          }
          if (lo > hi) atomicOr(&S.misc[1], DR_RES_INFEASIBLE);
          if (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
        }
        S.l[j] = lo;
        S.u[j] = hi;
        S.rel[p] = build_relax<T>(lo, hi, v, bj, split, n1, false, sc.margin_on);
      }
    }
    sub_sync<TPS>();

    // ---- a3/a4 deeper hidden layers
    for (int k = 2; k <= L - 1; ++k) {
      if (S.misc[1] & (DR_RES_INFEASIBLE | DR_RES_BADSPLIT)) break;
      const int nk = net.n[k];
      const int base = (k - 1) * n16, pbase = (k - 2) * n16;
      relu_box<TPS>(S.l + pbase, S.u + pbase, n16, S.hc, S.hr);
      sub_sync<TPS>();
      for (int j = t; j < n16; j += TPS) {
        double lo = 0.0, hi = 0.0, v = 0.0;
        if (j < nk) ibp_neuron<T, NT>(net, k, j, S.hc, S.hr, lo, hi, v);
        S.ibl[j] = lo; S.ibu[j] = hi; S.v[j] = v;
        S.l[base + j] = lo; S.u[base + j] = hi;
      }
      sub_sync<TPS>();
      auto unstable = [&](int j) {
        const int p = base + (j & ~15) + pos_of<T>(j & 15);
        return j < nk && S.ibl[j] < 0.0 && S.ibu[j] > 0.0 && S.slot[p] < 0 && inter_mode == DR_INTER_CROWN_IBP;
      };
      const int nU = compact_flags<TPS>(n16, unstable, S.U, S.misc + 2);
      const int nrows = 2 * nU;
      const int ntiles = (nrows + 15) >> 4;
      if constexpr (TPS == 64) {
        // one subdomain per wavefront: row tiles in pairs (a last odd tile alone)
        auto rows_n = [&](auto nr_tag, int tile0) {
          constexpr int NRS = decltype(nr_tag)::value;
          const int gq = lane >> 4;
          T g[NRS][NT][4];
          double acc[NRS];
          T marg[NRS];
          T w[NRS][1][4];
          int row[NRS], neuron[NRS];
          bool valid[NRS];
          // seeds: rows +-e_j at z_k, i.e. +-W_k[j][:] over h_{k-1}, one vector load per
          // 16-neuron tile from the adjoint-swizzled copy (block (j / 16, tile), lane
          // j % 16 + 16 gq holds W_k[j][16 tile + nrn(gq, 0..3)])
          gconst<V4<T>> Wa = as_global(uniform_ptr((const V4<T>*)net.Wa[k - 1]));
#pragma unroll
          for (int r = 0; r < NRS; ++r) {
            row[r] = (tile0 + r) * 16 + (lane & 15);
            valid[r] = row[r] < nrows;
            neuron[r] = valid[r] ? S.U[row[r] >> 1] : 0;
            const T sg = valid[r] ? ((row[r] & 1) ? (T)-1 : (T)1) : (T)0;
            const int lb0 = ((neuron[r] >> 4) * NT) * 64 + (neuron[r] & 15) + 16 * gq;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
              const V4<T> wv = Wa[lb0 + tt * 64];
#pragma unroll
              for (int i = 0; i < 4; ++i) g[r][tt][i] = sg * wv[i];
            }
            // the seed offset enters once per row (lane group 0)
            acc[r] = (gq == 0 ? (double)sg : 0.0) * (double)lds_b[(k - 1) * n16 + neuron[r]];
            marg[r] = 0;
          }
          chain_to_input_n<T, NT, NRS, WLDS>(net, k, g, S.rel, acc, marg, w, lane, lds_b, lds_w);
#pragma unroll
          for (int r = 0; r < NRS; ++r) {
            double conc = 0.0, wabs = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m = nrn<T>(gq, i);
              const double wm = (double)w[r][0][i];
              conc += wm * S.xc[m] - fabs(wm) * S.xr[m];
              wabs += fabs(wm) * (fabs(S.xc[m]) + S.xr[m]);
            }
            conc = row_sum(conc);
            wabs = row_sum(wabs);
            const double accs = row_sum(acc[r]);
            const double mg = (double)row_sum(marg[r]) * kMargInflate;
            const double lb = accs + conc - mg - 0x1p-48 * (fabs(accs) + wabs);
            if (valid[r] && lane < 16) {
              if (row[r] & 1) S.u[base + neuron[r]] = fmin(S.ibu[neuron[r]], -lb);
              else S.l[base + neuron[r]] = fmax(S.ibl[neuron[r]], lb);
            }
          }
        };
        static_assert(NR == 1 || (NR == 2 && TPS == 64), "tile pairs need one subdomain per wavefront");
        int tile = 0;
        if constexpr (NR == 2)
          for (; tile + 1 < ntiles; tile += 2) rows_n(std::integral_constant<int, 2>{}, tile);
        for (; tile < ntiles; ++tile) rows_n(std::integral_constant<int, 1>{}, tile);
      } else {
        for (int tile = wave_in_team; tile < ntiles; tile += n_team_waves) {
          const int row = tile * 16 + (lane & 15);
          const bool valid = row < nrows;
          const int neuron = valid ? S.U[row >> 1] : 0;
          const T sgn = (row & 1) ? (T)-1 : (T)1;
          auto g = make_stage<T, NT>(stage, lane);
          const int gq = lane >> 4;
          const T sg = valid ? sgn : (T)0;
          if (WLDS) {
  #pragma unroll
            for (int tt = 0; tt < NT; ++tt)
  #pragma unroll
              for (int i = 0; i < 4; ++i) g.set(tt, i, sg * lds_weight<T>(lds_w, k, NT, neuron, tt * 16 + nrn<T>(gq, i)));
          } else {
            gconst<T> Wr = as_global((const T*)net.Wn[k - 1] + (size_t)neuron * net.np[k - 1]);
  #pragma unroll
            for (int tt = 0; tt < NT; ++tt)
  #pragma unroll
              for (int i = 0; i < 4; ++i) g.set(tt, i, sg * Wr[tt * 16 + nrn<T>(gq, i)]);
          }
          // the seed offset enters once per row (lane group 0); the other groups add their neurons' terms
          double acc = (gq == 0 ? (double)sg : 0.0) * (double)lds_b[(k - 1) * n16 + neuron], acc2 = 0.0;
          T marg = 0;
          T w[1][4];
          chain_to_input<T, NT, false, WLDS>(net, k, g, S.rel, acc, acc2, marg, w, lane, lds_b, lds_w);
          double conc = 0.0, wabs = 0.0;
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = nrn<T>(gq, i);
            double wm = (double)w[0][i];
            conc += wm * S.xc[m] - fabs(wm) * S.xr[m];
            wabs += fabs(wm) * (fabs(S.xc[m]) + S.xr[m]);
          }
          conc = row_sum(conc);
          wabs = row_sum(wabs);
          acc = row_sum(acc);
          double mg = (double)row_sum(marg) * kMargInflate;
          double lb = acc + conc - mg - 0x1p-48 * (fabs(acc) + wabs);
          if (valid && lane < 16) {
            if (row & 1) S.u[base + neuron] = fmin(S.ibu[neuron], -lb);
            else S.l[base + neuron] = fmax(S.ibl[neuron], lb);
          }
        }
      }
      sub_sync<TPS>();
      for (int j = t; j < n16; j += TPS) {
        const int p = base + (j & ~15) + pos_of<T>(j & 15);
        double lo = S.l[base + j], hi = S.u[base + j];
        bool split = S.slot[p] >= 0;
        double bj = 0.0;
        if (j < nk) {
          bj = (double)lds_b[base + j];
          if (split) {
            if (S.slot[p] & 1) lo = fmax(lo, 0.0); else hi = fmin(hi, 0.0);
          }
          if (lo > hi) atomicOr(&S.misc[1], DR_RES_INFEASIBLE);
          if (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
          S.l[base + j] = lo;
          S.u[base + j] = hi;
        }
        S.rel[p] = build_relax<T>(lo, hi, S.v[j], bj, split, nk, false, sc.margin_on);
      }
      if (t == 0) sc.rows[(size_t)s * 8 + (k - 1)] = nrows;
      sub_sync<TPS>();
    }

    // ---- a5 fused: plain-CROWN spec rows of this subdomain while its relaxation is in LDS
    if (sc.fuse && wave_in_team == 0) {
      const bool live = !(S.misc[1] & (DR_RES_INFEASIBLE | DR_RES_BADSPLIT));
      const int r = lane & 15, gq = lane >> 4;
      const bool valid = live && r < net.R;
      const int rr = r < net.R ? r : 0;
      gconst<T> seed = as_global((const T*)net.seedT + (size_t)rr * net.np[L - 1]);
      gconst<T> seed_m = as_global((const T*)net.seedM + (size_t)rr * net.np[L - 1]);
      const int lbase = (L - 2) * n16;
      auto g = make_stage<T, NT>(stage, lane);
      T marg = 0;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = tt * 16 + nrn<T>(gq, i);
          g.set(tt, i, valid ? seed[m] : (T)0);
          if (sc.margin_on && valid) marg += seed_m[m] * (T)fmax(S.u[lbase + m], 0.0);
          if (i == 3) tile_fence<T, NT>();
        }
      double acc = net.seedB[rr] * ((valid && gq == 0) ? 1.0 : 0.0), acc2 = 0.0;
      T w[1][4];
      chain_to_input<T, NT, false, WLDS>(net, L, g, S.rel, acc, acc2, marg, w, lane, lds_b, lds_w);
      double wt[4], conc = 0.0, wabs = 0.0, ske = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = nrn<T>(gq, i);
        wt[i] = (double)w[0][i] + net.skip[(size_t)rr * 16 + m];
        conc += wt[i] * S.xc[m] - fabs(wt[i]) * S.xr[m];
        wabs += fabs(wt[i]) * (fabs(S.xc[m]) + S.xr[m]);
        ske += net.skipE[(size_t)rr * 16 + m] * (fabs(S.xc[m]) + S.xr[m]);
      }
      conc = row_sum(conc);
      wabs = row_sum(wabs);
      const double accs = row_sum(acc);
      const double seed_mg = sc.margin_on ? net.seedBe[rr] + row_sum(ske) : 0.0;
      const double mg = (double)row_sum(marg) * kMargInflate + 0x1p-48 * (fabs(accs) + wabs) + seed_mg;
      if (valid) {
        double* f = sc.fin + ((size_t)s * 16 + r) * 17;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = nrn<T>(gq, i);
          if (m < n0) f[m] = wt[i];
        }
        if (gq == 0) {
          const double ao = accs - mg;
          f[16] = ao;
          sc.margin[(size_t)s * 32 + r] = mg;
          if (!(fabs(ao) < INFINITY) || !(mg < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
          else if (mg > fmax(1.0, fabs(accs + conc - mg))) atomicOr(&S.misc[1], DR_RES_MARGIN);
        }
      }
    }
    sub_sync<TPS>();

    // ---- write back
    const size_t so = (size_t)s * HpS;
    for (int p = t; p < Hp; p += TPS) {
      sc.bl[so + p] = S.l[p];
      sc.bu[so + p] = S.u[p];
      ((V4<T>*)sc.rel)[so + p] = S.rel[p];
      sc.slot[so + p] = S.slot[p];
    }
    if (t == 0) {
      sc.st[s] = (uint32_t)S.misc[1];
      if (sc.st_out) sc.st_out[s] = (uint32_t)S.misc[1];
      sc.rows[(size_t)s * 8 + (L - 1)] = net.R;
    }
    sub_sync<TPS>();
  }
}

// ---------------------------------------------------------------------------
// a5 / a7: final spec rows.  One wave = one N-tile holding P = 16 / R subdomains.
// ---------------------------------------------------------------------------
// The caller's duals are projected on read onto their feasible sets (alpha in [0, 1],
// beta >= 0; NaN maps to 0, which both sets contain): every evaluated bound is then a
// valid bound whatever the caller passes, and bound, gradient and ascent step are
// those of the projected point.
__device__ __forceinline__ float proj_alpha(float a) { return fminf(fmaxf(a, 0.0f), 1.0f); }
__device__ __forceinline__ float proj_beta(float b) { return fmaxf(b, 0.0f); }

// Per-lane inputs of one 16-neuron tile of a dual-ascent relaxation step: the
// relaxation, the split slot and the current alpha / beta of the lane's row (alpha and
// beta are read at clamped addresses and selected by the caller).
template <typename T>
struct GroupIn {
  V4<T> rr[4];
  int sp[4];
  float a[4], b[4];
};
template <typename T, typename RP, typename SP>
__device__ __forceinline__ void load_group(GroupIn<T>& g, RP rk, SP sk, gmut<float> arow, gmut<float> brow, int t,
                                           int gq, int hoff, int nk) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = t * 16 + nrn<T>(gq, i);
    g.rr[i] = rk[t * 16 + gq * 4 + i];
    g.sp[i] = sk[t * 16 + gq * 4 + i];
    const bool uns = g.rr[i][2] > (T)0 && c < nk;
    g.a[i] = proj_alpha(arow[uns ? hoff + c : 0]);
    g.b[i] = proj_beta(brow[g.sp[i] >= 0 ? (g.sp[i] >> 1) : 0]);
  }
}

// alpha / beta of one 16-neuron tile (addresses from the relaxation and split slots).
template <typename T, typename RP, typename SP>
__device__ __forceinline__ void load_ab(float (&ao)[4], float (&bo)[4], RP rk, SP sk, gmut<float> arow,
                                        gmut<float> brow, int t, int gq, int hoff, int nk) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = t * 16 + nrn<T>(gq, i);
    const bool uns = rk[t * 16 + gq * 4 + i][2] > (T)0 && c < nk;
    const int sp = sk[t * 16 + gq * 4 + i];
    ao[i] = proj_alpha(arow[uns ? hoff + c : 0]);
    bo[i] = proj_beta(brow[sp >= 0 ? (sp >> 1) : 0]);
  }
}
// Pipeline depth (tiles) of the dual loads: deeper when the relaxation is in LDS.
template <bool CACHE> constexpr int dual_depth() { return CACHE ? 3 : 1; }


template <typename T, int NT, bool DUALS, bool CACHE = false, bool PGRAD = false>
__global__ void __launch_bounds__(kWG) k_final(const NetDev* __restrict__ nets, int net_index, FinalArgs fa) {
  static_assert(!PGRAD || DUALS, "the parameter gradient extends the dual adjoint");
  extern __shared__ __align__(16) char lds_raw[];
  // dynamic LDS: per-wave chain stages, the hidden biases, then (CACHE) per-wave item copies
  char* stage = lds_raw + (size_t)(threadIdx.x >> 6) * stage_bytes<T, NT, true>();
  const NetDev& net = nets[net_index];
  // biases in the chain type for the plain spec rows (tile partials in T), in FP64 for
  // the dual ascent (its offsets are summed in FP64 per neuron)
  using BT = std::conditional_t<DUALS, double, T>;
  BT* lds_b = (BT*)(lds_raw + kWavesPerWG * stage_bytes<T, NT, true>());
  stage_biases<T, BT>(net, lds_b);
  lds_barrier();
  const int Hp = net.Hp;
  char* cache = (char*)lds_b + (((size_t)Hp * sizeof(double) + 15) & ~(size_t)15) +
                (size_t)(threadIdx.x >> 6) * item_cache_bytes<T>(16 / net.R, Hp);
  const Scratch& sc = fa.sc;
  const int tid = threadIdx.x, lane = tid & 63, gq = lane >> 4, n = lane & 15;
  const int L = net.L, R = net.R, q = net.q, n0 = net.n[0];
  const int P = 16 / R;
  const int cnt = batch_count(sc, net_index);
  const int n_items = (cnt + P - 1) / P;
  const int HpS = sc.Hp_max;
  const unsigned n_workers = gridDim.x * kWavesPerWG;
  const int wave_global = blockIdx.x * kWavesPerWG + (tid >> 6);
  gmut<T> tape = as_global_mut(DUALS ? (T*)fa.tape + (size_t)wave_global * (L - 1) * NT * 256 : (T*)nullptr);

  bool first = true;
  for (;;) {
    const int item = next_item(fa.queue, first, wave_global, (int)n_workers);
    if (item >= n_items) break;
    const int sl = n / R, r = n % R;
    const int idx = item * P + sl;
    const bool inrange = (sl < P) && (idx < cnt);
    const int s = inrange ? subdomain_of(sc, net_index, idx) : 0;
    const uint32_t st = inrange ? sc.st[s] : 0u;
    const bool live = inrange && !(st & (DR_RES_INFEASIBLE | DR_RES_BADSPLIT));
    const size_t so = (size_t)s * HpS;
    gconst<V4<T>> rel = as_global((const V4<T>*)sc.rel + so);
    gconst<int> slot = as_global(sc.slot + so);
    // relaxation / slots of this lane's subdomain: global, or the wave's LDS copy
    using RelP = std::conditional_t<CACHE, lconst<V4<T>>, gconst<V4<T>>>;
    using SlotP = std::conditional_t<CACHE, lconst<int>, gconst<int>>;
    RelP relb;
    SlotP slotb;
    if constexpr (CACHE) {
      lmut<V4<T>> crel = (lmut<V4<T>>)cache;
      lmut<int> cslot = (lmut<int>)(cache + (size_t)P * Hp * sizeof(V4<T>));
      for (int e = lane; e < P * Hp; e += 64) {
        const int sle = e / Hp, p = e - sle * Hp;
        const int idxe = item * P + sle;
        const int se = idxe < cnt ? subdomain_of(sc, net_index, idxe) : 0;
        crel[e] = as_global((const V4<T>*)sc.rel)[(size_t)se * HpS + p];
        cslot[e] = as_global(sc.slot)[(size_t)se * HpS + p];
      }
      sub_sync<64>();
      const int slc = sl < P ? sl : 0;
      relb = (RelP)(crel + slc * Hp);
      slotb = (SlotP)(cslot + slc * Hp);
    } else {
      relb = rel;
      slotb = slot;
    }
    // loads below are unconditional (addresses are clamped into range) and masked
    // by selects, so the wave runs straight-line code
    double xcv[4], xrv[4];
    gconst<double> xcp = as_global(fa.batch.xc + (size_t)s * n0);
    gconst<double> xrp = as_global(fa.batch.xr + (size_t)s * n0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = nrn<T>(gq, i);
      const bool ok = inrange && m < n0;
      const int mm = m < n0 ? m : 0;
      const double xv = xcp[mm], rv = xrp[mm];
      xcv[i] = ok ? xv : 0.0;
      xrv[i] = ok ? rv : 0.0;
    }
    const double liveD = live ? 1.0 : 0.0;
    // parameter gradient: this lane's tape row and its weight (zero for dead rows)
    const size_t prow = (size_t)s * R + r;
    double omega = 0.0;
    if constexpr (PGRAD) {
      if (live) omega = r < q ? fa.g_lb[(size_t)s * q + r] : -fa.g_ub[(size_t)s * q + (r - q)];
    }
    auto ptape_at = [&](int col) -> gmut<T> { return as_global_mut((T*)fa.ptape + (size_t)col * fa.rows_pad + prow); };
    // seed margin: rounding of the FP64 seed g = a_L W_L to the chain type, times |h_{L-1}|
    gconst<T> seed = as_global((const T*)net.seedT + (size_t)r * net.np[L - 1]);
    gconst<T> seed_m = as_global((const T*)net.seedM + (size_t)r * net.np[L - 1]);
    const int lbase = (L - 2) * 16 * NT;
    gmut<float> arow = as_global_mut(DUALS ? fa.alpha + ((size_t)s * R + r) * fa.H_max : (float*)nullptr);
    gmut<float> brow = as_global_mut(DUALS ? fa.beta + ((size_t)s * R + r) * fa.max_splits : (float*)nullptr);
    gconst<double> bu = as_global(sc.bu + so + lbase);
    // the seed's rounding margin is the same in every evaluation
    T marg0 = 0;
    if (sc.margin_on) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = t * 16 + nrn<T>(gq, i);
          if (live) marg0 += seed_m[m] * (T)fmax(bu[m], 0.0);
          if (i == 3) tile_fence<T, NT>();
        }
    }
    double best = -INFINITY, lbv = 0.0, mgv = 0.0;
    const int n_eval = DUALS ? fa.iters + 1 : 1;
    for (int it = 0; it < n_eval; ++it) {
      // read the caller's duals unless they are initialised here (first iteration)
      const bool use_in = live && !(fa.init_duals && it == 0);
      auto st = make_stage<T, NT, true>(stage, lane);   // the chain state of this wavefront
      double acc = net.seedB[r] * ((gq == 0) ? liveD : 0.0), acc2 = 0.0;
      T marg = marg0;
      {
        // seeds of tile t + 1 are loaded while tile t is stored
        T sd_cur[4], sd_nxt[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) sd_cur[i] = seed[nrn<T>(gq, i)];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (t + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sd_nxt[i] = seed[(t + 1) * 16 + nrn<T>(gq, i)];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) st.set(t, i, live ? sd_cur[i] : (T)0);
          tile_fence<T, NT>();
          if (t + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sd_cur[i] = sd_nxt[i];
          }
        }
      }
      // forward (backward bound propagation) with optional alpha/beta and tape
      T w[1][4];
      {
        for (int k = L - 1; k >= 1; --k) {
          const RelP rk = relb + (k - 1) * 16 * NT;
          if (!DUALS) {
            relax_layer<T, NT, false>(st, rk, (lconst<BT>)(lds_b + (k - 1) * 16 * NT), gq, acc, acc2, marg);
          } else {
            lconst<double> bias = (lconst<double>)(lds_b + (k - 1) * 16 * NT);
            const int hoff = net.hoff[k - 1], nk = net.n[k];
            const SlotP sk = slotb + (k - 1) * 16 * NT;
            // the relaxation, split slots and duals of tile t + 1 are loaded while tile t
            // is processed (distance-one software pipelining across the scheduling fences)
            // relaxed multiplier of neuron (t, i) with the tile's inputs
            auto relax_one = [&](int t, int i, V4<T> rr, int sp, float aval, float bval) {
              const int c = t * 16 + nrn<T>(gq, i);
              T gv = st.get(t, i);
              tape[(((size_t)(k - 1) * NT + t) * 4 + i) * 64 + lane] = gv;
              const bool uns = rr[2] > (T)0 && c < nk;
              const T lo = uns ? (use_in ? (T)aval : rr[0]) : rr[0];
              T a = (gv >= (T)0 ? lo : rr[1]) * gv;
              const T bv = (sp >= 0 && use_in) ? (T)bval : (T)0;
              a -= (sp & 1) ? bv : -bv;
              double bj = (double)bias[c];
              acc += fmin((double)gv * (double)rr[2], 0.0) + (double)a * bj;
              marg += fabs(a) * rr[3];
              st.set(t, i, a);
            };
            if constexpr (CACHE) {
              // relaxation and slots from LDS at use; alpha / beta DEP tiles ahead
              constexpr int DEP = dual_depth<CACHE>();
              float a_r[DEP + 1][4], b_r[DEP + 1][4];
#pragma unroll
              for (int tt = 0; tt < DEP; ++tt)
                if (tt < NT) load_ab<T>(a_r[tt], b_r[tt], rk, sk, arow, brow, tt, gq, hoff, nk);
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if (t + DEP < NT)
                  load_ab<T>(a_r[(t + DEP) % (DEP + 1)], b_r[(t + DEP) % (DEP + 1)], rk, sk, arow, brow, t + DEP, gq,
                             hoff, nk);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  relax_one(t, i, rk[t * 16 + gq * 4 + i], sk[t * 16 + gq * 4 + i], a_r[t % (DEP + 1)][i],
                            b_r[t % (DEP + 1)][i]);
                tile_fence<T, NT>();
              }
            } else {
              GroupIn<T> cur_in, nxt_in;
              load_group<T>(cur_in, rk, sk, arow, brow, 0, gq, hoff, nk);
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if (t + 1 < NT) load_group<T>(nxt_in, rk, sk, arow, brow, t + 1, gq, hoff, nk);
#pragma unroll
                for (int i = 0; i < 4; ++i) relax_one(t, i, cur_in.rr[i], cur_in.sp[i], cur_in.a[i], cur_in.b[i]);
                tile_fence<T, NT>();
                if (t + 1 < NT) cur_in = nxt_in;
              }
            }
          }
          gconst<V4<T>> Wg = as_global(uniform_ptr((const V4<T>*)net.Wf[k - 1]));
          if (k > 1)
            gemm_inplace<T, NT>(Wg, st, lane);
          else
            gemm_k<T, 1, NT>(Wg, st, w, lane);
        }
      }
      double wt[4];
      double conc = 0.0, wabs = 0.0, ske = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = nrn<T>(gq, i);
        wt[i] = (double)w[0][i] + net.skip[(size_t)r * 16 + m];
        conc += wt[i] * xcv[i] - fabs(wt[i]) * xrv[i];
        wabs += fabs(wt[i]) * (fabs(xcv[i]) + xrv[i]);
        ske += net.skipE[(size_t)r * 16 + m] * (fabs(xcv[i]) + xrv[i]);
      }
      conc = row_sum(conc);
      wabs = row_sum(wabs);
      double accs = row_sum(acc);
      const double seed_mg = sc.margin_on ? (net.seedBe[r] + row_sum(ske)) * liveD : 0.0;
      double mg = (double)row_sum(marg) * kMargInflate + 0x1p-48 * (fabs(accs) + wabs) + seed_mg;
      lbv = accs + conc - mg;
      mgv = mg;
      if (!DUALS) {
        if (live) {
          // every lane group writes its own input coefficients; lane group 0 the offsets
          const bool lower = r < q;
          const int rr = lower ? r : r - q;
          double* lam = lower ? fa.lam_lo : fa.lam_hi;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = nrn<T>(gq, i);
            if (m < n0) lam[((size_t)s * q + rr) * n0 + m] = lower ? wt[i] : -wt[i];
          }
          if (gq == 0) {
            double ao = accs - mg;
            if (lower) fa.acc_lo[(size_t)s * q + rr] = ao;
            else fa.acc_hi[(size_t)s * q + rr] = -ao;
            sc.margin[(size_t)s * 32 + r] = mg;
            if (!(fabs(ao) < INFINITY) || !(mg < INFINITY)) atomicOr(&sc.st[s], (uint32_t)DR_RES_NONFINITE);
            else if (mg > fmax(1.0, fabs(lbv))) atomicOr(&sc.st[s], (uint32_t)DR_RES_MARGIN);
          }
        }
        if (inrange && !live && gq == 0) {
          const bool lower = r < q;
          const int rr = lower ? r : r - q;
          double* lam = lower ? fa.lam_lo : fa.lam_hi;
          for (int m = 0; m < n0; ++m) lam[((size_t)s * q + rr) * n0 + m] = 0.0;
          if (lower) fa.acc_lo[(size_t)s * q + rr] = INFINITY;
          else fa.acc_hi[(size_t)s * q + rr] = -INFINITY;
          sc.margin[(size_t)s * 32 + r] = 0.0;
        }
        break;
      }
      best = fmax(best, lbv);
      const bool last = (it == n_eval - 1);
      const bool init_now = fa.init_duals && it == 0;
      if (last && !PGRAD && fa.galpha == nullptr && fa.gbeta == nullptr && !init_now) break;
      if constexpr (PGRAD) {
        // d lb / d xc = w, d lb / d xr = -|w|, summed over the R rows of the subdomain
        // with their weights (lanes sl R .. sl R + R - 1 of the lane group)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double vc = omega * wt[i], vr = -omega * fabs(wt[i]);
          double sc_ = 0.0, sr_ = 0.0;
          for (int j = 0; j < R; ++j) {
            const int src = (lane & ~15) + (sl < P ? sl : 0) * R + j;
            sc_ += __shfl(vc, src);
            sr_ += __shfl(vr, src);
          }
          const int m = nrn<T>(gq, i);
          if (inrange && r == 0 && m < n0) {
            if (fa.dxc) fa.dxc[(size_t)s * n0 + m] = live ? sc_ : 0.0;
            if (fa.dxr) fa.dxr[(size_t)s * n0 + m] = live ? sr_ : 0.0;
          }
        }
        if (inrange) {
          // a^(L): the seed row (weighted); e^(0) = xc - sgn(w) xr
          const int npL = net.np[L];
          for (int t = 0; t < npL / 16; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int o = t * 16 + nrn<T>(gq, i);
              ptape_at(ptape_col_a(L, NT) + o)[0] = (T)(omega * net.seedA[(size_t)r * npL + o]);
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double sg = wt[i] > 0.0 ? 1.0 : (wt[i] < 0.0 ? -1.0 : 0.0);
            ptape_at(ptape_col_g(0, L, NT, npL) + nrn<T>(gq, i))[0] = live ? (T)(xcv[i] - sg * xrv[i]) : (T)0;
          }
        }
      }
      // ---- hand-written adjoint of lb = acc + w.xc - |w|.xr w.r.t. alpha, beta
      // the chain state now holds d lb / d(W_k^T a'^(k)) (without the bias term)
      {
        T dw[1][4], dlt[NT][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double sg = wt[i] > 0.0 ? 1.0 : (wt[i] < 0.0 ? -1.0 : 0.0);
          dw[0][i] = (T)(xcv[i] - sg * xrv[i]);
        }
        gemm_tiles<T, NT, 1>((const V4<T>*)net.Wa[0], dw, dlt, lane);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) st.set(t, i, dlt[t][i]);
      }
      for (int k = 1; k <= L - 1; ++k) {
        const RelP rk = relb + (k - 1) * 16 * NT;
        lconst<double> bias = (lconst<double>)(lds_b + (k - 1) * 16 * NT);
        const int hoff = net.hoff[k - 1], nk = net.n[k];
        const SlotP sk = slotb + (k - 1) * 16 * NT;
        // adjoint of neuron (t, i) with the tile's inputs; PGA update of alpha / beta
        auto adjoint_one = [&](int t, int i, V4<T> rr, int sp, float aval, float bval, T gv) {
          const int c = t * 16 + nrn<T>(gq, i);
          T delta = st.get(t, i) + (T)bias[c];    // d lb / d a'^(k)
          const bool uns = rr[2] > (T)0 && c < nk;
          const float av = use_in ? aval : (float)rr[0];
          const T lo = uns ? (T)av : rr[0];
          T d = gv >= (T)0 ? lo : rr[1];
          if (uns && live) {
            T da = gv >= (T)0 ? delta * gv : (T)0;
            if (!last) {
              float nv = av + fa.lr * (float)da;
              nv = fminf(fmaxf(nv, 0.0f), 1.0f);
              arow[hoff + c] = nv;
            } else {
              if (init_now) arow[hoff + c] = av;
              if (fa.galpha) fa.galpha[((size_t)s * R + r) * fa.H_max + hoff + c] = (float)da;
            }
          }
          if (sp >= 0 && live) {
            T db = (sp & 1) ? -delta : delta;    // -sigma * delta
            float bv = use_in ? bval : 0.0f;
            if (!last) {
              brow[sp >> 1] = fmaxf(0.0f, bv + fa.lr * (float)db);
            } else {
              if (init_now) brow[sp >> 1] = bv;
              if (fa.gbeta) fa.gbeta[((size_t)s * R + r) * fa.max_splits + (sp >> 1)] = (float)db;
            }
          }
          const T e = delta * d + ((uns && gv < (T)0) ? rr[2] : (T)0);
          if constexpr (PGRAD) {
            if (inrange) {
              const T bs = (sp >= 0 && use_in) ? (T)bval : (T)0;
              const T am = d * gv - ((sp & 1) ? bs : -bs);   // a^(k), as in the forward pass
              ptape_at(ptape_col_a(k, NT) + c)[0] = live ? (T)(omega * (double)am) : (T)0;
              ptape_at(ptape_col_g(k, L, NT, net.np[L]) + c)[0] = live ? e : (T)0;
            }
          }
          st.set(t, i, e);
        };
        auto tape_at = [&](int t, int i) { return tape[(((size_t)(k - 1) * NT + t) * 4 + i) * 64 + lane]; };
        if constexpr (CACHE) {
          constexpr int DEP = dual_depth<CACHE>();
          float a_r[DEP + 1][4], b_r[DEP + 1][4];
          T g_r[DEP + 1][4];
#pragma unroll
          for (int tt = 0; tt < DEP; ++tt)
            if (tt < NT) {
              load_ab<T>(a_r[tt], b_r[tt], rk, sk, arow, brow, tt, gq, hoff, nk);
#pragma unroll
              for (int i = 0; i < 4; ++i) g_r[tt][i] = tape_at(tt, i);
            }
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            if (t + DEP < NT) {
              constexpr int W = DEP + 1;
              load_ab<T>(a_r[(t + DEP) % W], b_r[(t + DEP) % W], rk, sk, arow, brow, t + DEP, gq, hoff, nk);
#pragma unroll
              for (int i = 0; i < 4; ++i) g_r[(t + DEP) % W][i] = tape_at(t + DEP, i);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
              adjoint_one(t, i, rk[t * 16 + gq * 4 + i], sk[t * 16 + gq * 4 + i], a_r[t % (DEP + 1)][i],
                          b_r[t % (DEP + 1)][i], g_r[t % (DEP + 1)][i]);
            tile_fence<T, NT>();
          }
        } else {
          GroupIn<T> cur_in, nxt_in;
          T g_cur[4], g_nxt[4];
          load_group<T>(cur_in, rk, sk, arow, brow, 0, gq, hoff, nk);
#pragma unroll
          for (int i = 0; i < 4; ++i) g_cur[i] = tape_at(0, i);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            if (t + 1 < NT) {
              load_group<T>(nxt_in, rk, sk, arow, brow, t + 1, gq, hoff, nk);
#pragma unroll
              for (int i = 0; i < 4; ++i) g_nxt[i] = tape_at(t + 1, i);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
              adjoint_one(t, i, cur_in.rr[i], cur_in.sp[i], cur_in.a[i], cur_in.b[i], g_cur[i]);
            tile_fence<T, NT>();
            if (t + 1 < NT) {
              cur_in = nxt_in;
#pragma unroll
              for (int i = 0; i < 4; ++i) g_cur[i] = g_nxt[i];
            }
          }
        }
        if (k < L - 1) gemm_inplace<T, NT>(as_global(uniform_ptr((const V4<T>*)net.Wa[k])), st, lane);
      }
      if (last) break;
    }
    if (DUALS && lane < 16 && inrange) {
      const bool lower = r < q;
      const int rr = lower ? r : r - q;
      double bv = live ? best : INFINITY;
      if (lower) fa.lb[(size_t)s * q + rr] = bv;
      else fa.ub[(size_t)s * q + rr] = -bv;
      sc.margin[(size_t)s * 32 + r] = live ? mgv : 0.0;
      if (live && !(fabs(best) < INFINITY)) atomicOr(&sc.st[s], (uint32_t)DR_RES_NONFINITE);
    }
  }
}

// ---------------------------------------------------------------------------
// a8: stepwise closed-loop reachability with linear TMs (one WG per box).
// One step of the stepwise reach on the Taylor model tm = (c 16, P 16 x 16, I_lo 16,
// I_hi 16, |x| bound 16) entering the step: the intermediate bounds of the network over
// the model (layer 1 exact, deeper layers shared-slope CROWN intersected with IBP) and
// the model of x' = A v + B f(v) in (nc, nP, nI_lo, nI_hi) at tm + 320 .. (see
// k_reach_dt).  Records the step into the tape tb (if not null) and writes the box of
// x' to bx (if not null).  Called by the whole workgroup.
template <typename T, int NT>
__device__ __forceinline__ void tm_crown_step(const NetDev& net, const Scratch& sc, SubLds<T>& S, char* stage,
                                              T* lds_b, double* tm, double* tb, int step, int H, int s, double* bx) {
  const int L = net.L, Hp = net.Hp;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, gq = lane >> 4;
  const int n0 = net.n[0], ns = net.n_state;
  double* c = tm;
  double* Pm = tm + 16;
  double* Ilo = tm + 272;
  double* Ihi = tm + 288;
  double* Xab = tm + 304;
  double* nc = tm + 320;
  double* nP = tm + 336;
  double* nIlo = tm + 592;
  double* nIhi = tm + 608;
      // ---- layer 1 on the TM input: exact range of W_1 (c + P z + r) + b_1
      {
        const int n1 = net.n[1];
        for (int j = tid; j < 16 * NT; j += kWG) {
          const int p = (j & ~15) + pos_of<T>(j & 15);
          double lo = 0.0, hi = 0.0, v = 0.0, bj = 0.0;
          if (j < n1) {
            const T* W = (const T*)net.Wn[0] + (size_t)j * net.np[0];
            bj = (double)((const T*)net.bn[0])[j];
            double zc = bj, zr = 0.0, za = 0.0, zab = 0.0;
            double wp[16];
            for (int z = 0; z < 16; ++z) wp[z] = 0.0;
            for (int m = 0; m < n0; ++m) {
              double w = (double)W[m];
              zc += w * (c[m] + 0.5 * (Ilo[m] + Ihi[m]));
              zr += fabs(w) * 0.5 * (Ihi[m] - Ilo[m]);
              za += fabs(w) * Xab[m];
              zab += fabs(w) * (fabs(c[m]) + 0.5 * fabs(Ilo[m] + Ihi[m]));
              for (int z = 0; z < n0; ++z) wp[z] += w * Pm[m * 16 + z];
            }
            for (int z = 0; z < n0; ++z) zr += fabs(wp[z]);
            double e = 0x1p-44 * (za + zab + zr + fabs(zc));
            lo = zc - zr - e;
            hi = zc + zr + e;
            v = za;
            if (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
          }
          S.l[j] = lo; S.u[j] = hi;
          S.rel[p] = build_relax<T>(lo, hi, v, bj, false, n1, true, sc.margin_on);
          if (tb) {
            double* tl = tb + reach_tape_bounds(step, H, Hp);
            tl[j] = lo; tl[Hp + j] = hi; tl[2 * Hp + j] = lo; tl[3 * Hp + j] = hi;
          }
        }
      }
      lds_barrier();
      // ---- deeper hidden layers: shared-slope CROWN on the TM input, intersected with IBP
      for (int k = 2; k <= L - 1; ++k) {
        const int nk = net.n[k];
        const int base = (k - 1) * 16 * NT, pbase = (k - 2) * 16 * NT;
        relu_box<kWG>(S.l + pbase, S.u + pbase, 16 * NT, S.hc, S.hr);
        lds_barrier();
        if (tid < 16 * NT) {
          const int j = tid;
          double lo = 0.0, hi = 0.0, v = 0.0;
          if (j < nk) ibp_neuron<T, NT>(net, k, j, S.hc, S.hr, lo, hi, v);
          S.ibl[j] = lo; S.ibu[j] = hi; S.v[j] = v;
          S.l[base + j] = lo; S.u[base + j] = hi;
        }
        lds_barrier();
        auto unstable = [&](int j) { return j < nk && S.ibl[j] < 0.0 && S.ibu[j] > 0.0; };
        const int nU = compact_flags<kWG>(16 * NT, unstable, S.U, S.misc + 2);
        const int ntiles = (nU + 15) >> 4;
        for (int tile = wid; tile < ntiles; tile += kWavesPerWG) {
          const int row = tile * 16 + (lane & 15);
          const bool valid = row < nU;
          const int neuron = valid ? S.U[row] : 0;
          auto g = make_stage<T, NT>(stage, lane);
          const T* Wrow = (const T*)net.Wn[k - 1] + (size_t)neuron * net.np[k - 1];
          const T sg = valid ? (T)1 : (T)0;
          gconst<T> Wr = as_global(Wrow);
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) g.set(t, i, sg * Wr[t * 16 + nrn<T>(gq, i)]);
          double acc = (gq == 0 ? (double)sg : 0.0) * (double)lds_b[base + neuron], acc2 = acc;
          T marg = 0;
          T w[1][4];
          chain_to_input<T, NT, true>(net, k, g, S.rel, acc, acc2, marg, w, lane, lds_b);
          // TM evaluation of w.x + [acc, acc2] over x = c + P z + r
          double base_v = 0.0, il = 0.0, ih = 0.0, wabs = 0.0;
          double wp[16];
#pragma unroll
          for (int z = 0; z < 16; ++z) wp[z] = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = nrn<T>(gq, i);
            double wm = (double)w[0][i];
            base_v += wm * c[m];
            double a1 = wm * Ilo[m], a2 = wm * Ihi[m];
            il += fmin(a1, a2); ih += fmax(a1, a2);
            wabs += fabs(wm) * Xab[m];
#pragma unroll
            for (int z = 0; z < 16; ++z) wp[z] += wm * Pm[m * 16 + z];
          }
          base_v = row_sum(base_v); il = row_sum(il); ih = row_sum(ih); wabs = row_sum(wabs);
          double rad = 0.0;
#pragma unroll
          for (int z = 0; z < 16; ++z) rad += fabs(row_sum(wp[z]));
          acc = row_sum(acc); acc2 = row_sum(acc2);
          double mg = (double)row_sum(marg) * kMargInflate + 0x1p-46 * (wabs + fabs(acc) + fabs(acc2));
          double lo = acc + base_v - rad + il - mg;
          double hi = acc2 + base_v + rad + ih + mg;
          if (valid && lane < 16) {
            S.l[base + neuron] = fmax(S.ibl[neuron], lo);
            S.u[base + neuron] = fmin(S.ibu[neuron], hi);
          }
        }
        lds_barrier();
        if (tid < 16 * NT) {
          const int j = tid;
          const int p = base + (j & ~15) + pos_of<T>(j & 15);
          double lo = S.l[base + j], hi = S.u[base + j], bj = 0.0;
          if (j < nk) {
            bj = (double)lds_b[base + j];
            if (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
          }
          S.rel[p] = build_relax<T>(lo, hi, S.v[j], bj, false, nk, true, sc.margin_on);
          if (tb) {
            double* tl = tb + reach_tape_bounds(step, H, Hp) + base;
            tl[j] = lo; tl[Hp + j] = hi; tl[2 * Hp + j] = S.ibl[j]; tl[3 * Hp + j] = S.ibu[j];
          }
        }
        if (tid == 0) sc.rows[(size_t)s * 8 + (k - 1)] += nU;
        lds_barrier();
      }
      // ---- output rows e_r on x' (r < n_state): multipliers B_r on y, skip A_r
      if (wid == 0) {
        const int r = lane & 15;
        const bool valid = r < ns;
        gconst<T> seed = as_global((const T*)net.seedT + (size_t)(valid ? r : 0) * net.np[L - 1]);
        gconst<T> seed_m = as_global((const T*)net.seedM + (size_t)(valid ? r : 0) * net.np[L - 1]);
        const int lbase = (L - 2) * 16 * NT;
        auto g = make_stage<T, NT>(stage, lane);
        T marg = 0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = t * 16 + nrn<T>(gq, i);
            g.set(t, i, valid ? seed[m] : (T)0);
            if (sc.margin_on && valid) marg += seed_m[m] * (T)fmax(S.u[lbase + m], 0.0);
            if (i == 3) tile_fence<T, NT>();
          }
        double acc = net.seedB[valid ? r : 0] * ((valid && gq == 0) ? 1.0 : 0.0), acc2 = acc;
        T w[1][4];
        chain_to_input<T, NT, true>(net, L, g, S.rel, acc, acc2, marg, w, lane, lds_b);
        // W_r = A_r + w (FP64); new TM row: c' = W c, P' = W P, I' = W (x) I + [acc, acc2] -+ margin
        double Wr[4];
        double cpart = 0.0, il = 0.0, ih = 0.0, wabs = 0.0, ske = 0.0;
        double pp[16];
#pragma unroll
        for (int z = 0; z < 16; ++z) pp[z] = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = nrn<T>(gq, i);
          Wr[i] = ((double)w[0][i] + net.skip[(size_t)(valid ? r : 0) * 16 + m]) * (valid ? 1.0 : 0.0);
          cpart += Wr[i] * c[m];
          double a1 = Wr[i] * Ilo[m], a2 = Wr[i] * Ihi[m];
          il += fmin(a1, a2); ih += fmax(a1, a2);
          wabs += fabs(Wr[i]) * Xab[m];
          ske += net.skipE[(size_t)(valid ? r : 0) * 16 + m] * Xab[m];
#pragma unroll
          for (int z = 0; z < 16; ++z) pp[z] += Wr[i] * Pm[m * 16 + z];
        }
        cpart = row_sum(cpart); il = row_sum(il); ih = row_sum(ih); wabs = row_sum(wabs);
        acc = row_sum(acc); acc2 = row_sum(acc2);
        const double seed_mg = sc.margin_on ? net.seedBe[valid ? r : 0] + row_sum(ske) : 0.0;
        double mg = (double)row_sum(marg) * kMargInflate + 0x1p-46 * (wabs + fabs(acc) + fabs(acc2)) + seed_mg;
        double rad = 0.0;
#pragma unroll
        for (int z = 0; z < 16; ++z) {
          double v = row_sum(pp[z]);
          pp[z] = v;
          rad += fabs(v);
        }
        if (valid && lane < 16) {
          nc[r] = cpart;
          nIlo[r] = il + acc - mg;
          nIhi[r] = ih + acc2 + mg;
#pragma unroll
          for (int z = 0; z < 16; ++z) nP[r * 16 + z] = (z < n0) ? pp[z] : 0.0;
          double blo = cpart - rad + nIlo[r], bhi = cpart + rad + nIhi[r];
          if (bx) {
            double* bo = bx + (size_t)(step + 1) * ns * 2;
            bo[r * 2 + 0] = blo;
            bo[r * 2 + 1] = bhi;
          }
          if (!(fabs(blo) < INFINITY) || !(fabs(bhi) < INFINITY)) atomicOr(&S.misc[1], DR_RES_NONFINITE);
        }
        if (lane == 0) sc.rows[(size_t)s * 8 + (L - 1)] += ns;
      }
}

// ---------------------------------------------------------------------------
// Two workgroups per CU for the FP32 reach of 64- and 96-wide networks: the register
// budget of 256 costs a few spills there and doubles the boxes in flight (measured);
// wider or FP64 instances keep one.
template <typename T, int NT> constexpr int reach_waves_per_eu() { return sizeof(T) == 4 && (NT == 4 || NT == 6) ? 2 : 1; }

template <typename T, int NT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(reach_waves_per_eu<T, NT>())))
k_reach_dt(const NetDev* __restrict__ nets, int net_index, ReachArgs ra) {
  extern __shared__ __align__(16) char lds_raw[];
  const NetDev& net = nets[net_index];
  const Scratch& sc = ra.sc;
  const int L = net.L, Hp = net.Hp;
  const int wid_ = threadIdx.x >> 6;
  // dynamic LDS: per-wave chain stages, the subdomain state, then the TM state
  char* stage = lds_raw + (size_t)wid_ * stage_bytes<T, NT>();
  char* lds_base = lds_raw + kWavesPerWG * stage_bytes<T, NT>();
  SubLds<T> S;
  S.carve(lds_base, Hp, NT);
  T* lds_b = (T*)(lds_base + SubLds<T>::bytes(Hp, NT) + kReachExtraLds);
  stage_biases<T, T>(net, lds_b);
  // TM state after the SubLds block: c[16], P[16*16], Ilo[16], Ihi[16], plus the next state
  // (offsets stay on the LDS base pointer so that every access is an LDS access)
  double* tm = (double*)(lds_base + ((SubLds<T>::bytes(Hp, NT) + 64 + 15) & ~(size_t)15));
  double* c = tm;            // 16
  double* Pm = tm + 16;      // 256 (row-major n x n)
  double* Ilo = tm + 272;    // 16
  double* Ihi = tm + 288;    // 16
  double* Xab = tm + 304;    // 16: bound on |x_m| over the TM
  double* nc = tm + 320;     // next state
  double* nP = tm + 336;
  double* nIlo = tm + 592;
  double* nIhi = tm + 608;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, gq = lane >> 4;
  const int cnt = batch_count(sc, net_index);
  const int n0 = net.n[0], ns = net.n_state, H = ra.horizon;

  bool first = true;
  for (;;) {
    int item;
    if (first) {
      first = false;
      item = blockIdx.x;
    } else {
      if (tid == 0) S.misc[0] = (int)gridDim.x + (int)atomicAdd(ra.queue, 1u);
      lds_barrier();
      item = S.misc[0];
      lds_barrier();
    }
    if (item >= cnt) break;
    const int s = subdomain_of(sc, net_index, item);
    double* bx = ra.boxes + (size_t)s * (H + 1) * ns * 2;
    double* tb = ra.tape ? ra.tape + (size_t)s * reach_tape_doubles(H, Hp) : nullptr;
    // TM normalisation of the state box: c = centre, P = diag(radius), I = [0, 0]; the
    // exogenous inputs (network inputs ns..n0-1) enter each step as points
    if (tid < 16) {
      double cc = tid < ns ? ra.batch.xc[(size_t)s * n0 + tid] : 0.0;
      double rr = tid < ns ? ra.batch.xr[(size_t)s * n0 + tid] : 0.0;
      c[tid] = cc; Ilo[tid] = 0.0; Ihi[tid] = 0.0;
      if (tid < ns) { bx[tid * 2 + 0] = cc - rr; bx[tid * 2 + 1] = cc + rr; }
    }
    for (int e = tid; e < 256; e += kWG) {
      int a = e >> 4, b = e & 15;
      Pm[e] = (a == b && a < ns) ? ra.batch.xr[(size_t)s * n0 + a] : 0.0;
    }
    for (int p = tid; p < Hp; p += kWG) S.slot[p] = -1;
    if (tid == 0) S.misc[1] = 0;
    if (tid < 8) sc.rows[(size_t)s * 8 + tid] = 0;
    lds_barrier();
    for (int step = 0; step < H; ++step) {
      // |x_m| bound over the TM, and the input-centre/radius for the layer-1 bounds
      if (tid < 16) {
        if (tid >= ns && tid < n0) c[tid] = ra.u[((size_t)s * H + step) * (n0 - ns) + (tid - ns)];
        double a = fabs(c[tid]) + fmax(fabs(Ilo[tid]), fabs(Ihi[tid]));
        for (int z = 0; z < n0; ++z) a += fabs(Pm[tid * 16 + z]);
        Xab[tid] = tid < n0 ? a : 0.0;
        S.xc[tid] = 0.0; S.xr[tid] = 0.0;
      }
      lds_barrier();
      if (tb) {
        double* tt = tb + reach_tape_tm(step);
        for (int e = tid; e < kTmDoubles; e += kWG) tt[e] = tm[e];
      }
      tm_crown_step<T, NT>(net, sc, S, stage, lds_b, tm, tb, step, H, s, bx);
      lds_barrier();
      if (tid < 16) {
        c[tid] = tid < ns ? nc[tid] : 0.0;
        Ilo[tid] = tid < ns ? nIlo[tid] : 0.0;
        Ihi[tid] = tid < ns ? nIhi[tid] : 0.0;
      }
      for (int e = tid; e < 256; e += kWG) Pm[e] = ((e >> 4) < ns) ? nP[e] : 0.0;
      lds_barrier();
    }
    if (tb) {
      double* tt = tb + reach_tape_tm(H);
      for (int e = tid; e < kTmDoubles; e += kWG) tt[e] = tm[e];
    }
    if (tid == 0) {
      sc.st[s] = (uint32_t)S.misc[1];
      if (ra.status) ra.status[s] = (uint32_t)S.misc[1];
      if (sc.st_out) sc.st_out[s] = (uint32_t)S.misc[1];
    }
    lds_barrier();
  }
}

}  // namespace dr
