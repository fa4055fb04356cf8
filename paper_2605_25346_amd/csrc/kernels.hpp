// Device building blocks of the bound-propagation kernels (gfx950, wave64).
//
// Data layout of a chain of backward bound propagation on one wavefront:
//   The wave owns an N-tile of 16 rows (row multipliers Lambda).  The product
//   Lambda . W_k is computed transposed, D^T = W_k^T Lambda^T, on the 16x16x4 MFMA:
//   the A operand is a 16x4 slice of W (pre-swizzled in global memory so that a
//   lane fetches its four A values of one K-tile with one vector load) and the B
//   operand is Lambda^T.  The D layout of one product is exactly the B layout of
//   the next one up to a fixed permutation of the summation index, so a whole
//   chain stays in registers: register cur[t][i] of lane l holds row (l % 16),
//   neuron 16 t + nrn(l / 16, i) of the current layer.
//   The permutation differs between the f32 and f64 MFMA output layouts (verified
//   on the device): f32 D[4 g + i][n], f64 D[4 i + g][n] for lane group g.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace dr {

constexpr int kMaxL = 8;         // affine layers per network
constexpr int kMaxNets = 8;
constexpr int kWG = 256;         // threads per workgroup (4 waves)
constexpr int kWavesPerWG = kWG / 64;

template <typename T> struct Vec4T;
template <> struct Vec4T<float> { typedef float v __attribute__((ext_vector_type(4))); };
template <> struct Vec4T<double> { typedef double v __attribute__((ext_vector_type(4))); };
template <typename T> using V4 = typename Vec4T<T>::v;

__device__ __forceinline__ V4<float> mfma16(float a, float b, V4<float> c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ V4<double> mfma16(double a, double b, V4<double> c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Neuron (within a 16-tile) held by lane group g in accumulator register i.
template <typename T> __host__ __device__ constexpr int nrn(int g, int i) {
  return sizeof(T) == 4 ? 4 * g + i : 4 * i + g;
}
// Position (within a 16-tile, permuted storage) of neuron c: inverse of nrn.
template <typename T> __host__ __device__ constexpr int pos_of(int c) {
  return sizeof(T) == 4 ? c : (c & 3) * 4 + (c >> 2);
}

// Unit roundoff of the chain arithmetic.
template <typename T> __host__ __device__ constexpr double unit_round() {
  return sizeof(T) == 4 ? 0x1p-24 : 0x1p-53;
}
// gamma_n = n u / (1 - n u) (Higham, dot-product error bound, any summation order).
template <typename T> __host__ __device__ inline double gamma_n(int n) {
  double nu = n * unit_round<T>();
  return nu / (1.0 - nu);
}

// Smallest float >= f (for finite f); used to round margins and intercepts outward.
__device__ __forceinline__ float next_up(float f) {
  if (!(f < __builtin_huge_valf())) return f;
  if (f == 0.0f) return 0x1p-149f;
  unsigned u = __float_as_uint(f);
  return __uint_as_float(f > 0.0f ? u + 1u : u - 1u);
}
__device__ __forceinline__ float round_up_to(float*, double x) {
  float f = (float)x;
  if ((double)f < x) f = next_up(f);
  return f;
}
__device__ __forceinline__ double round_up_to(double*, double x) { return x; }
template <typename T> __device__ __forceinline__ T rup(double x) { return round_up_to((T*)nullptr, x); }

// Per-network description in device memory (all arrays owned by the context,
// every dimension padded to a multiple of 16 with zeros).
struct NetDev {
  int L;                     // affine layers
  int NT;                    // 16-tiles of every hidden layer (hidden widths padded to 16 NT)
  int n[kMaxL + 1];          // true widths n_0..n_L
  int H;                     // true hidden count
  int Hp;                    // padded hidden count = (L - 1) * 16 NT
  int hoff[kMaxL];           // natural offset of hidden layer k (index k-1) in [0, H)
  const void* Wn[kMaxL];     // natural row-major, padded rows/cols: rows np_k, cols np_{k-1}
  const void* bn[kMaxL];     // padded biases
  const void* Wf[kMaxL];     // forward swizzle: A[m][kk] = W_k[kk][m]
  const void* Wa[kMaxL];     // adjoint swizzle: A[m][kk] = W_k[m][kk]
  int np[kMaxL + 1];         // padded widths (hidden: 16 NT; input/output: multiple of 16)
  const double* seedW;       // R x np_{L-1}: g = a_L W_L of every final row (FP64)
  const double* seedB;       // R: a_L . b_L
  const double* seedA;       // R x np_L: a_L, the multipliers of every final row on the network output
  const double* skip;        // R x 16: (+-c) A for the closed loop, zeros otherwise
  // a priori bounds of the FP64 rounding in the seeds (Higham's dot-product bound),
  // covered by the rounding margin of every final row: seedWe R x np_{L-1} bounds
  // |g - a W_L| including the error of a = c B itself (so it also covers the error of
  // a . y through y = W_L h + b_L), seedBe R the same for a . b_L, skipE R x 16 the
  // error of (+-c) A per input (times a bound on |x|)
  const double* seedWe;
  const double* seedBe;
  const double* skipE;
  // the seeds g in the chain type (R x np_{L-1}) and, per entry, the margin coefficient
  // of the seed (its rounding to the chain type plus seedWe, rounded up), so a final
  // row's seed margin is sum_m seedM[m] max(u_m, 0) over the last hidden layer
  const void* seedT;
  const void* seedM;
  const double* A;           // n_state x n_0 (closed loop) or null
  // closed loop: forward-swizzled M = B W_L (rows: the n_state state indices padded to
  // 16, columns: h_{L-1}) and A (16 x 16, columns: the network input v), in the chain
  // type, for carrying rows on x' back through a step (unrolled-loop CROWN); else null
  const void* jM;
  const void* jA;
  int n_state;
  int q;                     // spec directions
  int R;                     // 2q rows
};

// Scratch and outputs shared by the kernels of one context.
struct Scratch {
  double* bl;                // S x Hp_max lower pre-activation bounds (natural order)
  double* bu;                // S x Hp_max upper
  void* rel;                 // S x Hp_max x 4 T relaxation (lo, up, t, mu), permuted order
  int* slot;                 // S x Hp_max split slot (-1 or idx << 1 | positive), permuted
  uint32_t* st;              // S status bits
  int* rows;                 // S x 8 chain rows
  double* margin;            // S x 16 margin of final rows
  int* order;                // S subdomains sorted by network
  int* net_cnt;              // kMaxNets counts
  int* net_off;              // kMaxNets offsets into order
  int Hp_max;
  int margin_on;             // 1: rigorous rounding margins, 0: off (diagnostics)
  int direct;                // 1: single network, subdomain s = work item (no sorted order)
  int n_sub;                 // batch size of the current call
  uint32_t* st_out;          // caller's status array (nullable), written with st
  int fuse;                  // 1: k_bound_init also runs the plain spec rows into fin
  double* fin;               // S x 16 x 17: per final row, input coefficients (16) and offset
};

// Extra LDS of k_reach_dt after its subdomain state: alignment slack and the Taylor
// model state (current and next: 2 x (16 + 256 + 16 + 16) doubles, plus |x| bounds).
constexpr size_t kReachExtraLds = 64 + 16 + 640 * sizeof(double);

// Work items of network `net_index` in the current batch and the subdomain of an item.
__device__ __forceinline__ int batch_count(const Scratch& sc, int net_index) {
  return sc.direct ? sc.n_sub : sc.net_cnt[net_index];
}
__device__ __forceinline__ int subdomain_of(const Scratch& sc, int net_index, int item) {
  return sc.direct ? item : sc.order[sc.net_off[net_index] + item];
}

struct BatchDev {
  int n_sub;
  const int* net_id;
  const double* xc;
  const double* xr;
  const int* sptr;
  const uint32_t* spk;
};

// ---------------------------------------------------------------------------
// Work queue of a persistent launch: a counter of handed-out items, cleared by a
// one-block kernel on the same stream before every launch (k_reset_queue).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_fetch(unsigned* q) {
  int lane = threadIdx.x & 63;
  int v = 0;
  if (lane == 0) v = (int)atomicAdd(q, 1u);
  return __shfl(v, 0);
}
// Work item of a persistent worker: its first item is its own index (no atomic at
// launch, when every worker would contend for the counter); later ones come from the
// queue, offset by the number of workers.  Called by a whole wavefront.
__device__ __forceinline__ int next_item(unsigned* q, bool& first, int worker, int n_workers) {
  if (first) {
    first = false;
    return worker;
  }
  return n_workers + wave_fetch(q);
}

// Sum over the four lane groups holding the same row (lanes n, n+16, n+32, n+48):
// (v + v[l ^ 16]) then the same with l ^ 32, exchanged with v_permlane16_swap and
// v_permlane32_swap (VALU lane swaps, no LDS round trip).  With x = y = v, the two
// results of a swap are, per lane, its own value and its partner's (in an order that
// depends on the lane), so their sum is v + v[l ^ 16] (resp. l ^ 32) on every lane,
// bit-identical on both partners (addition is commutative).
__device__ __forceinline__ float xor_pair_sum16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor_pair_sum32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor_pair_sum16(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
  const double d0 = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
  const double d1 = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
  return d0 + d1;
}
__device__ __forceinline__ double xor_pair_sum32(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
  const double d0 = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
  const double d1 = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
  return d0 + d1;
}
template <typename S> __device__ __forceinline__ S row_sum(S v) {
  return xor_pair_sum32(xor_pair_sum16(v));
}

// ---------------------------------------------------------------------------
// Products on the matrix cores.
// ---------------------------------------------------------------------------
// nxt[mt] = sum_kt A(mt, kt) cur[kt] for MT x KT tiles (compile-time shape: the
// unrolled body is straight-line so loads can be hoisted ahead of the MFMAs).
// Global-memory views: loads and stores through these pointers are emitted as
// global (not flat) memory instructions with a scalar base where the base is uniform.
template <typename T> using gconst = const T __attribute__((address_space(1)))*;
template <typename T> using gmut = T __attribute__((address_space(1)))*;
template <typename T> __device__ __forceinline__ gconst<T> as_global(const T* p) { return (gconst<T>)p; }
template <typename T> __device__ __forceinline__ gmut<T> as_global_mut(T* p) { return (gmut<T>)p; }

// A pointer that is the same for every lane, moved to scalar registers so that
// loads through it use a scalar base and 32-bit lane offsets.
template <typename P> __device__ __forceinline__ P uniform_ptr(P p) {
  uint64_t v = (uint64_t)p;
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (P)(((uint64_t)hi << 32) | lo);
}

template <typename T> using lconst = const T __attribute__((address_space(3)))*;
template <typename T> using lmut = T __attribute__((address_space(3)))*;

// The B operand of a chain product (the row multipliers of the current layer in the
// lane layout described above) lives either in registers or, for wide layers, in a
// wave-private LDS area (lane l only touches its own slots, so no synchronisation is
// needed); the LDS form halves the registers a chain needs.
template <typename T, int NT>
struct RegStage {
  T v[NT][4];
  __device__ __forceinline__ T get(int t, int i) const { return v[t][i]; }
  __device__ __forceinline__ void set(int t, int i, T x) { v[t][i] = x; }
};
template <typename T, int NT>
struct LdsStage {
  lmut<T> p;   // NT * 4 * 64 elements, index (t * 4 + i) * 64 + lane
  int lane;
  __device__ __forceinline__ T get(int t, int i) const { return p[(t * 4 + i) * 64 + lane]; }
  __device__ __forceinline__ void set(int t, int i, T x) { p[(t * 4 + i) * 64 + lane] = x; }
};
// Wide chains keep their state in LDS: FP32 from 128 neurons, FP64 at 128 neurons,
// and FP64 at 256 neurons (32 KiB per wavefront) only in kernels without per-subdomain
// LDS state (`roomy`: the final-row and dual-ascent kernel).
__host__ __device__ constexpr bool stage_in_lds_rt(int tsz, int NT, bool roomy) {
  return tsz == 8 ? (NT == 8 || (roomy && NT == 16)) : NT >= 8;
}
__host__ __device__ constexpr size_t stage_bytes_rt(int tsz, int NT, bool roomy) {
  return stage_in_lds_rt(tsz, NT, roomy) ? (size_t)NT * 4 * 64 * tsz : 0;
}
template <typename T, int NT, bool ROOMY = false> __host__ __device__ constexpr bool stage_in_lds() {
  return stage_in_lds_rt((int)sizeof(T), NT, ROOMY);
}
template <typename T, int NT, bool ROOMY = false> __host__ __device__ constexpr size_t stage_bytes() {
  return stage_bytes_rt((int)sizeof(T), NT, ROOMY);
}
// The stage of one wavefront; `lds` is its private area (unused for register stages).
template <typename T, int NT, bool ROOMY = false> __device__ __forceinline__ auto make_stage(char* lds, int lane) {
  if constexpr (stage_in_lds<T, NT, ROOMY>()) return LdsStage<T, NT>{(lmut<T>)lds, lane};
  else return RegStage<T, NT>{};
}

// Scheduling fence between the unrolled tiles of a chain step: the loads of the next
// tile stay behind the current tile's arithmetic, which bounds register pressure for
// wide layers; narrow layers (NT tiles of at most kFenceFreeBytes bytes per lane)
// let the compiler overlap the tiles.
constexpr int kFenceFreeBytes = 0;
template <typename T, int NT> __device__ __forceinline__ void tile_fence() {
  if constexpr (NT * (int)sizeof(T) > kFenceFreeBytes) __builtin_amdgcn_sched_barrier(0);
}

// nxt[mt] = sum_kt A(mt, kt) B[kt] for MT x KT tiles, summation-tile outer: the MT
// accumulations of one K-tile are independent (no back-to-back dependent MFMAs) and
// the K-tile's B values are read once.  P: gconst<V4<T>> (swizzled weights in global
// memory) or lconst<V4<T>> (an LDS copy); B: RegStage or LdsStage (or a plain array
// through RegArr).
// Weights read from global memory (not from an LDS copy) are software-pipelined: the
// A tiles of K-tile kt + 1 are loaded before the products of K-tile kt, when they take
// at most kPrefetchBytes per lane (FP32 up to 256 neurons, FP64 up to 64).
template <typename P> struct lds_pointer { static constexpr bool value = false; };
template <typename U> struct lds_pointer<const U __attribute__((address_space(3)))*> {
  static constexpr bool value = true;
};
constexpr int kPrefetchBytes = 256;
// FP32 layers of 256 neurons: M-tile groups and prefetch distance (in K-tile steps).
// Measured on the 256-wide reach, bound and ascent kernels against the whole-tile
// double buffer (1 group): any split of 2 or 4 groups with distance 1-4 is 20-25%
// faster on the reach (fewer live registers, fewer spills); 4 groups, distance 2 best.
constexpr int kWideSplit = 4;
constexpr int kWideDist = 2;
// The same for FP32 layers of 128 neurons (2 groups, distance 2: 5% faster ascent than
// the whole-tile double buffer) and of 64 / 96 neurons (2 groups, distance 2: 2-4% faster
// candidate reach and mixed-batch kernels).
constexpr int kMidSplit = 2;
constexpr int kMidDist = 2;
constexpr int kNarrowSplit = 2;
constexpr int kNarrowDist = 2;
template <typename T> __host__ __device__ constexpr int prefetch_bytes() { return sizeof(T) == 4 ? kPrefetchBytes : 128; }
template <typename T, int MT, int KT, typename P, typename B>
__device__ __forceinline__ void gemm_k(P Wsw, const B& cur, T (&nxt)[MT][4], int lane) {
  V4<T> acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = V4<T>{0, 0, 0, 0};
  constexpr bool PF = !lds_pointer<P>::value && KT > 1 && MT * 4 * (int)sizeof(T) <= prefetch_bytes<T>();
  constexpr int SPLIT = MT >= 16 ? kWideSplit : (MT >= 8 ? kMidSplit : kNarrowSplit);
  constexpr int DIST = MT >= 16 ? kWideDist : (MT >= 8 ? kMidDist : kNarrowDist);
  constexpr int MH = MT / SPLIT;
  constexpr bool PFW = PF && sizeof(T) == 4 && MT >= 4 && MT % SPLIT == 0 && (SPLIT > 1 || DIST > 1);
  if constexpr (PFW) {
    // Wide layers: the M tiles are processed in SPLIT groups, each over all K-tiles, as
    // one stream of (group, K-tile) steps whose A tiles are loaded DIST steps ahead
    // into a ring of DIST + 1 slots (a group's A tiles are MH V4 per lane, so the ring
    // costs no more registers than a whole-tile double buffer while covering DIST
    // steps of MFMA work).  The B values are re-read from the stage once per group.
    constexpr int NS = SPLIT * KT, W = DIST + 1;
    V4<T> ring[W][MH];
#pragma unroll
    for (int s = 0; s < DIST; ++s)
      if (s < NS) {
#pragma unroll
        for (int m = 0; m < MH; ++m) ring[s][m] = Wsw[(((s / KT) * MH + m) * KT + s % KT) * 64 + lane];
      }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int h = s / KT, kt = s % KT;
      if (s + DIST < NS) {
        const int s2 = s + DIST;
#pragma unroll
        for (int m = 0; m < MH; ++m) ring[s2 % W][m] = Wsw[(((s2 / KT) * MH + m) * KT + s2 % KT) * 64 + lane];
      }
      const T b0 = cur.get(kt, 0), b1 = cur.get(kt, 1), b2 = cur.get(kt, 2), b3 = cur.get(kt, 3);
#pragma unroll
      for (int m = 0; m < MH; ++m) {
        const int mt = h * MH + m;
        acc[mt] = mfma16(ring[s % W][m][0], b0, acc[mt]);
        acc[mt] = mfma16(ring[s % W][m][1], b1, acc[mt]);
        acc[mt] = mfma16(ring[s % W][m][2], b2, acc[mt]);
        acc[mt] = mfma16(ring[s % W][m][3], b3, acc[mt]);
      }
      tile_fence<T, MT>();
    }
  } else if constexpr (PF) {
    V4<T> a_cur[MT], a_nxt[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) a_cur[mt] = Wsw[(mt * KT) * 64 + lane];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (kt + 1 < KT) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a_nxt[mt] = Wsw[(mt * KT + kt + 1) * 64 + lane];
      }
      const T b0 = cur.get(kt, 0), b1 = cur.get(kt, 1), b2 = cur.get(kt, 2), b3 = cur.get(kt, 3);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        acc[mt] = mfma16(a_cur[mt][0], b0, acc[mt]);
        acc[mt] = mfma16(a_cur[mt][1], b1, acc[mt]);
        acc[mt] = mfma16(a_cur[mt][2], b2, acc[mt]);
        acc[mt] = mfma16(a_cur[mt][3], b3, acc[mt]);
      }
      tile_fence<T, MT>();
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) a_cur[mt] = a_nxt[mt];
    }
  } else {
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const T b0 = cur.get(kt, 0), b1 = cur.get(kt, 1), b2 = cur.get(kt, 2), b3 = cur.get(kt, 3);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        V4<T> a = Wsw[(mt * KT + kt) * 64 + lane];
        acc[mt] = mfma16(a[0], b0, acc[mt]);
        acc[mt] = mfma16(a[1], b1, acc[mt]);
        acc[mt] = mfma16(a[2], b2, acc[mt]);
        acc[mt] = mfma16(a[3], b3, acc[mt]);
      }
      tile_fence<T, MT>();
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    nxt[mt][0] = acc[mt][0]; nxt[mt][1] = acc[mt][1]; nxt[mt][2] = acc[mt][2]; nxt[mt][3] = acc[mt][3];
  }
}

// A register array viewed as a stage.
template <typename T, int NT>
struct RegArr {
  const T (&v)[NT][4];
  __device__ __forceinline__ T get(int t, int i) const { return v[t][i]; }
};

template <typename T, int MT, int KT, typename P>
__device__ __forceinline__ void gemm_tiles_p(P Wsw, const T (&cur)[KT][4], T (&nxt)[MT][4], int lane) {
  gemm_k<T, MT, KT>(Wsw, RegArr<T, KT>{cur}, nxt, lane);
}

template <typename T, int MT, int KT>
__device__ __forceinline__ void gemm_tiles(const V4<T>* __restrict__ Wsw_, const T (&cur)[KT][4],
                                           T (&nxt)[MT][4], int lane) {
  gemm_tiles_p<T, MT, KT>(as_global(uniform_ptr(Wsw_)), cur, nxt, lane);
}


// Forward-swizzled weights of hidden-side layers 1..L-1 staged in LDS (small networks):
// V4 offset of layer k (1-based) inside the staged block.
__host__ __device__ inline int lds_w_offset(int k, int NT) {
  return k <= 1 ? 0 : NT * 64 + (k - 2) * NT * NT * 64;
}
__host__ __device__ inline int lds_w_count(int L, int NT) { return lds_w_offset(L, NT); }


// ---------------------------------------------------------------------------
// Per-subdomain shared state of k_bound_init / k_reach_dt (dynamic LDS).
// ---------------------------------------------------------------------------
template <typename T>
struct SubLds {
  V4<T>* rel;     // Hp, permuted
  double* l;      // Hp natural
  double* u;      // Hp natural
  int* slot;      // Hp permuted
  double* ibl;    // 16 NT
  double* ibu;
  double* v;
  double* hc;     // 16 NT: centre of relu(h) of the previous layer
  double* hr;     // 16 NT: radius
  int* U;         // 16 NT
  double* xc;     // 16
  double* xr;     // 16
  int* misc;      // 8 ints: [0] item, [1] flags, [2..5] wave counts
  __host__ __device__ static size_t bytes(int Hp, int NT) {
    size_t b = (size_t)Hp * (sizeof(V4<T>) + 2 * sizeof(double) + sizeof(int)) +
               (size_t)16 * NT * (5 * sizeof(double) + sizeof(int)) + 32 * sizeof(double) + 8 * sizeof(int);
    return (b + 63) & ~(size_t)63;
  }
  __device__ void carve(char* base, int Hp, int NT) {
    rel = (V4<T>*)base; base += (size_t)Hp * sizeof(V4<T>);
    l = (double*)base; base += (size_t)Hp * sizeof(double);
    u = (double*)base; base += (size_t)Hp * sizeof(double);
    ibl = (double*)base; base += (size_t)16 * NT * sizeof(double);
    ibu = (double*)base; base += (size_t)16 * NT * sizeof(double);
    v = (double*)base; base += (size_t)16 * NT * sizeof(double);
    hc = (double*)base; base += (size_t)16 * NT * sizeof(double);
    hr = (double*)base; base += (size_t)16 * NT * sizeof(double);
    xc = (double*)base; base += 16 * sizeof(double);
    xr = (double*)base; base += 16 * sizeof(double);
    slot = (int*)base; base += (size_t)Hp * sizeof(int);
    U = (int*)base; base += (size_t)16 * NT * sizeof(int);
    misc = (int*)base;
  }
};

struct FinalArgs {
  BatchDev batch;
  Scratch sc;
  unsigned* queue;
  // a5 outputs
  double* lam_lo; double* acc_lo; double* lam_hi; double* acc_hi;
  // a7
  int iters; float lr; int init_duals;
  float* alpha; float* beta; double* lb; double* ub; float* galpha; float* gbeta;
  uint32_t* status;
  void* tape;               // per-wave tape of g values (a7)
  int H_max;                // alpha row stride
  int max_splits;           // beta row stride
  int q;
  // parameter gradient (k_final with PGRAD): row weights, the column-major per-row
  // tapes of multipliers a^(k) (weighted) and adjoints e^(k), input gradients
  const double* g_lb; const double* g_ub;
  void* ptape; size_t rows_pad;
  double* dxc; double* dxr;
};

// LDS copy of a dual-ascent work item's relaxation and split slots (P subdomains):
// they do not change over the iterations.
template <typename T> __host__ __device__ constexpr size_t item_cache_bytes(int P, int Hp) {
  return ((size_t)P * Hp * (sizeof(V4<T>) + sizeof(int)) + 15) & ~(size_t)15;
}

// Column offsets of the parameter-gradient tapes (rows_pad entries per column): the
// multipliers a^(k) of layers k = 1..L, then the adjoints e^(k) of layers k = 0..L-1
// (e^(0) = xc - sgn(w) xr); every hidden layer has 16 NT columns, the input 16.
__host__ __device__ inline int ptape_col_a(int k, int NT) { return (k - 1) * 16 * NT; }
__host__ __device__ inline int ptape_col_g(int k, int L, int NT, int npL) {
  return (L - 1) * 16 * NT + npL + (k == 0 ? 0 : 16 + (k - 1) * 16 * NT);
}

struct ReachArgs {
  BatchDev batch;
  Scratch sc;
  unsigned* queue;
  int horizon;
  double* boxes;            // S x (horizon + 1) x n_state x 2
  uint32_t* status;
  const double* u;          // S x horizon x (n_0 - n_state) exogenous inputs, or null
  double* tape;             // null, or the record of the reach for its gradient (reach_tape_* layout)
};

// Record of one box's stepwise reach for the reverse pass (FP64): the Taylor model
// entering every step and the final one (c 16, P 16 x 16, I_lo 16, I_hi 16 per step,
// t = 0..H), then per step the final bounds l, u of every hidden neuron and the IBP
// bounds of layers >= 2 (layer 1: its exact bounds again), natural order.
constexpr int kTmDoubles = 304;
__host__ __device__ inline size_t reach_tape_tm(int t) { return (size_t)t * kTmDoubles; }
__host__ __device__ inline size_t reach_tape_bounds(int t, int H, int Hp) {
  return (size_t)(H + 1) * kTmDoubles + (size_t)t * 4 * Hp;
}
__host__ __device__ inline size_t reach_tape_doubles(int H, int Hp) { return reach_tape_bounds(H, H, Hp); }


// Arguments and per-box LDS state of k_reach_joint (CROWN through the unrolled loop).
struct JointArgs {
  BatchDev batch;
  Scratch sc;
  int horizon;
  double* boxes;            // S x (horizon + 1) x n_state x 2
  int* rows;                // S x horizon x 8 (nullable): CROWN rows per hidden layer and state rows
  uint32_t* status;
  const double* u;          // S x horizon x (n_0 - n_state) exogenous inputs, or null
};

// Per-box LDS state of k_reach_joint.
template <typename T>
struct JointLds {
  V4<T>* rel;     // H x Hp relaxation (lo, up, t, mu) of every step, permuted order
  double* l;      // Hp natural: bounds of the current step
  double* u;
  double* ibl;    // 16 NT: IBP bounds of the current layer
  double* ibu;
  double* v;      // 16 NT: |W_k| H_{k-1} of the current layer (margin coefficients)
  double* hc;     // 16 NT: centre/radius of relu of the previous layer
  double* hr;
  double* box;    // 6 x 16: initial centre, radius; current state box lo, hi; v box centre, radius
  double* uv;     // H x 16: exogenous inputs at their input positions (zero elsewhere)
  double* vab;    // H x 16: bound on |v_s|
  T* mux;         // H x 16: margin coefficient of a row multiplier on x_{s+1} at the step boundary
  T* bias;        // Hp: hidden biases in the chain type
  int* U;         // 16 NT
  int* misc;      // 8: [1] status flags, [2..] wave counts of the compaction
  __host__ __device__ static size_t r16(size_t n) { return (n + 15) & ~(size_t)15; }
  __host__ __device__ static size_t bytes(int H, int Hp, int NT) {
    const size_t n16 = (size_t)16 * NT;
    return r16((size_t)H * Hp * sizeof(V4<T>)) + 2 * r16((size_t)Hp * sizeof(double)) +
           5 * r16(n16 * sizeof(double)) + r16(96 * sizeof(double)) + 2 * r16((size_t)H * 16 * sizeof(double)) +
           r16((size_t)H * 16 * sizeof(T)) + r16((size_t)Hp * sizeof(T)) + r16(n16 * sizeof(int)) +
           r16(8 * sizeof(int));
  }
  __device__ void carve(char* base, int H, int Hp, int NT) {
    auto take = [&](size_t n) { char* p = base; base += r16(n); return p; };
    rel = (V4<T>*)take((size_t)H * Hp * sizeof(V4<T>));
    l = (double*)take((size_t)Hp * sizeof(double));
    u = (double*)take((size_t)Hp * sizeof(double));
    ibl = (double*)take((size_t)16 * NT * sizeof(double));
    ibu = (double*)take((size_t)16 * NT * sizeof(double));
    v = (double*)take((size_t)16 * NT * sizeof(double));
    hc = (double*)take((size_t)16 * NT * sizeof(double));
    hr = (double*)take((size_t)16 * NT * sizeof(double));
    box = (double*)take(96 * sizeof(double));
    uv = (double*)take((size_t)H * 16 * sizeof(double));
    vab = (double*)take((size_t)H * 16 * sizeof(double));
    mux = (T*)take((size_t)H * 16 * sizeof(T));
    bias = (T*)take((size_t)Hp * sizeof(T));
    U = (int*)take((size_t)16 * NT * sizeof(int));
    misc = (int*)take(8 * sizeof(int));
  }
};

// Row-tile records of one step of the reverse reach pass (chain type, per workgroup): slot 0
// holds the output rows, slot 1 + (k - 2) NT + tile the CROWN rows of hidden layer k.  A slot
// holds, in the lane-major layout of a chain state (entry (row, 16 t + nrn(g, i)) of a
// 16-row tile at (t 4 + i) 64 + 16 g + row): the multipliers g over h_j of every relaxed
// layer j = 1 .. L-1 (NT tiles each), the cotangent over the input (one tile) and over
// h_k for k = 1 .. L-1 (NT tiles each), then the rows' offset cotangents (16, padded).
__host__ __device__ constexpr int rg_slots(int L, int NT) { return 1 + (L - 2) * NT; }
__host__ __device__ constexpr size_t rg_slot_g(int j, int NT) { return (size_t)(j - 1) * NT * 256; }
__host__ __device__ constexpr size_t rg_slot_dg(int k, int L, int NT) {
  return (size_t)(L - 1) * NT * 256 + (k == 0 ? 0 : 256 + (size_t)(k - 1) * NT * 256);
}
__host__ __device__ constexpr size_t rg_slot_rho(int L, int NT) { return (size_t)2 * (L - 1) * NT * 256 + 256; }
__host__ __device__ constexpr size_t rg_slot_elems(int L, int NT) { return rg_slot_rho(L, NT) + 64; }
constexpr int kRgMaxSlots = 128;

// Arguments and per-box LDS state of k_reach_grad (reverse pass through the stepwise reach).
struct ReachGradArgs {
  BatchDev batch;
  Scratch sc;
  int horizon;
  const double* tape;       // per box reach_tape_doubles(H, Hp) doubles
  const double* gV;         // S: dJ/dV_s
  void* gtape;              // per workgroup: rg_slots x rg_slot_elems chain-type values (row-tile records of a step)
  double* du;               // S x H x (n_0 - n_state) or null
  double* dxc;              // S x n_state or null
  double* dxr;              // S x n_state or null
  double* dA;               // n_state x n_0 (summed over the batch, atomically) or null
  double* dB;               // n_state x n_L or null
  // weight and bias gradients: one region per workgroup (chain type, summed later in a
  // fixed order); layer k at woff[k-1], np_k rows of np_{k-1} + 1 entries (the last is
  // the bias); null when not asked for
  void* wreg;
  size_t wreg_stride;       // chain-type elements per workgroup region
  size_t woff[kMaxL];
  int wacc_lds;             // 1: the region is accumulated in LDS and stored once per workgroup
};

// Per-box LDS state of k_reach_grad.
template <typename T>
struct GradLds {
  V4<T>* rel;     // Hp relaxation of the current step (permuted order)
  double* l;      // Hp natural: bounds of the current step
  double* u;
  double* ibl;
  double* ibu;
  double* ds;     // Hp: cotangents of the chord slopes and intercepts of the current step
  double* dt;
  double* dl;     // Hp: cotangents of the bounds of the current step
  double* du;
  double* tm;     // 304: model entering the step (c, P, I_lo, I_hi)
  double* dO;     // 304: cotangent of the model leaving the step
  double* dI;     // 304: cotangent of the model entering the step
  double* Wr;     // 256: rows W_r = A_r + w_r of the output (r x v)
  double* dWr;    // 256: their cotangents (Wr, dWr contiguous: also the partial sums of the
                  //      interval bounds in reverse)
  double* rowc;   // 16 x 2: per-row cotangents of the offsets (output rows)
  signed char* wps;   // 16 NT x 16: signs of (W_1 P)_jz for layer 1 in reverse
  T* ob;          // per wave 2 x 16 x 16: blocks of an outer product over a row tile (weight gradient)
  double* orho;   // per wave 16: the rows' offset cotangents
  T* bias;        // Hp: hidden biases in the chain type
  int* U;         // 16 NT
  int* misc;      // 8
  int* sused;     // kRgMaxSlots: the step's row-tile records that were written
  T* wacc;        // the workgroup's weight-gradient accumulator (when it fits in LDS)
  __host__ __device__ static size_t r16(size_t n) { return (n + 15) & ~(size_t)15; }
  __host__ __device__ static size_t bytes(int Hp, int NT) {
    const size_t n16 = (size_t)16 * NT;
    return r16((size_t)Hp * sizeof(V4<T>)) + 8 * r16((size_t)Hp * sizeof(double)) + 3 * r16(304 * sizeof(double)) +
           2 * r16(256 * sizeof(double)) + r16(32 * sizeof(double)) + r16(n16 * 16) +
           r16(kWavesPerWG * 512 * sizeof(T)) + r16(kWavesPerWG * 16 * sizeof(double)) + r16((size_t)Hp * sizeof(T)) + r16(n16 * sizeof(int)) + r16(8 * sizeof(int)) +
           r16(kRgMaxSlots * sizeof(int));
  }
  __device__ void carve(char* base, int Hp, int NT) {
    auto take = [&](size_t n) { char* p = base; base += r16(n); return p; };
    const size_t n16 = (size_t)16 * NT;
    rel = (V4<T>*)take((size_t)Hp * sizeof(V4<T>));
    l = (double*)take((size_t)Hp * sizeof(double));
    u = (double*)take((size_t)Hp * sizeof(double));
    ibl = (double*)take((size_t)Hp * sizeof(double));
    ibu = (double*)take((size_t)Hp * sizeof(double));
    ds = (double*)take((size_t)Hp * sizeof(double));
    dt = (double*)take((size_t)Hp * sizeof(double));
    dl = (double*)take((size_t)Hp * sizeof(double));
    du = (double*)take((size_t)Hp * sizeof(double));
    tm = (double*)take(304 * sizeof(double));
    dO = (double*)take(304 * sizeof(double));
    dI = (double*)take(304 * sizeof(double));
    Wr = (double*)take(256 * sizeof(double));
    dWr = (double*)take(256 * sizeof(double));
    rowc = (double*)take(32 * sizeof(double));
    wps = (signed char*)take(n16 * 16);
    ob = (T*)take(kWavesPerWG * 512 * sizeof(T));
    orho = (double*)take(kWavesPerWG * 16 * sizeof(double));
    bias = (T*)take((size_t)Hp * sizeof(T));
    U = (int*)take(n16 * sizeof(int));
    misc = (int*)take(8 * sizeof(int));
    sused = (int*)take(kRgMaxSlots * sizeof(int));
    wacc = (T*)base;    // beyond bytes(): present when the launch added its size
  }
};

}  // namespace dr
