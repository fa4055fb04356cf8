// Host side of the C-ABI (libdiffreach.so): validation, context set-up, launches.
// The chain kernels are reached through the instance handles of instances.h (their own
// translation units); the small kernels of aux_kernels.hpp are compiled in here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "aux_kernels.hpp"
#include "diffreach.h"
#include "instances.h"

using dr::kMaxL;
using dr::kMaxNets;
using dr::kWG;

namespace {
thread_local std::string g_create_error;
enum { Q_BOUND = 0, Q_FINAL = 1, Q_DUAL = 2, Q_REACH = 3, Q_KINDS = 4 };
int pad16(int n) { return (n + 15) / 16 * 16; }

// Static scratch of dr_param_grad_static (the entry point that allocates nothing): each
// device holds its own copy of this array, from the library's first use on that device
// until the process ends.  Host code never uses the array's name as an address: the
// device address of each copy is resolved once per device (hipGetSymbolAddress with
// that device current, in dr_create) and kept in g_scratch_dev.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct dr_ctx {
  int dev = 0;
  int prec = DR_PREC_F32;
  int inter = DR_INTER_CROWN_IBP;
  int max_sub = 0, max_splits = 0, tile_cfg = 0;
  int n_nets = 0, n0 = 0, q = 0, R = 0, H_max = 0, Hp_max = 0;
  bool closed = false;
  bool has_spec = false;
  dr::NetDev hnet[kMaxNets];
  dr::NetDev* dnet = nullptr;
  std::vector<void*> allocs;
  dr::Scratch sc{};
  unsigned* queues = nullptr;
  void* tape = nullptr;
  size_t tape_off[kMaxNets] = {};   // per-network tape regions (the launches may overlap)
  // several networks: one stream per network, forked from and joined back into the
  // caller's stream around the per-network launches so that they overlap
  hipStream_t aux[kMaxNets] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kMaxNets] = {};
  int cus = 0;
  // launch configuration of each kernel kind and network, fixed at creation
  const void* fn[Q_KINDS][kMaxNets] = {};
  int block[Q_KINDS][kMaxNets] = {};
  int grid[Q_KINDS][kMaxNets] = {};
  size_t lds[Q_KINDS][kMaxNets] = {};
  dr::BatchDev batch{};
  bool have_batch = false;
  bool fused_ready = false;   // the last dr_bound_init also produced the plain spec rows
  const double* spec_dev[kMaxNets] = {};   // context-owned spec of each network (the default [I] if none given)
  const double* B_dev[kMaxNets] = {};      // the caller's closed-loop B (valid for the context's lifetime)
  const void* pg_fn = nullptr;  // parameter-gradient instance of k_final (single network)
  int pg_grid = 0;
  void* scratch = nullptr;      // device address of this device's static scratch
  void* jMn[kMaxNets] = {};     // natural copies of the unrolled loop's M and A (refilled by dr_set_weights)
  void* jAn[kMaxNets] = {};
  const void* joint_fn = nullptr;   // k_reach_joint instance (closed loop without a spec, one network)
  const void* rg_fn = nullptr;      // k_reach_grad instance (same contexts), its LDS and full grid
  size_t rg_lds = 0;
  int rg_grid = 0;
  const void* ct_fn = nullptr;      // k_ct_control instance (the context's network as a CT controller),
  size_t ct_lds = 0;                //   its LDS and full grid
  int ct_grid = 0;
  double* ct_state = nullptr;       // max_sub x kCtState: each box's state between the CT launches
  std::string err;
};

namespace {

dr_status fail(dr_ctx* c, dr_status st, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return st;
}

dr_status hip_fail(dr_ctx* c, hipError_t e, const char* what) {
  return fail(c, DR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename P>
hipError_t ctx_alloc(dr_ctx* c, P** p, size_t bytes) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(bytes, 16));
  if (e == hipSuccess) c->allocs.push_back(v);
  *p = (P*)v;
  return e;
}

// ---- kernel instance selection -------------------------------------------------
// The instance set of one chain type and tile count (see instances.hip).
template <typename T>
const void* instance(int NT, int kind, int variant) {
  constexpr bool F = sizeof(T) == 4;
  switch (NT) {
    case 2: return F ? dr_instance_float_2(kind, variant) : dr_instance_double_2(kind, variant);
    case 4: return F ? dr_instance_float_4(kind, variant) : dr_instance_double_4(kind, variant);
    case 6: return F ? dr_instance_float_6(kind, variant) : dr_instance_double_6(kind, variant);
    case 8: return F ? dr_instance_float_8(kind, variant) : dr_instance_double_8(kind, variant);
    case 16: return F ? dr_instance_float_16(kind, variant) : dr_instance_double_16(kind, variant);
    default: return nullptr;
  }
}

// k_final instance of the parameter gradient (the dual kernel that also writes the tapes)
template <typename T>
const void* pgrad_kernel_of(int NT, bool cache) {
  return instance<T>(NT, DR_KIND_PGRAD, cache ? 1 : 0);
}

static_assert(Q_BOUND == DR_KIND_BOUND && Q_FINAL == DR_KIND_FINAL && Q_DUAL == DR_KIND_DUAL &&
                  Q_REACH == DR_KIND_REACH,
              "queue kinds and kernel kinds share their numbering");

const void* kernel_for(const dr_ctx* c, int kind, int NT, int variant) {
  return c->prec == DR_PREC_F64 ? instance<double>(NT, kind, variant) : instance<float>(NT, kind, variant);
}

// LDS of one compute unit (gfx950).
constexpr size_t kMaxLds = 160 * 1024;

// Small networks keep their forward-swizzled weights in LDS inside k_bound_init.
constexpr size_t kLdsWeightBudget = 48 * 1024;
size_t lds_weight_bytes(const dr_ctx* c, const dr::NetDev& n) {
  const size_t v4 = c->prec == DR_PREC_F64 ? 32 : 16;
  return (size_t)dr::lds_w_count(n.L, n.NT) * v4;
}
bool use_lds_weights(const dr_ctx* c, const dr::NetDev& n) {
  return n.NT <= 4 && lds_weight_bytes(c, n) <= kLdsWeightBudget && !(c->tile_cfg & DR_TILE_GLOBAL_WEIGHTS);
}


// Dynamic LDS of a launch: one chain stage per wavefront (wide layers keep the chain
// state in LDS), the kernel's own state, then the hidden biases.
// The dual ascent copies each work item's relaxation and split slots to LDS when the
// copies of the four wavefronts fit beside the chain stages.
size_t item_cache_total(const dr_ctx* c, const dr::NetDev& n) {
  const int P = 16 / std::max(c->R, 1);
  const size_t one = c->prec == DR_PREC_F64 ? dr::item_cache_bytes<double>(P, n.Hp) : dr::item_cache_bytes<float>(P, n.Hp);
  return dr::kWavesPerWG * one;
}
size_t final_lds_base(const dr_ctx* c, const dr::NetDev& n) {
  const int tsz = c->prec == DR_PREC_F64 ? 8 : 4;
  return dr::kWavesPerWG * dr::stage_bytes_rt(tsz, n.NT, true) + (((size_t)n.Hp * sizeof(double) + 15) & ~(size_t)15);
}
bool use_item_cache(const dr_ctx* c, const dr::NetDev& n) {
  return c->R <= 16 && final_lds_base(c, n) + item_cache_total(c, n) <= kMaxLds && !(c->tile_cfg & DR_TILE_NO_ITEM_CACHE);
}

// `block`: threads per workgroup.
size_t lds_bytes(const dr_ctx* c, int kind, const dr::NetDev& n, int block = kWG) {
  const int tsz = c->prec == DR_PREC_F64 ? 8 : 4;
  if (kind == Q_FINAL) return final_lds_base(c, n);
  if (kind == Q_DUAL) return final_lds_base(c, n) + (use_item_cache(c, n) ? item_cache_total(c, n) : 0);
  const int waves = block / 64;
  const size_t stages = (size_t)waves * dr::stage_bytes_rt(tsz, n.NT, false);
  const size_t biases = (size_t)n.Hp * tsz;   // hidden biases staged in the chain type
  size_t b = c->prec == DR_PREC_F64 ? dr::SubLds<double>::bytes(n.Hp, n.NT) : dr::SubLds<float>::bytes(n.Hp, n.NT);
  if (kind == Q_BOUND) {
    const size_t teams = n.NT <= 4 ? waves : 1;   // per-wavefront subdomains for narrow networks
    return stages + teams * b + (use_lds_weights(c, n) ? lds_weight_bytes(c, n) : 0) + biases;
  }
  return stages + b + dr::kReachExtraLds + biases;   // Q_REACH
}

// Launch shape of a persistent kernel: workgroups per CU from the occupancy
// calculator, optionally capped by the launch configuration chosen by the autotuner:
// tile_cfg holds one 4-bit cap per kernel kind (bits 4*kind .. 4*kind+3; 0 = as many
// workgroups per CU as fit).
int persistent_grid(dr_ctx* c, const void* fn, size_t lds, int kind, int block = kWG) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess || nb < 1) nb = 1;
  const int cap = (c->tile_cfg >> (4 * kind)) & 15;
  if (cap > 0) nb = std::min(nb, cap);
  return std::max(1, nb * c->cus);
}

dr_status launch(dr_ctx* c, const void* fn, int grid, size_t lds, void** args, hipStream_t stream, int block = kWG) {
  hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return DR_OK;
}

unsigned* queue_of(dr_ctx* c, int kind, int net) { return c->queues + ((size_t)kind * kMaxNets + net) * 2; }

// Per-network launches of a multi-network context run on their own streams between a
// fork and a join on the caller's stream (also inside a graph capture).
dr_status fork_nets(dr_ctx* c, hipStream_t s) {
  if (c->n_nets < 2) return DR_OK;
  hipError_t e = hipEventRecord(c->fork_ev, s);
  for (int i = 0; e == hipSuccess && i < c->n_nets; ++i) e = hipStreamWaitEvent(c->aux[i], c->fork_ev, 0);
  return e == hipSuccess ? DR_OK : hip_fail(c, e, "stream fork");
}
hipStream_t net_stream(dr_ctx* c, hipStream_t s, int i) { return c->n_nets < 2 ? s : c->aux[i]; }
dr_status join_nets(dr_ctx* c, hipStream_t s) {
  if (c->n_nets < 2) return DR_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; e == hipSuccess && i < c->n_nets; ++i) {
    e = hipEventRecord(c->join_ev[i], c->aux[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->join_ev[i], 0);
  }
  return e == hipSuccess ? DR_OK : hip_fail(c, e, "stream join");
}

// A persistent launch: clear its queue, then launch (same stream, so in order).
dr_status launch_persistent(dr_ctx* c, const void* fn, int grid, size_t lds, void** args, unsigned* q,
                            hipStream_t stream, int block = kWG) {
  hipLaunchKernelGGL(dr::k_reset_queue, dim3(1), dim3(64), 0, stream, q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "queue reset");
  return launch(c, fn, grid, lds, args, stream, block);
}
// The persistent launch of kernel kind `kind` for network i with its stored configuration.
dr_status launch_kind(dr_ctx* c, int kind, int i, void** args, unsigned* q, hipStream_t stream) {
  return launch_persistent(c, c->fn[kind][i], c->grid[kind][i], c->lds[kind][i], args, q, stream, c->block[kind][i]);
}

dr_status check_batch(dr_ctx* c, const dr_batch* b) {
  if (!b) return fail(c, DR_EINVAL, "batch is NULL");
  if (b->n_sub < 0) return fail(c, DR_ESHAPE, "n_sub < 0");
  if (b->n_sub > c->max_sub) return fail(c, DR_ECAPACITY, "n_sub exceeds the context capacity max_sub");
  if (b->n_sub > 0 && (!b->x_center || !b->x_radius)) return fail(c, DR_EINVAL, "x_center/x_radius is NULL");
  if (b->split_ptr && !b->split_packed) return fail(c, DR_EINVAL, "split_ptr without split_packed");
  if (c->n_nets > 1 && !b->net_id && b->n_sub > 0) return fail(c, DR_EINVAL, "net_id required with several networks");
  return DR_OK;
}

// Device copies of one network's parameters and the seeds of its final rows: the
// natural padded copy, the forward and adjoint swizzles, and the seeds (a_L, a_L W_L,
// a_L b_L, skip).  `alloc` creates the buffers (context creation); without it the
// existing buffers are refilled (dr_set_weights: no allocation, capturable).
template <typename T>
dr_status setup_weights(dr_ctx* c, const dr_network& nw, dr::NetDev& nd, int net_i, bool alloc, hipStream_t stream) {
  const int L = nw.n_layers;
  hipError_t e;
  for (int k = 1; k <= L; ++k) {
    const int npk = nd.np[k], npkm1 = nd.np[k - 1];
    const int total = npk * npkm1;
    T *Wn, *bn, *Wf, *Wa;
    if (alloc) {
      if ((e = ctx_alloc(c, &Wn, sizeof(T) * total)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      if ((e = ctx_alloc(c, &bn, sizeof(T) * npk)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      if ((e = ctx_alloc(c, &Wf, sizeof(T) * total)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      if ((e = ctx_alloc(c, &Wa, sizeof(T) * total)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      nd.Wn[k - 1] = Wn; nd.bn[k - 1] = bn; nd.Wf[k - 1] = Wf; nd.Wa[k - 1] = Wa;
    } else {
      Wn = (T*)nd.Wn[k - 1]; bn = (T*)nd.bn[k - 1]; Wf = (T*)nd.Wf[k - 1]; Wa = (T*)nd.Wa[k - 1];
    }
    const int blocks = (std::max(total, npk) + 255) / 256;
    if (nw.wdtype == DR_DTYPE_F64)
      hipLaunchKernelGGL((dr::k_copy_weights<T, double>), dim3(blocks), dim3(256), 0, stream,
                         (const double*)nw.W[k - 1], (const double*)nw.b[k - 1], nd.n[k], nd.n[k - 1], npk, npkm1,
                         Wn, bn);
    else
      hipLaunchKernelGGL((dr::k_copy_weights<T, float>), dim3(blocks), dim3(256), 0, stream,
                         (const float*)nw.W[k - 1], (const float*)nw.b[k - 1], nd.n[k], nd.n[k - 1], npk, npkm1,
                         Wn, bn);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "weight copy");
    hipLaunchKernelGGL((dr::k_swizzle<T>), dim3((total + 255) / 256), dim3(256), 0, stream, Wn, npk, npkm1, 0, Wf);
    hipLaunchKernelGGL((dr::k_swizzle<T>), dim3((total + 255) / 256), dim3(256), 0, stream, Wn, npk, npkm1, 1, Wa);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "weight swizzle");
  }
  // seeds of the final rows
  const int npLm1 = nd.np[L - 1];
  double *seedW, *seedB, *skip, *seedA, *seedWe, *seedBe, *skipE;
  T *seedT, *seedM;
  if (alloc) {
    if ((e = ctx_alloc(c, &seedW, sizeof(double) * nd.R * npLm1)) != hipSuccess ||
        (e = ctx_alloc(c, &seedB, sizeof(double) * nd.R)) != hipSuccess ||
        (e = ctx_alloc(c, &skip, sizeof(double) * nd.R * 16)) != hipSuccess ||
        (e = ctx_alloc(c, &seedA, sizeof(double) * nd.R * nd.np[L])) != hipSuccess ||
        (e = ctx_alloc(c, &seedWe, sizeof(double) * nd.R * npLm1)) != hipSuccess ||
        (e = ctx_alloc(c, &seedBe, sizeof(double) * nd.R)) != hipSuccess ||
        (e = ctx_alloc(c, &skipE, sizeof(double) * nd.R * 16)) != hipSuccess ||
        (e = ctx_alloc(c, &seedT, sizeof(T) * nd.R * npLm1)) != hipSuccess ||
        (e = ctx_alloc(c, &seedM, sizeof(T) * nd.R * npLm1)) != hipSuccess)
      return hip_fail(c, e, "hipMalloc");
    nd.seedW = seedW; nd.seedB = seedB; nd.skip = skip; nd.seedA = seedA;
    nd.seedWe = seedWe; nd.seedBe = seedBe; nd.skipE = skipE; nd.seedT = seedT; nd.seedM = seedM;
  } else {
    seedW = (double*)nd.seedW; seedB = (double*)nd.seedB; skip = (double*)nd.skip; seedA = (double*)nd.seedA;
    seedWe = (double*)nd.seedWe; seedBe = (double*)nd.seedBe; skipE = (double*)nd.skipE;
    seedT = (T*)nd.seedT; seedM = (T*)nd.seedM;
  }
  // the spec: a context-owned copy of the caller's (or the default [I], q = n_target)
  const int n_target = nd.n_state > 0 ? nd.n_state : nd.n[L];
  if (alloc) {
    double* C;
    if ((e = ctx_alloc(c, &C, sizeof(double) * nd.q * n_target)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
    if (nw.spec) {
      e = hipMemcpyAsync(C, nw.spec, sizeof(double) * nd.q * n_target, hipMemcpyDeviceToDevice, stream);
    } else {
      std::vector<double> I((size_t)nd.q * n_target, 0.0);
      for (int i = 0; i < nd.q; ++i) I[(size_t)i * n_target + i] = 1.0;
      e = hipMemcpy(C, I.data(), sizeof(double) * I.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(c, e, "spec copy");
    c->spec_dev[net_i] = C;
    c->B_dev[net_i] = nw.B;
  }
  const double* Cdev = c->spec_dev[net_i];
  const int tot = nd.R * npLm1;
  hipLaunchKernelGGL((dr::k_seeds<T>), dim3((tot + 255) / 256), dim3(256), 0, stream, (const T*)nd.Wn[L - 1],
                     (const T*)nd.bn[L - 1], nd.n[L], npLm1, Cdev, nd.q, n_target, nd.A, c->B_dev[net_i], nd.n[0], nd.np[L],
                     seedW, seedB, skip, seedA, seedWe, seedBe, skipE, seedT, seedM);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "seed kernel");
  // closed loop without a spec: the step-boundary matrices of the unrolled loop (M = B W_L
  // from the seeds of the rows +e_r, and A), forward-swizzled like the weights
  if (nd.A && !c->has_spec) {
    T *Mn, *An, *jM, *jA;
    if (alloc) {
      if ((e = ctx_alloc(c, &Mn, sizeof(T) * 16 * npLm1)) != hipSuccess ||
          (e = ctx_alloc(c, &An, sizeof(T) * 256)) != hipSuccess ||
          (e = ctx_alloc(c, &jM, sizeof(T) * 16 * npLm1)) != hipSuccess ||
          (e = ctx_alloc(c, &jA, sizeof(T) * 256)) != hipSuccess)
        return hip_fail(c, e, "hipMalloc");
      c->jMn[net_i] = Mn; c->jAn[net_i] = An;
      nd.jM = jM; nd.jA = jA;
    } else {
      Mn = (T*)c->jMn[net_i]; An = (T*)c->jAn[net_i]; jM = (T*)nd.jM; jA = (T*)nd.jA;
    }
    const int tm = std::max(16 * npLm1, 256);
    hipLaunchKernelGGL((dr::k_joint_mats<T>), dim3((tm + 255) / 256), dim3(256), 0, stream, (const T*)seedT, npLm1,
                       nd.A, nd.n_state, nd.n[0], Mn, An);
    hipLaunchKernelGGL((dr::k_swizzle<T>), dim3((16 * npLm1 + 255) / 256), dim3(256), 0, stream, (const T*)Mn, 16,
                       npLm1, 0, jM);
    hipLaunchKernelGGL((dr::k_swizzle<T>), dim3(1), dim3(256), 0, stream, (const T*)An, 16, 16, 0, jA);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "step-boundary matrices");
  }
  return DR_OK;
}

constexpr int kWgradChunk = 512;   // rows per workgroup of the contraction

struct PgradLayout {
  size_t rows_pad = 0, cols = 0, tape_bytes = 0, part_off = 0, total = 0;
  int n_chunks = 0;
  size_t poff[kMaxL] = {};
};

PgradLayout pgrad_layout(const dr_ctx* c, int S) {
  PgradLayout pl;
  const dr::NetDev& nd = c->hnet[0];
  const size_t tsz = c->prec == DR_PREC_F64 ? sizeof(double) : sizeof(float);
  const size_t rows = (size_t)S * c->R;
  pl.rows_pad = (rows + 15) / 16 * 16;
  pl.cols = (size_t)dr::ptape_col_g(nd.L - 1, nd.L, nd.NT, nd.np[nd.L]) + 16 * nd.NT;
  pl.tape_bytes = (pl.cols * pl.rows_pad * tsz + 255) & ~(size_t)255;
  pl.n_chunks = (int)((pl.rows_pad + kWgradChunk - 1) / kWgradChunk);
  size_t off = 0;
  for (int k = 1; k <= nd.L; ++k) {
    pl.poff[k - 1] = off;
    off += (size_t)pl.n_chunks * nd.np[k] * (nd.np[k - 1] + 1);
  }
  pl.part_off = pl.tape_bytes;
  pl.total = pl.part_off + ((off * tsz + 255) & ~(size_t)255);
  return pl;
}
}  // namespace

extern "C" {

dr_status dr_create(dr_ctx** out, const dr_network* nets, int n_nets, const dr_options* opt, hipStream_t stream) {
  if (!out) return fail(nullptr, DR_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (!nets || !opt) return fail(nullptr, DR_EINVAL, "nets/opt is NULL");
  if (n_nets < 1 || n_nets > kMaxNets) return fail(nullptr, DR_ESHAPE, "n_nets must be in 1..8");
  if (opt->precision != DR_PREC_F32 && opt->precision != DR_PREC_F64) return fail(nullptr, DR_EINVAL, "bad precision");
  if (opt->intermediate != DR_INTER_CROWN_IBP && opt->intermediate != DR_INTER_IBP)
    return fail(nullptr, DR_EINVAL, "bad intermediate mode");
  if (opt->max_sub < 1 || opt->max_splits < 0 || opt->max_splits > 4096)
    return fail(nullptr, DR_ESHAPE, "max_sub must be >= 1 and max_splits in 0..4096");
  dr_ctx* c = new (std::nothrow) dr_ctx();
  if (!c) return fail(nullptr, DR_ENOMEM, "host allocation failed");
  c->prec = opt->precision;
  c->inter = opt->intermediate;
  c->max_sub = opt->max_sub;
  c->max_splits = opt->max_splits;
  c->tile_cfg = opt->tile_cfg;
  c->n_nets = n_nets;
  if (opt->margin_mode != DR_MARGIN_RIGOROUS && opt->margin_mode != DR_MARGIN_OFF) {
    delete c;
    return fail(nullptr, DR_EINVAL, "bad margin_mode");
  }
  auto bail = [&](dr_status st) {
    g_create_error = c->err;
    dr_destroy(c);
    return st;
  };
  hipError_t e;
  if ((e = hipGetDevice(&c->dev)) != hipSuccess) return bail(hip_fail(c, e, "hipGetDevice"));
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, c->dev)) != hipSuccess) return bail(hip_fail(c, e, "hipGetDeviceProperties"));
  c->cus = prop.multiProcessorCount;
  {
    // this device's copy of the static scratch, resolved once per device
    if (c->dev < 0 || c->dev >= kMaxDevices) return bail(fail(c, DR_EDEVICE, "device index out of range"));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[c->dev]) {
      void* p = nullptr;
      if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
        return bail(hip_fail(c, e, "hipGetSymbolAddress(scratch)"));
      g_scratch_dev[c->dev] = p;
    }
    c->scratch = g_scratch_dev[c->dev];
  }
  for (int i = 0; i < n_nets; ++i) {
    const dr_network& nw = nets[i];
    const int L = nw.n_layers;
    if (L < 2 || L > kMaxL) return bail(fail(c, DR_ESHAPE, "n_layers must be in 2..8"));
    if (!nw.widths || !nw.W || !nw.b) return bail(fail(c, DR_EINVAL, "network arrays are NULL"));
    if (nw.wdtype != DR_DTYPE_F32 && nw.wdtype != DR_DTYPE_F64) return bail(fail(c, DR_EINVAL, "bad wdtype"));
    if (nw.wdtype == DR_DTYPE_F64 && c->prec == DR_PREC_F32)
      return bail(fail(c, DR_EINVAL, "FP64 weights need precision DR_PREC_F64 (the network is its weights)"));
    dr::NetDev& nd = c->hnet[i];
    std::memset(&nd, 0, sizeof(nd));
    nd.L = L;
    int wmax = 0;
    for (int k = 0; k <= L; ++k) {
      nd.n[k] = nw.widths[k];
      if (nd.n[k] < 1) return bail(fail(c, DR_ESHAPE, "widths must be >= 1"));
      if (k >= 1 && k <= L - 1) wmax = std::max(wmax, nd.n[k]);
      if (!nw.W[std::max(k - 1, 0)] || !nw.b[std::max(k - 1, 0)]) return bail(fail(c, DR_EINVAL, "W/b pointer NULL"));
    }
    if (nd.n[0] > 16) return bail(fail(c, DR_ESHAPE, "n_0 must be <= 16"));
    if (nd.n[L] > 64) return bail(fail(c, DR_ESHAPE, "n_L must be <= 64"));
    if (wmax > 256) return bail(fail(c, DR_ESHAPE, "hidden widths must be <= 256"));
    // 16-tiles per hidden layer: 2, 4, 6 (the 96-wide layers of the paper's dynamics
    // models), 8 or 16
    int NT = 2;
    while (NT * 16 < wmax) NT = NT == 4 ? 6 : (NT == 6 ? 8 : 2 * NT);
    nd.NT = NT;
    nd.np[0] = 16;
    for (int k = 1; k <= L - 1; ++k) nd.np[k] = 16 * NT;
    nd.np[L] = pad16(nd.n[L]);
    nd.H = 0;
    for (int k = 1; k <= L - 1; ++k) { nd.hoff[k - 1] = nd.H; nd.H += nd.n[k]; }
    nd.Hp = (L - 1) * 16 * NT;
    const bool closed = nw.A != nullptr || nw.B != nullptr;
    if (closed && (!nw.A || !nw.B)) return bail(fail(c, DR_EINVAL, "closed loop needs both A and B"));
    if (closed && (nw.n_state < 1 || nw.n_state > 16 || nw.n_state > nd.n[0]))
      return bail(fail(c, DR_ESHAPE, "closed loop needs 1 <= n_state <= n_0 (<= 16)"));
    nd.A = nw.A;
    nd.n_state = closed ? nw.n_state : 0;
    const int n_target = closed ? nw.n_state : nd.n[L];
    nd.q = nw.spec ? nw.n_spec : n_target;
    if (nw.spec) c->has_spec = true;
    if (nd.q < 1 || nd.q > 16) return bail(fail(c, DR_ESHAPE, "spec directions q must be in 1..16"));
    nd.R = 2 * nd.q;
    if (i == 0) {
      c->n0 = nd.n[0]; c->q = nd.q; c->R = nd.R; c->closed = closed;
    } else if (nd.n[0] != c->n0 || nd.q != c->q || closed != c->closed) {
      return bail(fail(c, DR_ESHAPE, "all networks of a context need the same n_0, spec length and loop type"));
    }
    c->H_max = std::max(c->H_max, nd.H);
    c->Hp_max = std::max(c->Hp_max, nd.Hp);
    dr_status st = c->prec == DR_PREC_F64 ? setup_weights<double>(c, nw, nd, i, true, stream)
                                          : setup_weights<float>(c, nw, nd, i, true, stream);
    if (st != DR_OK) return bail(st);
  }
  if ((e = ctx_alloc(c, &c->dnet, sizeof(dr::NetDev) * n_nets)) != hipSuccess) return bail(hip_fail(c, e, "hipMalloc"));
  if ((e = hipMemcpyAsync(c->dnet, c->hnet, sizeof(dr::NetDev) * n_nets, hipMemcpyHostToDevice, stream)) != hipSuccess)
    return bail(hip_fail(c, e, "hipMemcpyAsync"));
  // scratch
  const size_t S = (size_t)c->max_sub, Hp = (size_t)c->Hp_max;
  const size_t tsz = c->prec == DR_PREC_F64 ? sizeof(double) : sizeof(float);
  dr::Scratch& sc = c->sc;
  sc.Hp_max = c->Hp_max;
  sc.margin_on = opt->margin_mode == DR_MARGIN_RIGOROUS ? 1 : 0;
  sc.fuse = (opt->fuse_spec && c->R <= 16) ? 1 : 0;
  sc.direct = n_nets == 1 ? 1 : 0;
  if ((e = ctx_alloc(c, &sc.bl, sizeof(double) * S * Hp)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.bu, sizeof(double) * S * Hp)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.rel, 4 * tsz * S * Hp)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.slot, sizeof(int) * S * Hp)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.st, sizeof(uint32_t) * S)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.rows, sizeof(int) * S * 8)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.margin, sizeof(double) * S * 32)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.order, sizeof(int) * S)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.net_cnt, sizeof(int) * kMaxNets)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.net_off, sizeof(int) * kMaxNets)) != hipSuccess ||
      (e = ctx_alloc(c, &sc.fin, sc.fuse ? sizeof(double) * S * 16 * 17 : 16)) != hipSuccess ||
      (e = ctx_alloc(c, &c->queues, sizeof(unsigned) * 2 * Q_KINDS * kMaxNets)) != hipSuccess)
    return bail(hip_fail(c, e, "hipMalloc scratch"));
  if ((e = hipMemsetAsync(c->queues, 0, sizeof(unsigned) * 2 * Q_KINDS * kMaxNets, stream)) != hipSuccess ||
      (e = hipMemsetAsync(sc.rows, 0, sizeof(int) * S * 8, stream)) != hipSuccess ||
      (e = hipMemsetAsync(sc.margin, 0, sizeof(double) * S * 32, stream)) != hipSuccess)
    return bail(hip_fail(c, e, "hipMemsetAsync"));
  // launch shapes and the per-wave tape of the dual ascent (one region per network)
  size_t tape_bytes = 0;
  for (int i = 0; i < n_nets; ++i) {
    const dr::NetDev& nd = c->hnet[i];
    for (int kind = 0; kind < Q_KINDS; ++kind) {
      int variant = 0, block = kWG;
      if (kind == Q_BOUND) {
        variant = (use_lds_weights(c, nd) ? 1 : 0) | ((c->tile_cfg & DR_TILE_PAIRED_TILES) ? 2 : 0);
      } else if (kind == Q_DUAL) {
        variant = use_item_cache(c, nd) ? 1 : 0;
      }
      const void* fn = kernel_for(c, kind, nd.NT, variant);
      if (!fn) return bail(fail(c, DR_ESHAPE, "no kernel instance for this width"));
      const size_t lds = lds_bytes(c, kind, nd, block);
      if (lds > kMaxLds) return bail(fail(c, DR_ESHAPE, "network too deep for the on-chip state of its kernels"));
      if (lds > 0) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return bail(hip_fail(c, e, "hipFuncSetAttribute"));
      }
      c->fn[kind][i] = fn;
      c->block[kind][i] = block;
      c->lds[kind][i] = lds;
      c->grid[kind][i] = persistent_grid(c, fn, lds, kind, block);
    }
    const size_t waves = (size_t)c->grid[Q_DUAL][i] * dr::kWavesPerWG;
    c->tape_off[i] = tape_bytes;
    tape_bytes += (waves * (size_t)(nd.L - 1) * nd.NT * 256 * tsz + 255) & ~(size_t)255;
  }
  if ((e = ctx_alloc(c, &c->tape, tape_bytes)) != hipSuccess) return bail(hip_fail(c, e, "hipMalloc tape"));
  if (n_nets == 1) {
    // the parameter-gradient instance of the dual kernel: same LDS, at most the dual
    // kernel's grid (the per-wave g tape is sized for it)
    const dr::NetDev& nd = c->hnet[0];
    const bool cache = use_item_cache(c, nd);
    c->pg_fn = c->prec == DR_PREC_F64 ? pgrad_kernel_of<double>(nd.NT, cache) : pgrad_kernel_of<float>(nd.NT, cache);
    if (!c->pg_fn) return bail(fail(c, DR_ESHAPE, "no kernel instance for this width"));
    const size_t lds = c->lds[Q_DUAL][0];
    if (lds > 0 && (e = hipFuncSetAttribute(c->pg_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
      return bail(hip_fail(c, e, "hipFuncSetAttribute"));
    c->pg_grid = std::min(persistent_grid(c, c->pg_fn, lds, Q_DUAL), c->grid[Q_DUAL][0]);
  }
  if (n_nets == 1 && c->closed && !c->has_spec) {
    // CROWN through the unrolled loop: its LDS grows with the horizon, so the launch shape
    // is fixed per call; the kernel may use all of a CU's LDS
    c->joint_fn = kernel_for(c, DR_KIND_JOINT, c->hnet[0].NT, 0);
    if (c->joint_fn &&
        (e = hipFuncSetAttribute(c->joint_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess)
      return bail(hip_fail(c, e, "hipFuncSetAttribute"));
    const dr::NetDev& nd = c->hnet[0];
    c->rg_fn = kernel_for(c, DR_KIND_RGRAD, nd.NT, 0);
    const int tsz = c->prec == DR_PREC_F64 ? 8 : 4;
    c->rg_lds = (size_t)dr::kWavesPerWG * dr::stage_bytes_rt(tsz, nd.NT, false) +
                (c->prec == DR_PREC_F64 ? dr::GradLds<double>::bytes(nd.Hp, nd.NT) : dr::GradLds<float>::bytes(nd.Hp, nd.NT));
    if (c->rg_fn && c->rg_lds <= kMaxLds && dr::rg_slots(nd.L, nd.NT) <= dr::kRgMaxSlots && nd.np[0] == 16) {
      if ((e = hipFuncSetAttribute(c->rg_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess)
        return bail(hip_fail(c, e, "hipFuncSetAttribute"));
      c->rg_grid = persistent_grid(c, c->rg_fn, c->rg_lds, Q_REACH);
    } else {
      c->rg_fn = nullptr;
    }
    // the CT closed loop: the controller step has the stepwise reach's on-chip state; each
    // box's state between the launches (n_0 <= 16 states)
    c->ct_fn = nd.n[0] <= dr::kCtMax ? kernel_for(c, DR_KIND_CT, nd.NT, 0) : nullptr;
    c->ct_lds = lds_bytes(c, Q_REACH, nd);
    if (c->ct_fn && c->ct_lds <= kMaxLds) {
      if ((e = hipFuncSetAttribute(c->ct_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->ct_lds)) != hipSuccess)
        return bail(hip_fail(c, e, "hipFuncSetAttribute"));
      c->ct_grid = persistent_grid(c, c->ct_fn, c->ct_lds, Q_REACH);
      if ((e = ctx_alloc(c, &c->ct_state, sizeof(double) * dr::kCtState * std::max(c->max_sub, 1))) != hipSuccess)
        return bail(hip_fail(c, e, "hipMalloc CT state"));
    } else {
      c->ct_fn = nullptr;
    }
  }
  if (n_nets > 1) {
    if ((e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming)) != hipSuccess)
      return bail(hip_fail(c, e, "hipEventCreate"));
    for (int i = 0; i < n_nets; ++i)
      if ((e = hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking)) != hipSuccess ||
          (e = hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming)) != hipSuccess)
        return bail(hip_fail(c, e, "stream/event creation"));
  }
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return bail(hip_fail(c, e, "set-up"));
  *out = c;
  return DR_OK;
}

dr_status dr_set_weights(dr_ctx* c, int net_index, const dr_network* nw, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (net_index < 0 || net_index >= c->n_nets) return fail(c, DR_EINVAL, "net_index out of range");
  if (!nw || !nw->widths || !nw->W || !nw->b) return fail(c, DR_EINVAL, "network arrays are NULL");
  dr::NetDev& nd = c->hnet[net_index];
  if (nw->n_layers != nd.L) return fail(c, DR_ESHAPE, "n_layers differs from the network of the context");
  for (int k = 0; k <= nd.L; ++k)
    if (nw->widths[k] != nd.n[k]) return fail(c, DR_ESHAPE, "widths differ from the network of the context");
  if (nw->wdtype != DR_DTYPE_F32 && nw->wdtype != DR_DTYPE_F64) return fail(c, DR_EINVAL, "bad wdtype");
  if (nw->wdtype == DR_DTYPE_F64 && c->prec == DR_PREC_F32)
    return fail(c, DR_EINVAL, "FP64 weights need precision DR_PREC_F64 (the network is its weights)");
  for (int k = 0; k < nd.L; ++k)
    if (!nw->W[k] || !nw->b[k]) return fail(c, DR_EINVAL, "W/b pointer NULL");
  dr_status st = c->prec == DR_PREC_F64 ? setup_weights<double>(c, *nw, nd, net_index, false, stream)
                                        : setup_weights<float>(c, *nw, nd, net_index, false, stream);
  if (st != DR_OK) return st;
  // state computed with the old weights is stale
  c->have_batch = false;
  c->fused_ready = false;
  return DR_OK;
}

dr_status dr_bound_init(dr_ctx* c, const dr_batch* b, uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  dr_status st = check_batch(c, b);
  if (st != DR_OK) return st;
  c->batch.n_sub = b->n_sub;
  c->batch.net_id = b->net_id;
  c->batch.xc = b->x_center;
  c->batch.xr = b->x_radius;
  c->batch.sptr = b->split_ptr;
  c->batch.spk = b->split_packed;
  c->have_batch = true;
  c->fused_ready = false;
  c->sc.n_sub = b->n_sub;
  if (b->n_sub == 0) return DR_OK;
  hipError_t e;
  if (!c->sc.direct) {
    // several networks: counting sort of the batch by network id
    hipLaunchKernelGGL(dr::k_order, dim3(1), dim3(1024), 0, stream, b->n_sub, b->net_id, c->n_nets, c->sc.order,
                       c->sc.net_cnt, c->sc.net_off, c->sc.st);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "order kernel");
  }
  if ((st = fork_nets(c, stream)) != DR_OK) return st;
  for (int i = 0; i < c->n_nets; ++i) {
    int net_index = i, inter = c->inter, ms = c->max_splits;
    dr::BatchDev bd = c->batch;
    dr::Scratch sc = c->sc;
    sc.st_out = status;
    void* args[] = {&c->dnet, &net_index, &bd, &sc, &inter, &ms};
    // static item assignment: no queue to clear
    if ((st = launch(c, c->fn[Q_BOUND][i], c->grid[Q_BOUND][i], c->lds[Q_BOUND][i], args, net_stream(c, stream, i),
                     c->block[Q_BOUND][i])) != DR_OK)
      return st;
  }
  if ((st = join_nets(c, stream)) != DR_OK) return st;
  if (status && !c->sc.direct) {
    // subdomains with an invalid network id are not processed by any launch
    e = hipMemcpyAsync(status, c->sc.st, sizeof(uint32_t) * b->n_sub, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(c, e, "status copy");
  }
  c->fused_ready = c->sc.fuse != 0;
  return DR_OK;
}

static dr_status run_final(dr_ctx* c, bool duals, dr::FinalArgs fa, hipStream_t stream) {
  fa.batch = c->batch;
  fa.sc = c->sc;
  fa.sc.st_out = nullptr;
  fa.H_max = c->H_max;
  fa.max_splits = std::max(c->max_splits, 1);
  fa.q = c->q;
  dr_status st = fork_nets(c, stream);
  if (st != DR_OK) return st;
  for (int i = 0; i < c->n_nets; ++i) {
    const int kind = duals ? Q_DUAL : Q_FINAL;
    fa.queue = queue_of(c, kind, i);
    fa.tape = (char*)c->tape + c->tape_off[i];
    int net_index = i;
    void* args[] = {&c->dnet, &net_index, &fa};
    st = launch_kind(c, kind, i, args, fa.queue, net_stream(c, stream, i));
    if (st != DR_OK) return st;
  }
  return join_nets(c, stream);
}

dr_status dr_propagate_backward(dr_ctx* c, double* lam_lo, double* acc_lo, double* lam_hi, double* acc_hi,
                                hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->have_batch) return fail(c, DR_EINVAL, "dr_bound_init has not been called");
  if (c->batch.n_sub == 0) return DR_OK;
  if (!lam_lo || !acc_lo || !lam_hi || !acc_hi) return fail(c, DR_EINVAL, "output pointer is NULL");
  if (c->R > 16) return fail(c, DR_ESHAPE, "spec rows 2q must be <= 16 for the spec chains");
  if (c->fused_ready) {
    const int S = c->batch.n_sub, tot = S * c->R;
    hipLaunchKernelGGL(dr::k_copy_final, dim3((tot + 255) / 256), dim3(256), 0, stream, S, c->q, c->n0, c->sc.fin,
                       c->sc.st, lam_lo, acc_lo, lam_hi, acc_hi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "copy kernel");
    return DR_OK;
  }
  dr::FinalArgs fa{};
  fa.lam_lo = lam_lo; fa.acc_lo = acc_lo; fa.lam_hi = lam_hi; fa.acc_hi = acc_hi;
  return run_final(c, false, fa, stream);
}

dr_status dr_concretize(dr_ctx* c, const double* lam_lo, const double* acc_lo, const double* lam_hi,
                        const double* acc_hi, double* lb, double* ub, uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->have_batch) return fail(c, DR_EINVAL, "dr_bound_init has not been called");
  if (c->batch.n_sub == 0) return DR_OK;
  if (!lam_lo || !acc_lo || !lam_hi || !acc_hi || !lb || !ub) return fail(c, DR_EINVAL, "array pointer is NULL");
  const int S = c->batch.n_sub;
  int Q2 = 1;
  while (Q2 < c->q) Q2 *= 2;     // q <= 16
  const long long threads = (long long)S * Q2;
  hipLaunchKernelGGL(dr::k_concretize, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, S, c->q, c->n0,
                     Q2, c->batch.xc, c->batch.xr, lam_lo, acc_lo, lam_hi, acc_hi, lb, ub, c->sc.st, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "concretize kernel");
  return DR_OK;
}

dr_status dr_optimize_duals(dr_ctx* c, int iters, float lr, int init_duals, float* alpha, float* beta, double* lb,
                            double* ub, float* grad_alpha, float* grad_beta, uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->have_batch) return fail(c, DR_EINVAL, "dr_bound_init has not been called");
  if (iters < 0 || iters > 100000) return fail(c, DR_EINVAL, "iters must be in 0..100000");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(c, DR_EINVAL, "lr must be finite and >= 0");
  if (c->batch.n_sub == 0) return DR_OK;
  if (!alpha || !beta || !lb || !ub) return fail(c, DR_EINVAL, "alpha/beta/lb/ub is NULL");
  if (c->R > 16) return fail(c, DR_ESHAPE, "spec rows 2q must be <= 16 for the dual ascent");
  dr::FinalArgs fa{};
  fa.iters = iters; fa.lr = lr; fa.init_duals = init_duals ? 1 : 0;
  fa.alpha = alpha; fa.beta = beta; fa.lb = lb; fa.ub = ub; fa.galpha = grad_alpha; fa.gbeta = grad_beta;
  dr_status st = run_final(c, true, fa, stream);
  if (st != DR_OK) return st;
  if (status) {
    hipError_t e = hipMemcpyAsync(status, c->sc.st, sizeof(uint32_t) * c->batch.n_sub, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(c, e, "status copy");
  }
  return DR_OK;
}


size_t dr_param_grad_workspace(const dr_ctx* c, int n_sub) {
  if (!c || n_sub < 0 || c->n_nets != 1) return 0;
  return pgrad_layout(c, std::max(n_sub, 1)).total;
}

}  // extern "C"

// The parameter gradient with its tapes and partial sums in `workspace` (the caller's
// buffer, or the library's static scratch).
static dr_status param_grad_impl(dr_ctx* c, float* alpha, float* beta, int init_duals, const double* g_lb,
                                 const double* g_ub, double* lb, double* ub, double* const* dW, double* const* db,
                                 double* dxc, double* dxr, void* workspace, size_t workspace_bytes, uint32_t* status,
                                 hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->have_batch) return fail(c, DR_EINVAL, "dr_bound_init has not been called");
  if (c->n_nets != 1) return fail(c, DR_EINVAL, "the parameter gradient takes a single-network context");
  if (c->R > 16) return fail(c, DR_ESHAPE, "spec rows 2q must be <= 16 for the spec chains");
  const dr::NetDev& nd = c->hnet[0];
  if (!dW || !db) return fail(c, DR_EINVAL, "dW/db is NULL");
  for (int k = 0; k < nd.L; ++k)
    if (!dW[k] || !db[k]) return fail(c, DR_EINVAL, "a dW/db layer pointer is NULL");
  const int S = c->batch.n_sub;
  if (S > 0 && (!alpha || !beta || !g_lb || !g_ub || !lb || !ub))
    return fail(c, DR_EINVAL, "alpha/beta/g_lb/g_ub/lb/ub is NULL");
  const PgradLayout pl = pgrad_layout(c, std::max(S, 1));
  if (!workspace || workspace_bytes < pl.total) return fail(c, DR_EINVAL, "workspace is NULL or smaller than dr_param_grad_workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(c, DR_EINVAL, "workspace must be 256-byte aligned");
  dr::WgradArgs wa{};
  wa.tape = workspace;
  wa.rows_pad = pl.rows_pad;
  wa.rows = S * c->R;
  wa.chunk_rows = kWgradChunk;
  wa.n_chunks = pl.n_chunks;
  for (int k = 0; k < nd.L; ++k) { wa.poff[k] = pl.poff[k]; wa.dW[k] = dW[k]; wa.db[k] = db[k]; }
  wa.part = (char*)workspace + pl.part_off;
  int net_index = 0;
  if (S > 0) {
    dr::FinalArgs fa{};
    fa.iters = 0; fa.lr = 0.0f; fa.init_duals = init_duals ? 1 : 0;
    fa.alpha = alpha; fa.beta = beta; fa.lb = lb; fa.ub = ub;
    fa.g_lb = g_lb; fa.g_ub = g_ub; fa.ptape = workspace; fa.rows_pad = pl.rows_pad; fa.dxc = dxc; fa.dxr = dxr;
    fa.batch = c->batch;
    fa.sc = c->sc;
    fa.sc.st_out = nullptr;
    fa.H_max = c->H_max;
    fa.max_splits = std::max(c->max_splits, 1);
    fa.q = c->q;
    fa.queue = queue_of(c, Q_DUAL, 0);
    fa.tape = c->tape;
    void* args[] = {&c->dnet, &net_index, &fa};
    dr_status st = launch_persistent(c, c->pg_fn, c->pg_grid, c->lds[Q_DUAL][0], args, fa.queue, stream);
    if (st != DR_OK) return st;
  }
  // the contraction (rows of an empty batch sum to zero)
  int max_mt = 1;
  for (int k = 1; k <= nd.L; ++k) max_mt = std::max(max_mt, nd.np[k] / 16);
  const dim3 gw(pl.n_chunks, max_mt, nd.L);
  if (c->prec == DR_PREC_F64)
    hipLaunchKernelGGL(dr::k_wgrad<double>, gw, dim3(256), 0, stream, c->dnet, net_index, wa);
  else
    hipLaunchKernelGGL(dr::k_wgrad<float>, gw, dim3(256), 0, stream, c->dnet, net_index, wa);
  int max_el = 1;
  for (int k = 1; k <= nd.L; ++k) max_el = std::max(max_el, nd.n[k] * (nd.n[k - 1] + 1));
  const dim3 gr((max_el + 255) / 256, nd.L);
  if (c->prec == DR_PREC_F64)
    hipLaunchKernelGGL(dr::k_wgrad_reduce<double>, gr, dim3(256), 0, stream, c->dnet, net_index, wa);
  else
    hipLaunchKernelGGL(dr::k_wgrad_reduce<float>, gr, dim3(256), 0, stream, c->dnet, net_index, wa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "parameter-gradient kernels");
  if (status && S > 0) {
    e = hipMemcpyAsync(status, c->sc.st, sizeof(uint32_t) * S, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(c, e, "status copy");
  }
  return DR_OK;
}

extern "C" {

dr_status dr_param_grad(dr_ctx* c, float* alpha, float* beta, int init_duals, const double* g_lb, const double* g_ub,
                        double* lb, double* ub, double* const* dW, double* const* db, double* dxc, double* dxr,
                        void* workspace, size_t workspace_bytes, uint32_t* status, hipStream_t stream) {
  return param_grad_impl(c, alpha, beta, init_duals, g_lb, g_ub, lb, ub, dW, db, dxc, dxr, workspace, workspace_bytes,
                         status, stream);
}

dr_status dr_param_grad_static(dr_ctx* c, float* alpha, float* beta, int init_duals, const double* g_lb,
                               const double* g_ub, double* lb, double* ub, double* const* dW, double* const* db,
                               double* dxc, double* dxr, uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->scratch) return fail(c, DR_EDEVICE, "the static scratch of this device was not resolved");
  if (c->have_batch && c->n_nets == 1) {
    const size_t need = pgrad_layout(c, std::max(c->batch.n_sub, 1)).total;
    if (need > kStaticScratchBytes)
      return fail(c, DR_ECAPACITY,
                  "batch needs " + std::to_string(need) + " bytes of parameter-gradient scratch; the static buffer "
                  "holds " + std::to_string(kStaticScratchBytes) + " (use dr_param_grad with a workspace)");
  }
  return param_grad_impl(c, alpha, beta, init_duals, g_lb, g_ub, lb, ub, dW, db, dxc, dxr, c->scratch,
                         kStaticScratchBytes, status, stream);
}

}  // extern "C"

static dr_status reach(dr_ctx* c, const dr_batch* b, int horizon, const double* u, double* boxes, uint32_t* status,
                       hipStream_t stream, double* tape = nullptr) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->closed) return fail(c, DR_EINVAL, "reach_dt needs a closed-loop network");
  if (c->has_spec) return fail(c, DR_EINVAL, "reach_dt bounds every state: create the context without a spec");
  const bool exo = c->q < c->n0;   // without a spec q = n_state
  if (exo && !u && horizon > 0 && b && b->n_sub > 0)
    return fail(c, DR_EINVAL, "the network has exogenous inputs: use dr_reach_dt_exo with the input sequences");
  if (!exo && u) return fail(c, DR_EINVAL, "u given but the network has no exogenous inputs");
  if (horizon < 0 || horizon > 10000) return fail(c, DR_EINVAL, "horizon must be in 0..10000");
  dr_status st = check_batch(c, b);
  if (st != DR_OK) return st;
  if (b->split_ptr) return fail(c, DR_EINVAL, "reach_dt takes no split constraints");
  if (!boxes) return fail(c, DR_EINVAL, "boxes is NULL");
  c->batch.n_sub = b->n_sub;
  c->batch.net_id = b->net_id;
  c->batch.xc = b->x_center;
  c->batch.xr = b->x_radius;
  c->batch.sptr = nullptr;
  c->batch.spk = nullptr;
  c->have_batch = false;  // bound_init state is not valid for this batch
  c->fused_ready = false;
  c->sc.n_sub = b->n_sub;
  if (b->n_sub == 0) return DR_OK;
  if (!c->sc.direct) {
    hipLaunchKernelGGL(dr::k_order, dim3(1), dim3(1024), 0, stream, b->n_sub, b->net_id, c->n_nets, c->sc.order,
                       c->sc.net_cnt, c->sc.net_off, c->sc.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "order kernel");
  }
  if ((st = fork_nets(c, stream)) != DR_OK) return st;
  for (int i = 0; i < c->n_nets; ++i) {
    dr::ReachArgs ra{};
    ra.batch = c->batch; ra.sc = c->sc; ra.sc.st_out = nullptr; ra.queue = queue_of(c, Q_REACH, i);
    ra.horizon = horizon; ra.boxes = boxes; ra.status = status; ra.u = u; ra.tape = tape;
    int net_index = i;
    void* args[] = {&c->dnet, &net_index, &ra};
    if ((st = launch_kind(c, Q_REACH, i, args, ra.queue, net_stream(c, stream, i))) != DR_OK) return st;
  }
  if ((st = join_nets(c, stream)) != DR_OK) return st;
  return DR_OK;
}

// LDS of k_reach_joint over `horizon` steps: the chain stages and the per-box state
// (the relaxation of every step is kept on chip).
static size_t joint_lds(const dr_ctx* c, const dr::NetDev& n, int horizon) {
  const int tsz = c->prec == DR_PREC_F64 ? 8 : 4;
  const size_t st = (size_t)dr::kWavesPerWG * dr::stage_bytes_rt(tsz, n.NT, false);
  return st + (c->prec == DR_PREC_F64 ? dr::JointLds<double>::bytes(horizon, n.Hp, n.NT)
                                      : dr::JointLds<float>::bytes(horizon, n.Hp, n.NT));
}

static dr_status reach_joint(dr_ctx* c, const dr_batch* b, int horizon, const double* u, double* boxes, int* rows,
                             uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->closed) return fail(c, DR_EINVAL, "reach_dt_joint needs a closed-loop network");
  if (c->has_spec) return fail(c, DR_EINVAL, "reach_dt_joint bounds every state: create the context without a spec");
  if (c->n_nets != 1) return fail(c, DR_EINVAL, "reach_dt_joint takes a context with one network");
  const bool exo = c->q < c->n0;
  if (exo && !u && horizon > 0 && b && b->n_sub > 0)
    return fail(c, DR_EINVAL, "the network has exogenous inputs: u (the input sequences) is required");
  if (!exo && u) return fail(c, DR_EINVAL, "u given but the network has no exogenous inputs");
  if (horizon < 0 || horizon > 10000) return fail(c, DR_EINVAL, "horizon must be in 0..10000");
  dr_status st = check_batch(c, b);
  if (st != DR_OK) return st;
  if (b->split_ptr) return fail(c, DR_EINVAL, "reach_dt_joint takes no split constraints");
  if (!boxes) return fail(c, DR_EINVAL, "boxes is NULL");
  if (!c->joint_fn) return fail(c, DR_ESHAPE, "no kernel instance for this width");
  const dr::NetDev& nd = c->hnet[0];
  if (nd.n[0] > 16 || nd.n_state > 16) return fail(c, DR_ESHAPE, "reach_dt_joint needs n_0 <= 16");
  const size_t lds = joint_lds(c, nd, horizon);
  if (lds > kMaxLds) {
    int hmax = 0;
    while (joint_lds(c, nd, hmax + 1) <= kMaxLds) ++hmax;
    return fail(c, DR_ECAPACITY, "horizon too long for the on-chip relaxation store of this network: at most " +
                                     std::to_string(hmax) + " steps");
  }
  c->batch.n_sub = b->n_sub;
  c->batch.net_id = b->net_id;
  c->batch.xc = b->x_center;
  c->batch.xr = b->x_radius;
  c->batch.sptr = nullptr;
  c->batch.spk = nullptr;
  c->have_batch = false;  // bound_init state is not valid for this batch
  c->fused_ready = false;
  c->sc.n_sub = b->n_sub;
  if (b->n_sub == 0) return DR_OK;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, c->joint_fn, kWG, lds) != hipSuccess || nb < 1) nb = 1;
  const int grid = std::min(nb * c->cus, b->n_sub);
  dr::JointArgs ja{};
  ja.batch = c->batch; ja.sc = c->sc; ja.sc.st_out = nullptr;
  ja.horizon = horizon; ja.boxes = boxes; ja.rows = rows; ja.status = status; ja.u = u;
  int net_index = 0;
  void* args[] = {&c->dnet, &net_index, &ja};
  return launch(c, c->joint_fn, grid, lds, args, stream);
}

// Workspace of dr_reach_dt_grad: the forward record of every box, the row-tile records
// of one step per workgroup of the reverse kernel, then one weight-gradient region per
// workgroup.
struct ReachGradLayout {
  size_t gtape_off = 0, wreg_off = 0, total = 0, wstride = 0;
  size_t woff[dr::kMaxL] = {};
  int grid = 0;
};
static ReachGradLayout reach_grad_layout(const dr_ctx* c, int S, int horizon) {
  ReachGradLayout g;
  const dr::NetDev& nd = c->hnet[0];
  const size_t tsz = c->prec == DR_PREC_F64 ? sizeof(double) : sizeof(float);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  g.grid = std::max(1, std::min(c->rg_grid, std::max(S, 1)));
  g.gtape_off = al((size_t)std::max(S, 1) * dr::reach_tape_doubles(horizon, nd.Hp) * sizeof(double));
  g.wreg_off = al(g.gtape_off + (size_t)g.grid * dr::rg_slots(nd.L, nd.NT) * dr::rg_slot_elems(nd.L, nd.NT) * tsz);
  size_t w = 0;
  for (int k = 1; k <= nd.L; ++k) {
    g.woff[k - 1] = w;
    w += (size_t)nd.np[k] * (nd.np[k - 1] + 1);
  }
  g.wstride = (w + 63) & ~(size_t)63;
  g.total = g.wreg_off + (size_t)g.grid * g.wstride * tsz;
  return g;
}

extern "C" {

size_t dr_reach_grad_workspace(const dr_ctx* c, int n_sub, int horizon) {
  if (!c || !c->rg_fn || n_sub < 0 || horizon < 0) return 0;
  return reach_grad_layout(c, n_sub, horizon).total;
}

dr_status dr_reach_dt_grad(dr_ctx* c, const dr_batch* b, int horizon, const double* u, const double* g_V,
                           double* boxes, double* du, double* dxc, double* dxr, double* dA, double* dB,
                           double* const* dW, double* const* db, void* workspace, size_t workspace_bytes,
                           uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!c->closed || c->has_spec || c->n_nets != 1)
    return fail(c, DR_EINVAL, "reach_dt_grad needs a context with one closed-loop network and no spec");
  if (!c->rg_fn) return fail(c, DR_ESHAPE, "no reverse-pass kernel for this network (on-chip state too large)");
  if (!b) return fail(c, DR_EINVAL, "batch is NULL");
  if (b->n_sub > 0 && horizon > 0 && !g_V) return fail(c, DR_EINVAL, "g_V is NULL");
  const bool exo = c->q < c->n0;
  if (exo && du && !u && horizon > 0 && b->n_sub > 0) return fail(c, DR_EINVAL, "du needs the input sequences u");
  const ReachGradLayout lay = reach_grad_layout(c, b->n_sub, horizon);
  if (b->n_sub > 0 && (!workspace || workspace_bytes < lay.total))
    return fail(c, DR_EINVAL, "workspace is NULL or smaller than dr_reach_grad_workspace(ctx, S, horizon)");
  // the forward reach with its record
  dr_status st = reach(c, b, horizon, u, boxes, status, stream, (double*)workspace);
  if (st != DR_OK) return st;
  const dr::NetDev& nd = c->hnet[0];
  const int ns = nd.n_state;
  if (dA) hipLaunchKernelGGL(dr::k_zero, dim3(1), dim3(256), 0, stream, dA, (size_t)ns * nd.n[0]);
  if (dB) hipLaunchKernelGGL(dr::k_zero, dim3(1), dim3(256), 0, stream, dB, (size_t)ns * nd.n[nd.L]);
  bool want_w = false;
  for (int k = 0; k < nd.L; ++k) want_w = want_w || (dW && dW[k]) || (db && db[k]);
  const size_t tsz = c->prec == DR_PREC_F64 ? sizeof(double) : sizeof(float);
  // the weight-gradient regions: accumulated in LDS and stored once per workgroup when they
  // fit beside the kernel's state, else accumulated in global memory (cleared first)
  const bool wacc_lds = want_w && c->rg_lds + lay.wstride * tsz <= kMaxLds;
  if (want_w && !wacc_lds && b->n_sub > 0) {
    const size_t words = (size_t)lay.grid * lay.wstride * tsz / sizeof(double);
    hipLaunchKernelGGL(dr::k_zero, dim3(1024), dim3(256), 0, stream, (double*)((char*)workspace + lay.wreg_off), words);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "zero kernel");
  if (b->n_sub == 0) return DR_OK;
  if (horizon == 0) {
    // no step: the volume is 0 and every gradient is zero
    if (dxc) hipLaunchKernelGGL(dr::k_zero, dim3(1), dim3(256), 0, stream, dxc, (size_t)b->n_sub * ns);
    if (dxr) hipLaunchKernelGGL(dr::k_zero, dim3(1), dim3(256), 0, stream, dxr, (size_t)b->n_sub * ns);
    for (int k = 0; want_w && k < nd.L; ++k) {
      if (dW && dW[k]) hipLaunchKernelGGL(dr::k_zero, dim3(64), dim3(256), 0, stream, dW[k], (size_t)nd.n[k + 1] * nd.n[k]);
      if (db && db[k]) hipLaunchKernelGGL(dr::k_zero, dim3(1), dim3(256), 0, stream, db[k], (size_t)nd.n[k + 1]);
    }
    e = hipGetLastError();
    return e == hipSuccess ? DR_OK : hip_fail(c, e, "zero kernel");
  }
  dr::ReachGradArgs ga{};
  ga.batch = c->batch; ga.sc = c->sc; ga.horizon = horizon;
  ga.tape = (const double*)workspace;
  ga.gV = g_V;
  ga.gtape = (char*)workspace + lay.gtape_off;
  ga.du = du; ga.dxc = dxc; ga.dxr = dxr; ga.dA = dA; ga.dB = dB;
  ga.wreg = want_w ? (char*)workspace + lay.wreg_off : nullptr;
  ga.wreg_stride = lay.wstride;
  ga.wacc_lds = wacc_lds ? 1 : 0;
  for (int k = 0; k < dr::kMaxL; ++k) ga.woff[k] = lay.woff[k];
  int net_index = 0;
  void* args[] = {&c->dnet, &net_index, &ga};
  const size_t lds = c->rg_lds + (wacc_lds ? lay.wstride * tsz : 0);
  if ((st = launch(c, c->rg_fn, lay.grid, lds, args, stream)) != DR_OK) return st;
  if (want_w) {
    dr::ReachWreduceArgs ra{};
    ra.wreg = (char*)workspace + lay.wreg_off;
    ra.stride = lay.wstride;
    for (int k = 0; k < dr::kMaxL; ++k) ra.woff[k] = lay.woff[k];
    ra.n_regions = lay.grid;
    int maxe = 0;
    for (int k = 0; k < nd.L; ++k) {
      ra.dW[k] = dW ? dW[k] : nullptr;
      ra.db[k] = db ? db[k] : nullptr;
      maxe = std::max(maxe, nd.n[k + 1] * (nd.n[k] + 1));
    }
    const dim3 grid((maxe + 255) / 256, nd.L);
    if (c->prec == DR_PREC_F64)
      hipLaunchKernelGGL(dr::k_reach_wreduce<double>, grid, dim3(256), 0, stream, c->dnet, 0, ra);
    else
      hipLaunchKernelGGL(dr::k_reach_wreduce<float>, grid, dim3(256), 0, stream, c->dnet, 0, ra);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "weight-gradient reduction");
  }
  return DR_OK;
}

dr_status dr_reach_dt_joint(dr_ctx* c, const dr_batch* b, int horizon, const double* u, double* boxes, int* rows,
                            uint32_t* status, hipStream_t stream) {
  return reach_joint(c, b, horizon, u, boxes, rows, status, stream);
}

dr_status dr_reach_dt(dr_ctx* c, const dr_batch* b, int horizon, double* boxes, uint32_t* status, hipStream_t stream) {
  return reach(c, b, horizon, nullptr, boxes, status, stream);
}

dr_status dr_reach_dt_exo(dr_ctx* c, const dr_batch* b, int horizon, const double* u, double* boxes, uint32_t* status,
                          hipStream_t stream) {
  return reach(c, b, horizon, u, boxes, status, stream);
}

// ---- continuous time ------------------------------------------------------------
static dr_status check_ct(dr_ctx* c, const dr_ct_field* f, const dr_ct_options* o) {
  if (!f || !o) return fail(c, DR_EINVAL, "field or options is NULL");
  if (f->n < 1 || f->n > dr::kCtMax) return fail(c, DR_ESHAPE, "the CT state dimension n must be in 1..16");
  if (f->n_u < 0 || f->n_u > dr::kCtMax) return fail(c, DR_ESHAPE, "the CT input dimension n_u must be in 0..16");
  if (!f->a || !f->F) return fail(c, DR_EINVAL, "the field's a and F are required");
  if ((f->n_u > 0) != (f->G != nullptr)) return fail(c, DR_EINVAL, "G is required exactly when n_u > 0");
  if (!(o->h > 0.0) || !std::isfinite(o->h)) return fail(c, DR_EINVAL, "h must be positive and finite");
  if (o->steps < 1 || o->intervals < 0 || (long long)o->steps * o->intervals > 100000)
    return fail(c, DR_EINVAL, "steps >= 1, intervals >= 0 and steps * intervals <= 100000 are required");
  if (o->tries < 1 || o->tries > 1000 || o->rounds < 0 || o->rounds > 100)
    return fail(c, DR_EINVAL, "tries must be in 1..1000 and rounds in 0..100");
  if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(c, DR_EINVAL, "eps must be positive and finite");
  return DR_OK;
}

static dr::CtArgs ct_args(const dr_ct_field* f, const dr_ct_options* o, double* boxes, double* segs, uint32_t* status) {
  dr::CtArgs ca{};
  ca.dyn.n = f->n; ca.dyn.n_u = f->n_u;
  ca.dyn.a = f->a; ca.dyn.F = f->F; ca.dyn.G = f->G; ca.dyn.Q = f->Q;
  ca.h = o->h; ca.K = o->steps; ca.n_ctl = o->intervals;
  ca.tries = o->tries; ca.rounds = o->rounds; ca.eps = o->eps;
  ca.boxes = boxes; ca.segs = segs; ca.status = status;
  return ca;
}

dr_status dr_flowpipe_ct(const dr_ct_field* f, const dr_ct_options* o, int n_sub, const double* xc, const double* xr,
                         double* boxes, double* segs, uint32_t* status, hipStream_t stream) {
  dr_status st = check_ct(nullptr, f, o);
  if (st != DR_OK) return st;
  if (f->n_u != 0) return fail(nullptr, DR_EINVAL, "dr_flowpipe_ct takes a field without an input (n_u = 0)");
  if (n_sub < 0) return fail(nullptr, DR_EINVAL, "n_sub must be >= 0");
  if (n_sub == 0) return DR_OK;
  if (!xc || !xr || !boxes) return fail(nullptr, DR_EINVAL, "x_center, x_radius and boxes are required");
  dr::CtArgs ca = ct_args(f, o, boxes, segs, status);
  ca.batch.n_sub = n_sub; ca.batch.xc = xc; ca.batch.xr = xr;
  int dev = 0, cus = 0, nb = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(nullptr, e, "device query");
  const size_t lds = dr::CtLds::bytes(0);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)dr::k_flowpipe_ct, 64, lds) != hipSuccess || nb < 1)
    nb = 1;
  const int grid = (int)std::min<long long>((long long)nb * std::max(cus, 1), n_sub);
  hipLaunchKernelGGL(dr::k_flowpipe_ct, dim3(grid), dim3(64), lds, stream, ca);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(nullptr, e, "kernel launch");
  return DR_OK;
}

dr_status dr_reach_ct(dr_ctx* c, const dr_ct_field* f, const dr_ct_options* o, const dr_batch* b, double* boxes,
                      double* segs, uint32_t* status, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  dr_status st = check_ct(c, f, o);
  if (st != DR_OK) return st;
  if (!c->closed || c->has_spec || c->n_nets != 1)
    return fail(c, DR_EINVAL, "reach_ct needs a context with one closed-loop network and no spec");
  const dr::NetDev& nd = c->hnet[0];
  if (f->n_u < 1) return fail(c, DR_EINVAL, "reach_ct needs a field with an input (n_u >= 1)");
  if (nd.n[0] != f->n || nd.n_state != f->n_u)
    return fail(c, DR_ESHAPE, "the controller context needs n_0 = n (the state) and n_state = n_u (its outputs)");
  if ((st = check_batch(c, b)) != DR_OK) return st;
  if (b->split_ptr) return fail(c, DR_EINVAL, "reach_ct takes no split constraints");
  if (!boxes) return fail(c, DR_EINVAL, "boxes is NULL");
  if (!c->ct_fn) return fail(c, DR_ESHAPE, "no kernel instance for this width, or its on-chip state does not fit");
  c->batch.n_sub = b->n_sub;
  c->batch.net_id = b->net_id;
  c->batch.xc = b->x_center;
  c->batch.xr = b->x_radius;
  c->batch.sptr = nullptr;
  c->batch.spk = nullptr;
  c->have_batch = false;  // bound_init state is not valid for this batch
  c->fused_ready = false;
  c->sc.n_sub = b->n_sub;
  if (b->n_sub == 0) return DR_OK;
  dr::CtArgs ca = ct_args(f, o, boxes, segs, status);
  ca.batch = c->batch; ca.sc = c->sc; ca.sc.st_out = nullptr;
  ca.state = c->ct_state;
  // per control interval: certify every box's controller, then K held-input flowpipe
  // steps of every box (the state stays in c->ct_state between the launches)
  int nb = 0;
  const size_t flds = dr::CtLds::bytes(f->n_u);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)dr::k_flowpipe_ct_held, 64, flds) != hipSuccess ||
      nb < 1)
    nb = 1;
  const int fgrid = (int)std::min<long long>((long long)nb * c->cus, b->n_sub);
  const int cgrid = std::min(c->ct_grid, b->n_sub);
  int net_index = 0;
  for (int k = 0; k < std::max(o->intervals, 1); ++k) {
    int seed = k == 0 ? 1 : 0, control = o->intervals > 0 ? 1 : 0;
    void* args[] = {&c->dnet, &net_index, &ca, &seed, &control};
    if ((st = launch(c, c->ct_fn, cgrid, c->ct_lds, args, stream)) != DR_OK) return st;
    if (!control) break;
    hipLaunchKernelGGL(dr::k_flowpipe_ct_held, dim3(fgrid), dim3(64), flds, stream, ca, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  }
  return DR_OK;
}

dr_status dr_get_bounds(dr_ctx* c, double* l, double* u, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!l || !u) return fail(c, DR_EINVAL, "l/u is NULL");
  const int S = c->batch.n_sub;
  if (S == 0 || c->H_max == 0) return DR_OK;
  const int tot = S * c->H_max;
  hipLaunchKernelGGL(dr::k_export_bounds, dim3((tot + 255) / 256), dim3(256), 0, stream, S, c->Hp_max, c->H_max,
                     c->dnet, c->n_nets, c->sc.direct, c->batch.net_id, c->sc.bl, c->sc.bu, l, u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "export kernel");
  return DR_OK;
}

dr_status dr_get_rows(dr_ctx* c, int* rows, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!rows) return fail(c, DR_EINVAL, "rows is NULL");
  if (c->batch.n_sub == 0) return DR_OK;
  hipError_t e = hipMemcpyAsync(rows, c->sc.rows, sizeof(int) * 8 * c->batch.n_sub, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(c, e, "rows copy");
  return DR_OK;
}

dr_status dr_get_margins(dr_ctx* c, double* margin, hipStream_t stream) {
  if (!c) return fail(nullptr, DR_EINVAL, "ctx is NULL");
  if (!margin) return fail(c, DR_EINVAL, "margin is NULL");
  const int S = c->batch.n_sub;
  if (S == 0) return DR_OK;
  hipError_t e = hipMemcpy2DAsync(margin, sizeof(double) * c->R, c->sc.margin, sizeof(double) * 32,
                                  sizeof(double) * c->R, S, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(c, e, "margin copy");
  return DR_OK;
}

int dr_hidden_max(const dr_ctx* c) { return c ? c->H_max : 0; }
int dr_spec_rows(const dr_ctx* c) { return c ? c->R : 0; }

const char* dr_last_error(const dr_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void dr_destroy(dr_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (void* p : c->allocs) (void)hipFree(p);
  for (int i = 0; i < kMaxNets; ++i) {
    if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
    if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  delete c;
}

}  // extern "C"
