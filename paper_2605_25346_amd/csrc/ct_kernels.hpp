// gfx950 controller step of the continuous-time closed loop with an NN controller
// (Algorithm "Reachability of CT NN Control Systems").  The loop alternates two launches
// per control interval over the whole batch: this kernel certifies every box's
// controller on the box's current state model by the TM-CROWN step of the stepwise
// reach (Theorem "CROWN bounds of NN with linear TM input": the step of k_reach_dt for
// the loop u = A x + B f(x), one workgroup per box, the matrix cores), writing a linear
// model of u over the same generators; then k_flowpipe_ct_held (aux_kernels.hpp) runs K
// flowpipe steps of every box with u held (zero-order hold; ct_flow.hpp).  Between the
// launches each box's state lives in global memory (kCtState doubles, ct_flow.hpp).
#pragma once
#include "bound_kernels.hpp"
#include "ct_flow.hpp"

namespace dr {

// seed: write the initial state of every box (centre, diag(radius), no remainder) and the
// box of time point 0, and clear the box's status and row counts; control: certify the
// controller on the state and write the input's model.
template <typename T, int NT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(reach_waves_per_eu<T, NT>())))
k_ct_control(const NetDev* __restrict__ nets, int net_index, CtArgs ca, int seed, int control) {
  extern __shared__ __align__(16) char lds_raw[];
  const NetDev& net = nets[net_index];
  const Scratch& sc = ca.sc;
  const int Hp = net.Hp;
  const int tid = threadIdx.x, wid = tid >> 6;
  char* stage = lds_raw + (size_t)wid * stage_bytes<T, NT>();
  char* lds_base = lds_raw + kWavesPerWG * stage_bytes<T, NT>();
  SubLds<T> S;
  S.carve(lds_base, Hp, NT);
  T* lds_b = (T*)(lds_base + SubLds<T>::bytes(Hp, NT) + kReachExtraLds);
  stage_biases<T, T>(net, lds_b);
  double* tm = (double*)(lds_base + ((SubLds<T>::bytes(Hp, NT) + 64 + 15) & ~(size_t)15));
  const int n = ca.dyn.n, n_u = ca.dyn.n_u, n0 = net.n[0];
  const int N = ca.n_ctl * ca.K;
  for (int b = blockIdx.x; b < ca.batch.n_sub; b += gridDim.x) {
    double* st = ca.state + (size_t)b * kCtState;
    // ---- the state model: tm = (c, S, lo, hi), from the box or from the last interval
    if (seed) {
      if (tid < 16) {
        const bool v = tid < n;
        const double cc = v ? ca.batch.xc[(size_t)b * n0 + tid] : 0.0, rr = v ? ca.batch.xr[(size_t)b * n0 + tid] : 0.0;
        tm[tid] = cc; tm[272 + tid] = 0.0; tm[288 + tid] = 0.0;
        st[tid] = cc; st[272 + tid] = 0.0; st[288 + tid] = 0.0;
        if (v) {
          double* bo = ca.boxes + (size_t)b * (N + 1) * n * 2;
          bo[tid * 2 + 0] = cc - rr; bo[tid * 2 + 1] = cc + rr;
        }
      }
      for (int e = tid; e < 256; e += kWG) {
        const int r = e >> 4, z = e & 15;
        const double v = (r == z && r < n) ? ca.batch.xr[(size_t)b * n0 + r] : 0.0;
        tm[16 + e] = v; st[16 + e] = v;
      }
      if (tid < 8) sc.rows[(size_t)b * 8 + tid] = 0;
      if (tid == 0 && ca.status) ca.status[b] = 0u;
    } else {
      for (int e = tid; e < 304; e += kWG) tm[e] = st[e];
    }
    if (!control) continue;
    for (int p = tid; p < Hp; p += kWG) S.slot[p] = -1;
    if (tid == 0) S.misc[1] = 0;
    lds_barrier();
    if (tid < 16) {
      double a = fabs(tm[tid]) + fmax(fabs(tm[272 + tid]), fabs(tm[288 + tid]));
      for (int z = 0; z < n0; ++z) a += fabs(tm[16 + tid * 16 + z]);
      tm[304 + tid] = tid < n0 ? a : 0.0;
      S.xc[tid] = 0.0; S.xr[tid] = 0.0;
    }
    lds_barrier();
    tm_crown_step<T, NT>(net, sc, S, stage, lds_b, tm, nullptr, 0, 1, b, nullptr);
    lds_barrier();
    // the input's model: centre + midpoint of the interval part, linear part over y
    if (tid < 16) {
      const bool v = tid < n_u;
      const double lo = tm[592 + tid], hi = tm[608 + tid];
      const double mid = v ? 0.5 * (lo + hi) : 0.0, rad = v ? 0.5 * (hi - lo) : 0.0;
      st[304 + tid] = v ? tm[320 + tid] + mid : 0.0;
      st[576 + tid] = -rad;
      st[592 + tid] = rad;
    }
    for (int e = tid; e < 256; e += kWG) st[320 + e] = (e >> 4) < n_u ? tm[336 + e] : 0.0;
    if (tid == 0 && ca.status && S.misc[1]) ca.status[b] |= (uint32_t)S.misc[1];
    lds_barrier();
  }
}

}  // namespace dr
