// gfx950 kernel of the continuous-time closed loop with an NN controller (Algorithm
// "Reachability of CT NN Control Systems"): at every control boundary the controller is
// certified on the state's Taylor model by the TM-CROWN interface of the stepwise reach
// (Theorem "CROWN bounds of NN with linear TM input": the step of k_reach_dt for the
// loop u = 0 x + I f(x), all four waves, matrix cores), giving a linear model of u over
// the same generators; the first wavefront then runs K flowpipe steps of x' = f(x, u)
// with u held (zero-order hold; ct_flow.hpp).  One workgroup per box.
#pragma once
#include "bound_kernels.hpp"
#include "ct_flow.hpp"

namespace dr {

template <typename T, int NT>
__global__ void __launch_bounds__(kWG) k_reach_ct(const NetDev* __restrict__ nets, int net_index, CtArgs ca) {
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
  CtLds C;
  C.carve((double*)(lds_base + SubLds<T>::bytes(Hp, NT) + kReachExtraLds + (((size_t)Hp * sizeof(T) + 15) & ~(size_t)15)));
  const int n = ca.dyn.n, n_u = ca.dyn.n_u, n0 = net.n[0];
  const int N = ca.n_ctl * ca.K;
  for (int b = blockIdx.x; b < ca.batch.n_sub; b += gridDim.x) {
    if (wid == 0) {
      ct_seed(C, ca, b, n0);
      if (tid < n) {
        double lo, hi;
        ct_point_box(C, tid, lo, hi);
        double* bo = ca.boxes + (size_t)b * (N + 1) * n * 2;
        bo[tid * 2 + 0] = lo; bo[tid * 2 + 1] = hi;
      }
    }
    for (int p = tid; p < Hp; p += kWG) S.slot[p] = -1;
    if (tid == 0) S.misc[1] = 0;
    if (tid < 8) sc.rows[(size_t)b * 8 + tid] = 0;
    lds_barrier();
    for (int k = 0; k < ca.n_ctl; ++k) {
      // ---- the controller on the state's model: tm = (c, S, lo, hi, |x| bound)
      for (int e = tid; e < 256; e += kWG) tm[16 + e] = C.S[e];
      if (tid < 16) {
        tm[tid] = C.c[tid]; tm[272 + tid] = C.lo[tid]; tm[288 + tid] = C.hi[tid];
        double a = fabs(C.c[tid]) + fmax(fabs(C.lo[tid]), fabs(C.hi[tid]));
        for (int z = 0; z < n0; ++z) a += fabs(C.S[tid * 16 + z]);
        tm[304 + tid] = tid < n0 ? a : 0.0;
        S.xc[tid] = 0.0; S.xr[tid] = 0.0;
      }
      lds_barrier();
      tm_crown_step<T, NT>(net, sc, S, stage, lds_b, tm, nullptr, 0, 1, b, nullptr);
      lds_barrier();
      // the input's model: centre + midpoint of the interval part, linear part over y
      if (tid < 16) {
        const double* nc = tm + 320;
        const double* nIlo = tm + 592;
        const double* nIhi = tm + 608;
        const bool v = tid < n_u;
        const double mid = v ? 0.5 * (nIlo[tid] + nIhi[tid]) : 0.0, rad = v ? 0.5 * (nIhi[tid] - nIlo[tid]) : 0.0;
        C.U.c[tid] = v ? nc[tid] + mid : 0.0;
        C.U.lo[tid] = -rad; C.U.hi[tid] = rad;
        C.U.l[tid] = 0.0; C.U.w[tid] = 0.0;
      }
      for (int e = tid; e < 256; e += kWG) {
        C.U.L[e] = (e / 16) < n_u ? tm[336 + e] : 0.0;
        C.U.M[e] = 0.0;
      }
      lds_barrier();
      // ---- K flowpipe steps with the input held (wave 0)
      if (wid == 0) {
        const bool ok = ct_steps(C, ca, true, b, k * ca.K);
        if (tid == 0 && !ok) atomicOr(&S.misc[1], DR_RES_NONFINITE);
      }
      lds_barrier();
    }
    if (tid == 0 && ca.status) ca.status[b] = (uint32_t)S.misc[1];
    lds_barrier();
  }
}

}  // namespace dr
