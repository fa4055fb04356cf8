// gfx950 kernel of the continuous-time closed loop with an NN controller (Algorithm
// "Reachability of CT NN Control Systems").  A workgroup (four wavefronts) carries up to
// four boxes.  At every control boundary each box's controller is certified on the box's
// Taylor model by the TM-CROWN step of the stepwise reach (Theorem "CROWN bounds of NN
// with linear TM input": the step of k_reach_dt for the loop u = A x + B f(x), all four
// wavefronts and the matrix cores, one box after the other), giving a linear model of u
// over the same generators; then every wavefront runs K flowpipe steps of its own box
// with u held (zero-order hold; ct_flow.hpp).
#pragma once
#include "bound_kernels.hpp"
#include "ct_flow.hpp"

namespace dr {

// LDS of k_reach_ct after the stepwise reach's: the bias block rounded to 16 bytes, then
// one flowpipe state per box, then the boxes' status words (16 bytes).
template <typename T>
__host__ __device__ constexpr size_t ct_bias_bytes(int Hp) { return ((size_t)Hp * sizeof(T) + 15) & ~(size_t)15; }

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
  char* ct_base = lds_base + SubLds<T>::bytes(Hp, NT) + kReachExtraLds + ct_bias_bytes<T>(Hp);
  const int nb = ca.boxes_per_wg;
  CtLds C;   // the flowpipe state of this wavefront's box
  C.carve((double*)(ct_base + (size_t)min(wid, nb - 1) * CtLds::bytes(true)), true);
  int* box_st = (int*)(ct_base + (size_t)nb * CtLds::bytes(true));   // status bits per box
  const int n = ca.dyn.n, n_u = ca.dyn.n_u, n0 = net.n[0];
  if (wid < nb) ct_pairs(C, ca.dyn);
  for (int b0 = blockIdx.x * nb; b0 < ca.batch.n_sub; b0 += gridDim.x * nb) {
    const int nbox = min(nb, ca.batch.n_sub - b0);
    if (wid < nbox) ct_seed(C, ca, b0 + wid, n0);
    if (tid < kWavesPerWG) box_st[tid] = 0;
    for (int p = tid; p < Hp; p += kWG) S.slot[p] = -1;
    if (tid < 8 * nbox) sc.rows[(size_t)b0 * 8 + tid] = 0;
    lds_barrier();
    for (int k = 0; k < ca.n_ctl; ++k) {
      for (int q = 0; q < nbox; ++q) {
        // ---- the controller of box b0 + q on its state's model: tm = (c, S, lo, hi, |x| bound)
        CtLds Cq;
        Cq.carve((double*)(ct_base + (size_t)q * CtLds::bytes(true)), true);
        for (int e = tid; e < 256; e += kWG) tm[16 + e] = Cq.S[(e >> 4) * kCtLd + (e & 15)];
        if (tid < 16) {
          tm[tid] = Cq.c[tid]; tm[272 + tid] = Cq.lo[tid]; tm[288 + tid] = Cq.hi[tid];
          double a = fabs(Cq.c[tid]) + fmax(fabs(Cq.lo[tid]), fabs(Cq.hi[tid]));
          for (int z = 0; z < n0; ++z) a += fabs(Cq.S[tid * kCtLd + z]);
          tm[304 + tid] = tid < n0 ? a : 0.0;
          S.xc[tid] = 0.0; S.xr[tid] = 0.0;
        }
        if (tid == 0) S.misc[1] = 0;
        lds_barrier();
        tm_crown_step<T, NT>(net, sc, S, stage, lds_b, tm, nullptr, 0, 1, b0 + q, nullptr);
        lds_barrier();
        // the input's model: centre + midpoint of the interval part, linear part over y
        if (tid < 16) {
          const double* nc = tm + 320;
          const double* nIlo = tm + 592;
          const double* nIhi = tm + 608;
          const bool v = tid < n_u;
          const double mid = v ? 0.5 * (nIlo[tid] + nIhi[tid]) : 0.0, rad = v ? 0.5 * (nIhi[tid] - nIlo[tid]) : 0.0;
          Cq.U.c[tid] = v ? nc[tid] + mid : 0.0;
          Cq.U.lo[tid] = -rad; Cq.U.hi[tid] = rad;
          Cq.U.l[tid] = 0.0; Cq.U.w[tid] = 0.0;
        }
        for (int e = tid; e < 256; e += kWG) {
          const int r = e >> 4, z = e & 15;
          Cq.U.L[r * kCtLd + z] = r < n_u ? tm[336 + e] : 0.0;
          Cq.U.M[r * kCtLd + z] = 0.0;
        }
        if (tid == 0) box_st[q] |= S.misc[1];
        lds_barrier();
      }
      // ---- K flowpipe steps of every box with its input held (one wavefront per box)
      if (wid < nbox) {
        const bool ok = ct_steps(C, ca, true, b0 + wid, k * ca.K);
        if ((tid & 63) == 0 && !ok) box_st[wid] |= DR_RES_NONFINITE;
      }
      lds_barrier();
    }
    if (tid < nbox && ca.status) ca.status[b0 + tid] = (uint32_t)box_st[tid];
    lds_barrier();
  }
}

}  // namespace dr
