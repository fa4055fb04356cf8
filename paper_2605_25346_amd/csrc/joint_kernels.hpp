// gfx950 kernel of CROWN through the closed loop unrolled over the horizon (the
// joint, non-truncated DT reachability that the paper compares its stepwise engine
// with, Section "Reachability Tool Evaluations"): every hidden neuron of step t is
// bounded by rows carried back through all earlier steps to the initial box, and the
// state box of x_{t+1} by rows +-e_i on x_{t+1} carried back the same way.
//
// The graph: v_t = [x_t; u_t] (u_t given), x_{t+1} = A v_t + B f(v_t).  Rows lam on
// x_{s+1} pass step s as
//   lam . x_{s+1} = (lam A) . v_s + (lam B W_L) . h_{L-1} + lam B b_L,
// so one step back is: g = lam M (M = B W_L, a 16-row product on the matrix cores),
// the CROWN chain of the network of step s from h_{L-1} down to its input (that
// step's relaxation), the skip product lam A added to the input coefficients, and the
// exogenous coefficients times u_s moved into the offset.
//
// One workgroup per box (static assignment, the boxes cost the same); the relaxation
// of every step so far stays in LDS, so the launch needs H x (hidden neurons) x 4
// values of the chain type on chip.
#pragma once
#include "bound_kernels.hpp"

namespace dr {

// Rows lam (one 16-row tile, B-operand layout of a 16-wide input) on x_{s0+1} carried
// back through steps s0, ..., 0: on return lam holds the coefficients on x_0, acc the
// lane's share of the offsets and marg its share of the rounding margin.
template <typename T, int NT>
__device__ __forceinline__ void joint_back(const NetDev& net, const JointLds<T>& J, int Hp, int s0, T (&lam)[1][4],
                                           double& acc, T& marg, char* stage, int lane) {
  const int gq = lane >> 4, ns = net.n_state;
  gconst<V4<T>> Mw = as_global(uniform_ptr((const V4<T>*)net.jM));
  gconst<V4<T>> Aw = as_global(uniform_ptr((const V4<T>*)net.jA));
  for (int s = s0; s >= 0; --s) {
    // the step boundary: offsets lam . (B b_L) and the margin of the products lam M, lam A
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = nrn<T>(gq, i);
      if (m < ns) {
        acc += (double)lam[0][i] * net.seedB[m];
        marg += fabs(lam[0][i]) * J.mux[s * 16 + m];
      }
    }
    T g[NT][4], sk[1][4];
    gemm_k<T, NT, 1>(Mw, RegArr<T, 1>{lam}, g, lane);
    gemm_k<T, 1, 1>(Aw, RegArr<T, 1>{lam}, sk, lane);
    auto st = make_stage<T, NT>(stage, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) st.set(t, i, g[t][i]);
    T w[1][4];
    double acc2 = 0.0;
    chain_to_input<T, NT, false>(net, net.L, st, J.rel + (size_t)s * Hp, acc, acc2, marg, w, lane, J.bias);
    // input coefficients of step s: the chain's plus the skip; exogenous ones become offsets
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = nrn<T>(gq, i);
      const T lf = w[0][i] + sk[0][i];
      const double uu = J.uv[s * 16 + m];
      acc += (double)lf * uu;
      // rounding of the sum (relative 2^-24 / 2^-53 of |lf| on |v_s|) and of the FP64 offset
      marg += fabs(lf) * rup<T>(unit_round<T>() * J.vab[s * 16 + m] + 0x1p-42 * fabs(uu));
      lam[0][i] = m < ns ? lf : (T)0;
    }
  }
}

// Lower bound of one tile of rows (lam on x_0, offsets and margin per lane) over the
// initial box; every lane of a row returns the row's bound.
template <typename T>
__device__ __forceinline__ double joint_concretize(const JointLds<T>& J, const T (&lam)[1][4], double acc, T marg,
                                                   int gq, int margin_on) {
  double base = 0.0, wabs = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = nrn<T>(gq, i);
    const double wm = (double)lam[0][i];
    base += wm * J.box[m] - fabs(wm) * J.box[16 + m];
    wabs += fabs(wm) * (fabs(J.box[m]) + J.box[16 + m]);
  }
  base = row_sum(base); wabs = row_sum(wabs); acc = row_sum(acc);
  const double mg = margin_on ? (double)row_sum(marg) * kMargInflate + 0x1p-46 * (wabs + fabs(acc)) : 0.0;
  return acc + base - mg;
}

template <typename T, int NT>
__global__ void __launch_bounds__(kWG) k_reach_joint(const NetDev* __restrict__ nets, int net_index, JointArgs ja) {
  extern __shared__ __align__(16) char lds_raw[];
  const NetDev& net = nets[net_index];
  const Scratch& sc = ja.sc;
  const int L = net.L, Hp = net.Hp, H = ja.horizon;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, gq = lane >> 4;
  char* stage = lds_raw + (size_t)wid * stage_bytes<T, NT>();
  JointLds<T> J;
  J.carve(lds_raw + kWavesPerWG * stage_bytes<T, NT>(), H, Hp, NT);
  for (int e = tid; e < Hp; e += kWG) {
    const int k = e / (16 * NT);
    J.bias[e] = as_global((const T*)net.bn[k])[e - k * 16 * NT];
  }
  const int n0 = net.n[0], ns = net.n_state, nx = n0 - ns;
  const int S = ja.batch.n_sub;
  const int margin_on = sc.margin_on;
  double* Xc0 = J.box;
  double* Xr0 = J.box + 16;
  double* Xlo = J.box + 32;
  double* Xhi = J.box + 48;
  double* Vc = J.box + 64;
  double* Vr = J.box + 80;

  for (int b = blockIdx.x; b < S; b += gridDim.x) {
    double* bx = ja.boxes + (size_t)b * (H + 1) * ns * 2;
    if (tid < 16) {
      const double cc = tid < ns ? ja.batch.xc[(size_t)b * n0 + tid] : 0.0;
      const double rr = tid < ns ? ja.batch.xr[(size_t)b * n0 + tid] : 0.0;
      Xc0[tid] = cc; Xr0[tid] = rr;
      Xlo[tid] = cc - rr; Xhi[tid] = cc + rr;
      if (tid < ns) { bx[tid * 2 + 0] = cc - rr; bx[tid * 2 + 1] = cc + rr; }
    }
    if (tid == 0) J.misc[1] = 0;
    lds_barrier();
    if (tid < 16 && tid < ns && (!(fabs(Xc0[tid]) < INFINITY) || !(Xr0[tid] < INFINITY)))
      atomicOr(&J.misc[1], DR_RES_NONFINITE);
    for (int t = 0; t < H; ++t) {
      V4<T>* rel_t = J.rel + (size_t)t * Hp;
      // the input box of step t: the state box and the given exogenous inputs
      if (tid < 16) {
        double uu = 0.0, lo = 0.0, hi = 0.0;
        if (tid < ns) {
          lo = Xlo[tid]; hi = Xhi[tid];
        } else if (tid < n0) {
          uu = ja.u[((size_t)b * H + t) * nx + (tid - ns)];
          lo = hi = uu;
        }
        J.uv[t * 16 + tid] = uu;
        J.vab[t * 16 + tid] = fmax(fabs(lo), fabs(hi));
        Vc[tid] = 0.5 * (lo + hi);
        Vr[tid] = 0.5 * (hi - lo);
      }
      lds_barrier();
      // ---- layer 1: the affine range over the input box (exact at t = 0)
      const int n1 = net.n[1];
      for (int j = tid; j < 16 * NT; j += kWG) {
        double lo = 0.0, hi = 0.0, v = 0.0;
        if (j < n1) {
          gconst<T> W = as_global((const T*)net.Wn[0] + (size_t)j * net.np[0]);
          double zc = (double)J.bias[j], zr = 0.0, za = 0.0;
          for (int m = 0; m < n0; ++m) {
            const double w = (double)W[m];
            zc += w * Vc[m];
            zr += fabs(w) * Vr[m];
            za += fabs(w) * J.vab[t * 16 + m];
          }
          const double e = 0x1p-44 * (za + zr + fabs(zc));
          lo = zc - zr - e; hi = zc + zr + e; v = za;
        }
        J.ibl[j] = lo; J.ibu[j] = hi; J.v[j] = v;
        J.l[j] = lo; J.u[j] = hi;
      }
      lds_barrier();
      int nU = 0;
      if (t > 0) {
        auto unstable = [&](int j) { return j < n1 && J.ibl[j] < 0.0 && J.ibu[j] > 0.0; };
        nU = compact_flags<kWG>(16 * NT, unstable, J.U, J.misc + 2);
        const int ntiles = (2 * nU + 15) >> 4;
        for (int tile = wid; tile < ntiles; tile += kWavesPerWG) {
          const int row = tile * 16 + (lane & 15);
          const bool valid = row < 2 * nU;
          const int neuron = valid ? J.U[row < nU ? row : row - nU] : 0;
          const T sg = valid ? (row < nU ? (T)1 : (T)-1) : (T)0;
          // rows +-e_j on z_1 are +-W_1[j, :] on v_t
          gconst<T> Wr = as_global((const T*)net.Wn[0] + (size_t)neuron * net.np[0]);
          T lam[1][4];
          T marg = 0;
          double acc = gq == 0 ? (double)sg * (double)J.bias[neuron] : 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = nrn<T>(gq, i);
            const T x = sg * Wr[m];
            acc += (double)x * J.uv[t * 16 + m];
            marg += fabs(x) * rup<T>(0x1p-42 * fabs(J.uv[t * 16 + m]));
            lam[0][i] = m < ns ? x : (T)0;
          }
          joint_back<T, NT>(net, J, Hp, t - 1, lam, acc, marg, stage, lane);
          const double lb = joint_concretize<T>(J, lam, acc, marg, gq, margin_on);
          if (valid && lane < 16) {
            if (row < nU) J.l[neuron] = fmax(J.ibl[neuron], lb);
            else J.u[neuron] = fmin(J.ibu[neuron], -lb);
          }
        }
        lds_barrier();
      }
      if (tid == 0 && ja.rows) ja.rows[((size_t)b * H + t) * 8 + 0] = 2 * nU;
      for (int j = tid; j < 16 * NT; j += kWG) {
        const int p = (j & ~15) + pos_of<T>(j & 15);
        const double lo = J.l[j], hi = J.u[j];
        if (j < n1 && (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY))) atomicOr(&J.misc[1], DR_RES_NONFINITE);
        rel_t[p] = build_relax<T>(lo, hi, J.v[j], j < n1 ? (double)J.bias[j] : 0.0, false, n1, false, margin_on);
      }
      lds_barrier();
      // ---- deeper hidden layers: IBP, then CROWN rows of the unstable neurons to x_0
      for (int k = 2; k <= L - 1; ++k) {
        const int nk = net.n[k];
        const int base = (k - 1) * 16 * NT, pbase = (k - 2) * 16 * NT;
        relu_box<kWG>(J.l + pbase, J.u + pbase, 16 * NT, J.hc, J.hr);
        lds_barrier();
        if (tid < 16 * NT) {
          const int j = tid;
          double lo = 0.0, hi = 0.0, v = 0.0;
          if (j < nk) ibp_neuron<T, NT>(net, k, j, J.hc, J.hr, lo, hi, v);
          J.ibl[j] = lo; J.ibu[j] = hi; J.v[j] = v;
          J.l[base + j] = lo; J.u[base + j] = hi;
        }
        lds_barrier();
        auto unstable = [&](int j) { return j < nk && J.ibl[j] < 0.0 && J.ibu[j] > 0.0; };
        const int nUk = compact_flags<kWG>(16 * NT, unstable, J.U, J.misc + 2);
        const int ntiles = (2 * nUk + 15) >> 4;
        for (int tile = wid; tile < ntiles; tile += kWavesPerWG) {
          const int row = tile * 16 + (lane & 15);
          const bool valid = row < 2 * nUk;
          const int neuron = valid ? J.U[row < nUk ? row : row - nUk] : 0;
          const T sg = valid ? (row < nUk ? (T)1 : (T)-1) : (T)0;
          auto g = make_stage<T, NT>(stage, lane);
          gconst<T> Wr = as_global((const T*)net.Wn[k - 1] + (size_t)neuron * net.np[k - 1]);
#pragma unroll
          for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int i = 0; i < 4; ++i) g.set(tt, i, sg * Wr[tt * 16 + nrn<T>(gq, i)]);
          double acc = gq == 0 ? (double)sg * (double)J.bias[base + neuron] : 0.0, acc2 = 0.0;
          T marg = 0;
          T w[1][4];
          chain_to_input<T, NT, false>(net, k, g, rel_t, acc, acc2, marg, w, lane, J.bias);
          T lam[1][4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = nrn<T>(gq, i);
            acc += (double)w[0][i] * J.uv[t * 16 + m];
            marg += fabs(w[0][i]) * rup<T>(0x1p-42 * fabs(J.uv[t * 16 + m]));
            lam[0][i] = m < ns ? w[0][i] : (T)0;
          }
          joint_back<T, NT>(net, J, Hp, t - 1, lam, acc, marg, stage, lane);
          const double lb = joint_concretize<T>(J, lam, acc, marg, gq, margin_on);
          if (valid && lane < 16) {
            if (row < nUk) J.l[base + neuron] = fmax(J.ibl[neuron], lb);
            else J.u[base + neuron] = fmin(J.ibu[neuron], -lb);
          }
        }
        lds_barrier();
        if (tid < 16 * NT) {
          const int j = tid;
          const int p = base + (j & ~15) + pos_of<T>(j & 15);
          const double lo = J.l[base + j], hi = J.u[base + j];
          if (j < nk && (!(fabs(lo) < INFINITY) || !(fabs(hi) < INFINITY))) atomicOr(&J.misc[1], DR_RES_NONFINITE);
          rel_t[p] = build_relax<T>(lo, hi, J.v[j], j < nk ? (double)J.bias[base + j] : 0.0, false, nk, false,
                                    margin_on);
        }
        if (tid == 0 && ja.rows) ja.rows[((size_t)b * H + t) * 8 + (k - 1)] = 2 * nUk;
        lds_barrier();
      }
      // ---- margin coefficients of the step boundary of step t, per state index r:
      // the products g = lam M (M = B W_L held as seedT with entry error seedM) and
      // lam A (A rounded to the chain type), gamma_32 each, on |h_{L-1}| and |v_t|, plus
      // the FP64 seed offset B_r b_L (error seedBe)
      if (tid < 16) {
        const int r = tid;
        double mu = 0.0;
        if (margin_on && r < ns) {
          const int npl = net.np[L - 1], lbase = (L - 2) * 16 * NT;
          gconst<T> Mr = as_global((const T*)net.seedT + (size_t)r * npl);
          gconst<T> Me = as_global((const T*)net.seedM + (size_t)r * npl);
          const double gam = gamma_n<T>(32);
          for (int m = 0; m < net.n[L - 1]; ++m)
            mu += (gam * fabs((double)Mr[m]) + (double)Me[m]) * fmax(J.u[lbase + m], 0.0);
          for (int m = 0; m < n0; ++m)
            mu += (gam * (1.0 + unit_round<T>()) + unit_round<T>()) * fabs(net.skip[(size_t)r * 16 + m]) * J.vab[t * 16 + m];
          mu += net.seedBe[r] + 0x1p-42 * fabs(net.seedB[r]);
          mu *= 1.0 + 0x1p-40;
        }
        J.mux[t * 16 + r] = rup<T>(mu);
      }
      lds_barrier();
      // ---- the state box of x_{t+1}: rows +-e_r on x_{t+1} carried back to x_0
      const int srows = 2 * ns, stiles = (srows + 15) >> 4;
      for (int tile = wid; tile < stiles; tile += kWavesPerWG) {
        const int row = tile * 16 + (lane & 15);
        const bool valid = row < srows;
        const int r = valid ? (row < ns ? row : row - ns) : 0;
        const T sg = valid ? (row < ns ? (T)1 : (T)-1) : (T)0;
        T lam[1][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) lam[0][i] = nrn<T>(gq, i) == r ? sg : (T)0;
        double acc = 0.0;
        T marg = 0;
        joint_back<T, NT>(net, J, Hp, t, lam, acc, marg, stage, lane);
        const double lb = joint_concretize<T>(J, lam, acc, marg, gq, margin_on);
        if (valid && lane < 16) {
          double* bo = bx + (size_t)(t + 1) * ns * 2;
          if (row < ns) { Xlo[r] = lb; bo[r * 2 + 0] = lb; }
          else { Xhi[r] = -lb; bo[r * 2 + 1] = -lb; }
          if (!(fabs(lb) < INFINITY)) atomicOr(&J.misc[1], DR_RES_NONFINITE);
        }
      }
      if (tid == 0 && ja.rows) ja.rows[((size_t)b * H + t) * 8 + (L - 1)] = srows;
      lds_barrier();
    }
    if (tid == 0) {
      if (ja.status) ja.status[b] = (uint32_t)J.misc[1];
      sc.st[b] = (uint32_t)J.misc[1];
    }
    lds_barrier();
  }
}

}  // namespace dr
