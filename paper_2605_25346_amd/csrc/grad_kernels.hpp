// gfx950 kernel of the reverse pass through the stepwise TM reach: the gradient of
// J = sum_s gV_s V_s, V_s the tube volume of box s (sum over steps t = 1..H and states
// of the widths of X_t), the quantity the paper's reachability-aware loss is built on
// (Section "Certified training of neural dynamics and controllers"; the top-candidate
// refinement of Section "Reachability-aware MPC" uses its gradient w.r.t. the actions).
//
// The forward reach (k_reach_dt with a tape) records per box and step the Taylor model
// entering the step and the final and interval bounds of every hidden neuron.  This
// kernel walks the steps backwards, one workgroup per box.  Per step, with the
// cotangent of the Taylor model leaving the step (c', P', I') given:
//   * output rows (x' = A v + B y, shared slope): recompute each row's chain with a
//     record of its multipliers g, then the Taylor-model composition in reverse
//     (cotangents of W_r = A_r + w_r, of the incoming model, of the offsets), then the
//     chain in reverse on the matrix cores with the adjoint-swizzled weights; every
//     relaxed neuron collects d/ds and d/dt (summed over the rows);
//   * hidden layers from the last to the first: d/ds, d/dt become d/dl, d/du through
//     the chord (s = u/(u-l), t = -s l); the side of the intersection that won takes
//     the cotangent: an interval bound passes it to the previous layer's bounds (IBP in
//     reverse), a CROWN row runs its chain in reverse like an output row, and layer 1
//     (the exact range of W_1 over the model) passes it to the incoming model;
//   * the incoming model's cotangent is the next (earlier) step's; its exogenous centre
//     entries are the gradient w.r.t. the actions, and at step 0 the centre and the
//     diagonal of P give the gradient w.r.t. the box centre and radius.
// Rounding margins are treated as constants (the gradient is that of the bound in exact
// arithmetic); discrete choices (stability, intersection side, signs) are those of the
// forward pass.
#pragma once
#include "bound_kernels.hpp"

namespace dr {

// Sum of v over the 16 rows of a tile (the 16 lanes of a lane group).
__device__ __forceinline__ double sum16(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  return v;
}

// Weight gradient: the workgroup's region (null when not asked for), and the wave's LDS
// blocks and row cotangents for the products of one row tile.
template <typename T>
struct WgradTile {
  T* reg;             // LDS accumulator or global region
  bool lds;           // reg is the LDS accumulator
  const size_t* woff;
  lmut<T> A;          // 16 rows x 16 outputs of W_k
  lmut<T> B;          // 16 rows x 16 inputs of W_k
  lmut<double> rho;   // 16: the rows' offset cotangents (both offsets)
};

// reg[off] += v with the address space spelled out, so that the LDS accumulator takes
// the LDS unit's atomic and the global region the global one (a generic pointer would
// take the flat path for both)
template <typename T>
__device__ __forceinline__ void wacc_add(const WgradTile<T>& W, size_t off, T v) {
  if (W.lds)
    __hip_atomic_fetch_add((lmut<T>)(W.reg + off), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_fetch_add((gmut<T>)(W.reg + off), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// dW_k += sum_r a(r, i) b(r, j) (and db_k += sum_r rho_r a(r, i) when `bias`): the tile's
// rows are the summation index; each 16 x 16 block of outputs is one product a^T b on the
// matrix cores (four 16x16x4 steps over the 16 rows) from LDS copies of a 16 x 16 block
// of a and of b (each lane stages its own four values of a block), the lane then holding
// outputs (nrn(g, c), r) of the block, added atomically to the region.
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void wgrad_blocks(const WgradTile<T>& W, int k, int ld, int ti, int tj, int ni, int nj,
                                             FA a_of, FB b_of, bool bias, int lane) {
  const int r = lane & 15, g = lane >> 4;
  const size_t reg = W.woff[k - 1];
  for (int it = 0; it < ti; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) W.A[r * 16 + nrn<T>(g, i)] = a_of(it, i);
    for (int jt = 0; jt < tj; ++jt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) W.B[r * 16 + nrn<T>(g, i)] = b_of(jt, i);
      sub_sync<64>();
      // D[i][j] = sum_rows A[row][i] B[row][j]: in step s lane group g brings row 4 s + g
      // (output r of A, input r of B)
      V4<T> acc{0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int row = 4 * s4 + g;
        acc = mfma16(W.A[row * 16 + r], W.B[row * 16 + r], acc);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = it * 16 + nrn<T>(g, c), j = jt * 16 + r;
        if (i < ni && j < nj && acc[c] != (T)0) wacc_add(W, reg + (size_t)i * ld + j, acc[c]);
      }
      if (bias && jt == 0 && r == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double bsum = 0.0;
          for (int rr = 0; rr < 16; ++rr) bsum += W.rho[rr] * (double)W.A[rr * 16 + 4 * g + c];
          const int i = it * 16 + 4 * g + c;
          if (i < ni && bsum != 0.0) wacc_add(W, reg + (size_t)i * ld + (ld - 1), (T)bsum);
        }
      }
      sub_sync<64>();
    }
  }
}

// Forward chain of one row tile from h_{K-1} (seeds in st) down to the input with the
// shared-slope relaxation of the step, recording the multipliers g of every relaxed
// layer in the wave's tape; w gets the input coefficients.
template <typename T, int NT, typename Stage>
__device__ __forceinline__ void chain_recorded(const NetDev& net, int K, Stage& st, const V4<T>* rel_all, const T* lds_b,
                                               T (&w)[1][4], int lane, gmut<T> tape) {
  const int gq = lane >> 4;
  double acc = 0.0, acc2 = 0.0;
  T marg = 0;
  for (int k = K - 1; k >= 1; --k) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) tape[(((size_t)(k - 1) * NT + t) * 4 + i) * 64 + lane] = st.get(t, i);
    relax_layer<T, NT, true>(st, rel_all + (k - 1) * 16 * NT, (lconst<T>)(lds_b + (k - 1) * 16 * NT), gq, acc, acc2,
                             marg);
    gconst<V4<T>> Wg = as_global(uniform_ptr((const V4<T>*)net.Wf[k - 1]));
    if (k > 1)
      gemm_inplace<T, NT>(Wg, st, lane);
    else
      gemm_k<T, 1, NT>(Wg, st, w, lane);
  }
}

// The chain in reverse: dw (cotangent of the input coefficients w, per lane its four
// inputs) and the row's offset cotangents rlo, rhi (of the lower / upper offset sums)
// go back through layers 1 .. K-1; the relaxed neurons of every layer add d/ds and d/dt
// to the step's accumulators (summed over the tile's rows); on return st holds the
// cotangent of the seed multipliers over h_{K-1}.  The tile's record (slot, rg_slot_*
// layout) holds the forward multipliers; when weight gradients are asked for, the
// cotangents over every layer's input and the rows' offset cotangents are added to it
// for the step's contraction (step_wgrad).
template <typename T, int NT, typename Stage>
__device__ __forceinline__ void chain_reverse(const NetDev& net, int K, Stage& st, const GradLds<T>& G,
                                              const T (&dw)[1][4], double rlo, double rhi, int lane, gmut<T> slot,
                                              const WgradTile<T>& W) {
  const int gq = lane >> 4, L = net.L;
  const double rsum = rlo + rhi;
  const bool wg = W.reg != nullptr;
  auto tape_g = [&](int layer, int t, int i) { return slot[(((size_t)layer * NT + t) * 4 + i) * 64 + lane]; };
  if (wg) {
    if ((lane & 15) == lane) {
      W.rho[lane] = rsum;
      slot[rg_slot_rho(L, NT) + lane] = (T)rsum;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) slot[rg_slot_dg(0, L, NT) + (size_t)i * 64 + lane] = dw[0][i];
  }
  {
    T dlt[NT][4];
    gemm_tiles<T, NT, 1>((const V4<T>*)net.Wa[0], dw, dlt, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) st.set(t, i, dlt[t][i]);
  }
  for (int k = 1; k <= K - 1; ++k) {
    const int base = (k - 1) * 16 * NT;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = t * 16 + nrn<T>(gq, i);
        const V4<T> rr = G.rel[base + t * 16 + gq * 4 + i];
        const double g = (double)tape_g(k - 1, t, i);
        // d/da' of this neuron: the product's cotangent plus the bias term of both offsets
        const double delta = (double)st.get(t, i) + rsum * (double)G.bias[base + c];
        const bool uns = rr[2] > (T)0;
        const double s = (double)rr[0], tc = (double)rr[2];
        const double side = g < 0.0 ? rlo : (g > 0.0 ? rhi : 0.0);
        const double dg = delta * s + (uns ? side * tc : 0.0);
        const double dsv = sum16(uns ? delta * g : 0.0);
        const double dtv = sum16(uns ? side * g : 0.0);
        if ((lane & 15) == 0 && uns) {
          atomicAdd(&G.ds[base + c], dsv);
          atomicAdd(&G.dt[base + c], dtv);
        }
        st.set(t, i, (T)dg);
        if (wg) slot[rg_slot_dg(k, L, NT) + ((size_t)t * 4 + i) * 64 + lane] = (T)dg;
      }
      tile_fence<T, NT>();
    }
    if (k < K - 1) gemm_inplace<T, NT>(as_global(uniform_ptr((const V4<T>*)net.Wa[k])), st, lane);
  }
}

// The weight gradients of one step from the records of its row tiles (every record
// written and visible): for hidden layer j, dW_j[i][m] += s_i sum_rows g_j[row][i]
// dg_{j-1}[row][m] and db_j[i] += s_i sum_rows g_j[row][i] rho[row] (a' = s g with the
// step's shared slope s_i of neuron i), the rows being those of every record whose
// chain passes layer j.  Items (layer j, 16-row tile of dW_j, 16-column tile or the bias
// column) are dealt to the waves in groups of GI; for every record a lane loads four
// rows of its column of each operand with one vector load, the next record's loads
// issued before the current record's 16x16x4 products; each item's sums are scaled by
// the slopes and added to the region once.
template <typename T, int NT>
__device__ __forceinline__ void step_wgrad(const NetDev& net, const GradLds<T>& G, const WgradTile<T>& W, gmut<T> slots,
                                        int wid, int lane) {
  constexpr int GI = sizeof(T) == 4 ? 8 : 4;
  const int L = net.L, g = lane >> 4, l = lane & 15;
  const int n_slots = rg_slots(L, NT);
  const size_t ssz = rg_slot_elems(L, NT);
  // column l of a 16-wide block: lane group gl, element il of the lane-major layout
  const int pl = pos_of<T>(l), gl = pl >> 2, il = pl & 3;
  const size_t col_off = (size_t)il * 64 + 16 * gl + 4 * g;
  const int n_items = 2 * NT + (L - 2) * NT * (NT + 1);
  auto next_used = [&](int s) {
    for (++s; s < n_slots; ++s)
      if (G.sused[s]) break;
    return s;
  };
  for (int it0 = wid * GI; it0 < n_items; it0 += kWavesPerWG * GI) {
    int jq[GI], mq[GI], tq[GI];
#pragma unroll
    for (int q = 0; q < GI; ++q) {
      const int it = it0 + q;
      if (it >= n_items) { jq[q] = L; mq[q] = 0; tq[q] = 0; continue; }   // L: no record covers it
      if (it < 2 * NT) { jq[q] = 1; mq[q] = it >> 1; tq[q] = it & 1; }     // JT = 1 (the input tile), bias = 1
      else {
        const int r = it - 2 * NT;
        jq[q] = 2 + r / (NT * (NT + 1));
        mq[q] = (r % (NT * (NT + 1))) / (NT + 1);
        tq[q] = r % (NT + 1);                                             // NT: the bias column
      }
    }
    V4<T> acc[GI], a_c[GI], b_c[GI], a_n[GI], b_n[GI];
#pragma unroll
    for (int q = 0; q < GI; ++q) acc[q] = V4<T>{0, 0, 0, 0};
    auto load = [&](int s, V4<T> (&av)[GI], V4<T> (&bv)[GI]) {
      gmut<T> sp = slots + (size_t)s * ssz;
#pragma unroll
      for (int q = 0; q < GI; ++q) {
        const int j = jq[q] < L ? jq[q] : 1;
        const int jt_bias = j == 1 ? 1 : NT;
        av[q] = *(gmut<V4<T>>)(sp + rg_slot_g(j, NT) + (size_t)mq[q] * 256 + col_off);
        if (tq[q] == jt_bias)
          bv[q] = *(gmut<V4<T>>)(sp + rg_slot_rho(L, NT) + 4 * g);
        else
          bv[q] = *(gmut<V4<T>>)(sp + rg_slot_dg(j - 1, L, NT) + (size_t)tq[q] * 256 + col_off);
      }
    };
    int s = next_used(-1);
    if (s < n_slots) load(s, a_c, b_c);
    while (s < n_slots) {
      const int sn = next_used(s);
      if (sn < n_slots) load(sn, a_n, b_n);
      const int Ks = s == 0 ? L : 2 + (s - 1) / NT;   // the record's chain covers layers 1 .. Ks - 1
#pragma unroll
      for (int q = 0; q < GI; ++q) {
        if (jq[q] < Ks) {
          const bool bias = tq[q] == (jq[q] == 1 ? 1 : NT);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[q] = mfma16(a_c[q][v], (bias && l != 0) ? (T)0 : b_c[q][v], acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < GI; ++q) { a_c[q] = a_n[q]; b_c[q] = b_n[q]; }
      s = sn;
    }
#pragma unroll
    for (int q = 0; q < GI; ++q) {
      const int j = jq[q];
      if (j >= L) continue;
      const bool bias = tq[q] == (j == 1 ? 1 : NT);
      const int nj = net.n[j], nm = net.n[j - 1], ld = net.np[j - 1] + 1;
      const int col = bias ? ld - 1 : tq[q] * 16 + l;
      const bool col_ok = bias ? l == 0 : col < nm;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = mq[q] * 16 + nrn<T>(g, c);
        const T sl = G.rel[(j - 1) * 16 * NT + mq[q] * 16 + 4 * g + c][0];
        const T v = acc[q][c] * sl;
        if (col_ok && i < nj && v != (T)0) wacc_add(W, W.woff[j - 1] + (size_t)i * ld + col, v);
      }
    }
  }
}

template <typename T, int NT>
__global__ void __launch_bounds__(kWG) k_reach_grad(const NetDev* __restrict__ nets, int net_index, ReachGradArgs ga) {
  extern __shared__ __align__(16) char lds_raw[];
  const NetDev& net = nets[net_index];
  const int L = net.L, Hp = net.Hp, H = ga.horizon;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, gq = lane >> 4;
  char* stage = lds_raw + (size_t)wid * stage_bytes<T, NT>();
  GradLds<T> G;
  G.carve(lds_raw + kWavesPerWG * stage_bytes<T, NT>(), Hp, NT);
  for (int e = tid; e < Hp; e += kWG) {
    const int k = e / (16 * NT);
    G.bias[e] = as_global((const T*)net.bn[k])[e - k * 16 * NT];
  }
  const int n0 = net.n[0], ns = net.n_state, nx = n0 - ns, n1 = net.n[1];
  const int S = ga.batch.n_sub;
  // this workgroup's row-tile records of the current step
  const int n_slots = rg_slots(L, NT);
  gmut<T> slots = as_global_mut((T*)ga.gtape + (size_t)blockIdx.x * n_slots * rg_slot_elems(L, NT));
  auto slot_of = [&](int sl) { return slots + (size_t)sl * rg_slot_elems(L, NT); };
  WgradTile<T> W;
  T* wglob = ga.wreg ? (T*)ga.wreg + (size_t)blockIdx.x * ga.wreg_stride : nullptr;
  if (ga.wreg && ga.wacc_lds) {
    for (size_t e = tid; e < ga.wreg_stride; e += kWG) G.wacc[e] = (T)0;
  }
  W.reg = ga.wreg ? (ga.wacc_lds ? G.wacc : wglob) : nullptr;
  W.lds = ga.wacc_lds;
  W.woff = ga.woff;
  W.A = (lmut<T>)(G.ob + wid * 512);
  W.B = (lmut<T>)(G.ob + wid * 512 + 256);
  W.rho = (lmut<double>)(G.orho + wid * 16);
  const bool wg = W.reg != nullptr;
  // atomic add into this workgroup's weight-gradient region: layer k, entry (i, j)
  auto wadd = [&](int k, int i, int j, double v) {
    if (v != 0.0) wacc_add(W, ga.woff[k - 1] + (size_t)i * (net.np[k - 1] + 1) + j, (T)v);
  };
  const double* c = G.tm;
  const double* Pm = G.tm + 16;
  const double* Ilo = G.tm + 272;
  const double* Ihi = G.tm + 288;

  for (int b = blockIdx.x; b < S; b += gridDim.x) {
    const double* tb = ga.tape + (size_t)b * reach_tape_doubles(H, Hp);
    const double gV = ga.gV[b];
    for (int e = tid; e < kTmDoubles; e += kWG) G.dO[e] = 0.0;
    lds_barrier();
    for (int t = H - 1; t >= 0; --t) {
      // ---- the step's record; the volume term of X_{t+1} = c' +- |P'| 1 + I'
      {
        const double* tt = tb + reach_tape_tm(t);
        const double* tn = tb + reach_tape_tm(t + 1);
        const double* tl = tb + reach_tape_bounds(t, H, Hp);
        for (int e = tid; e < kTmDoubles; e += kWG) {
          G.tm[e] = tt[e];
          double d = G.dO[e];
          if (e >= 16 && e < 272) {
            const int r = (e - 16) >> 4, z = (e - 16) & 15;
            const double p = tn[e];
            if (r < ns && z < ns) d += 2.0 * gV * (p > 0.0 ? 1.0 : (p < 0.0 ? -1.0 : 0.0));
          } else if (e >= 272 && e < 288) {
            if (e - 272 < ns) d -= gV;
          } else if (e >= 288) {
            if (e - 288 < ns) d += gV;
          }
          G.dO[e] = d;
          G.dI[e] = 0.0;
        }
        for (int e = tid; e < Hp; e += kWG) {
          G.l[e] = tl[e]; G.u[e] = tl[Hp + e]; G.ibl[e] = tl[2 * Hp + e]; G.ibu[e] = tl[3 * Hp + e];
          G.ds[e] = 0.0; G.dt[e] = 0.0; G.dl[e] = 0.0; G.du[e] = 0.0;
        }
        for (int e = tid; e < n_slots; e += kWG) G.sused[e] = 0;
        for (int e = tid; e < Hp; e += kWG) {
          const int k = e / (16 * NT), j = e - k * 16 * NT;
          const int p = k * 16 * NT + (j & ~15) + pos_of<T>(j & 15);
          G.rel[p] = build_relax<T>(tl[e], tl[Hp + e], 0.0, 0.0, false, 1, true, 0);
        }
      }
      lds_barrier();
      // ---- output rows e_r on x' (wave 0): recompute, compose in reverse, chain in reverse
      if (wid == 0) {
        const int r = lane & 15;
        const bool valid = r < ns;
        gconst<T> seed = as_global((const T*)net.seedT + (size_t)(valid ? r : 0) * net.np[L - 1]);
        auto st = make_stage<T, NT>(stage, lane);
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
          for (int i = 0; i < 4; ++i) st.set(tt, i, valid ? seed[tt * 16 + nrn<T>(gq, i)] : (T)0);
        T w[1][4];
        chain_recorded<T, NT>(net, L, st, G.rel, G.bias, w, lane, slot_of(0));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = nrn<T>(gq, i);
          G.Wr[r * 16 + m] = valid ? (double)w[0][i] + net.skip[(size_t)r * 16 + m] : 0.0;
        }
      }
      lds_barrier();
      // cotangents of W_r (thread per (r, m)) and of the incoming model (thread per entry)
      {
        const int r = tid >> 4, m = tid & 15;
        double dWv = 0.0;
        if (r < ns && m < n0) {
          const double Wv = G.Wr[r * 16 + m];
          dWv = G.dO[r] * c[m] + (Wv >= 0.0 ? G.dO[272 + r] * Ilo[m] + G.dO[288 + r] * Ihi[m]
                                             : G.dO[272 + r] * Ihi[m] + G.dO[288 + r] * Ilo[m]);
          for (int z = 0; z < ns; ++z) dWv += G.dO[16 + r * 16 + z] * Pm[m * 16 + z];
          if (ga.dA) atomicAdd(&ga.dA[(size_t)r * n0 + m], dWv);
        }
        G.dWr[tid] = dWv;
        if (tid < 16) {
          G.rowc[tid] = tid < ns ? G.dO[272 + tid] : 0.0;
          G.rowc[16 + tid] = tid < ns ? G.dO[288 + tid] : 0.0;
          // incoming model: centre and interval ends of input m = tid
          double dc = 0.0, dlo = 0.0, dhi = 0.0;
          for (int rr = 0; rr < ns; ++rr) {
            const double Wv = G.Wr[rr * 16 + tid];
            dc += Wv * G.dO[rr];
            dlo += Wv >= 0.0 ? G.dO[272 + rr] * Wv : G.dO[288 + rr] * Wv;
            dhi += Wv >= 0.0 ? G.dO[288 + rr] * Wv : G.dO[272 + rr] * Wv;
          }
          G.dI[tid] += dc; G.dI[272 + tid] += dlo; G.dI[288 + tid] += dhi;
        }
        // dP[m][z] = sum_r W_rm dO_P[r][z]  (thread (m = tid >> 4, z = tid & 15))
        {
          double dp = 0.0;
          for (int rr = 0; rr < ns; ++rr) dp += G.Wr[rr * 16 + r] * G.dO[16 + rr * 16 + m];
          G.dI[16 + tid] += dp;
        }
      }
      lds_barrier();
      if (wid == 0) {
        const int r = lane & 15;
        const bool valid = r < ns;
        T dw[1][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) dw[0][i] = (T)G.dWr[r * 16 + nrn<T>(gq, i)];
        auto st = make_stage<T, NT>(stage, lane);
        const double rlo = valid ? G.rowc[r] : 0.0, rhi = valid ? G.rowc[16 + r] : 0.0;
        chain_reverse<T, NT>(net, L, st, G, dw, rlo, rhi, lane, slot_of(0), W);
        if (lane == 0) G.sused[0] = 1;
        if (wg) {
          // the seed g = B_r W_L: dW_L += B_r (x) dg^(L-1), db_L += rho_r B_r
          const int npL = net.np[L];
          auto a_seed = [&](int it, int i) {
            return valid ? (T)net.seedA[(size_t)r * npL + it * 16 + nrn<T>(gq, i)] : (T)0;
          };
          gmut<T> dgl = slot_of(0) + rg_slot_dg(L - 1, L, NT);
          auto b_buf = [&](int t, int i) { return dgl[((size_t)t * 4 + i) * 64 + lane]; };
          wgrad_blocks<T>(W, L, net.np[L - 1] + 1, npL / 16, NT, net.n[L], net.n[L - 1], a_seed, b_buf, true, lane);
        }
        // the seed g = B_r W_L (and the offset B_r b_L): d/dB_r
        if (ga.dB) {
          const int nL = net.n[L], npl = net.np[L - 1];
          for (int o = 0; o < nL; ++o) {
            gconst<T> WL = as_global((const T*)net.Wn[L - 1] + (size_t)o * npl);
            double part = 0.0;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
              for (int i = 0; i < 4; ++i) part += (double)st.get(tt, i) * (double)WL[tt * 16 + nrn<T>(gq, i)];
            part = row_sum(part) + (rlo + rhi) * (double)((const T*)net.bn[L - 1])[o];
            if (valid && lane < 16) atomicAdd(&ga.dB[(size_t)r * nL + o], part);
          }
        }
      }
      lds_barrier();
      // ---- hidden layers, last to first
      for (int k = L - 1; k >= 1; --k) {
        const int nk = net.n[k], base = (k - 1) * 16 * NT;
        // chord: d/ds, d/dt -> d/dl, d/du (s = u / (u - l), t = -s l)
        for (int j = tid; j < 16 * NT; j += kWG) {
          const int e = base + j;
          const double lv = G.l[e], uv = G.u[e];
          if (j < nk && lv < 0.0 && uv > 0.0) {
            const double den = uv - lv, s = uv / den;
            const double dsdu = -lv / (den * den), dsdl = uv / (den * den);
            const double dtdl = -s - lv * dsdl, dtdu = -lv * dsdu;
            G.dl[e] += G.ds[e] * dsdl + G.dt[e] * dtdl;
            G.du[e] += G.ds[e] * dsdu + G.dt[e] * dtdu;
          }
        }
        lds_barrier();
        if (k >= 2) {
          // the side of each intersection that won: CROWN row (strictly tighter) or IBP
          auto crown_row = [&](int j) { return j < nk && G.ibl[base + j] < 0.0 && G.ibu[base + j] > 0.0; };
          const int nU = compact_flags<kWG>(16 * NT, crown_row, G.U, G.misc + 2);
          const int ntiles = (nU + 15) >> 4;
          for (int tile = wid; tile < ntiles; tile += kWavesPerWG) {
            const int row = tile * 16 + (lane & 15);
            const bool valid = row < nU;
            const int neuron = valid ? G.U[row] : 0;
            const int e = base + neuron;
            const double rlo = (valid && G.l[e] > G.ibl[e]) ? G.dl[e] : 0.0;
            const double rhi = (valid && G.u[e] < G.ibu[e]) ? G.du[e] : 0.0;
            if (__ballot(rlo != 0.0 || rhi != 0.0) == 0ull) continue;
            auto st = make_stage<T, NT>(stage, lane);
            gconst<T> Wrow = as_global((const T*)net.Wn[k - 1] + (size_t)neuron * net.np[k - 1]);
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
              for (int i = 0; i < 4; ++i) st.set(tt, i, valid ? Wrow[tt * 16 + nrn<T>(gq, i)] : (T)0);
            T w[1][4];
            const int sl = 1 + (k - 2) * NT + tile;
            chain_recorded<T, NT>(net, k, st, G.rel, G.bias, w, lane, slot_of(sl));
            // (w P)_z over the row, for the sign of each radius term
            double wv[4], wp[16];
#pragma unroll
            for (int z = 0; z < 16; ++z) wp[z] = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m = nrn<T>(gq, i);
              wv[i] = (double)w[0][i];
#pragma unroll
              for (int z = 0; z < 16; ++z) wp[z] += wv[i] * Pm[m * 16 + z];
            }
#pragma unroll
            for (int z = 0; z < 16; ++z) wp[z] = row_sum(wp[z]);
            T dw[1][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m = nrn<T>(gq, i);
              double d = (rlo + rhi) * c[m] + (wv[i] >= 0.0 ? rlo * Ilo[m] + rhi * Ihi[m] : rlo * Ihi[m] + rhi * Ilo[m]);
#pragma unroll
              for (int z = 0; z < 16; ++z) {
                const double sg = wp[z] > 0.0 ? 1.0 : (wp[z] < 0.0 ? -1.0 : 0.0);
                d += (rhi - rlo) * sg * Pm[m * 16 + z];
              }
              dw[0][i] = (T)d;
              // the incoming model's cotangent, summed over the tile's rows
              const double vc = sum16((rlo + rhi) * wv[i]);
              const double vlo = sum16(wv[i] >= 0.0 ? rlo * wv[i] : rhi * wv[i]);
              const double vhi = sum16(wv[i] >= 0.0 ? rhi * wv[i] : rlo * wv[i]);
              if ((lane & 15) == 0) {
                atomicAdd(&G.dI[m], vc);
                atomicAdd(&G.dI[272 + m], vlo);
                atomicAdd(&G.dI[288 + m], vhi);
              }
#pragma unroll
              for (int z = 0; z < 16; ++z) {
                const double sg = wp[z] > 0.0 ? 1.0 : (wp[z] < 0.0 ? -1.0 : 0.0);
                const double vp = sum16((rhi - rlo) * sg * wv[i]);
                if ((lane & 15) == 0) atomicAdd(&G.dI[16 + m * 16 + z], vp);
              }
            }
            chain_reverse<T, NT>(net, k, st, G, dw, rlo, rhi, lane, slot_of(sl), W);
            if (lane == 0) G.sused[sl] = 1;
            if (wg && valid) {
              // the seed is row `neuron` of W_k (and its bias): dW_k[neuron, :] += dg^(k-1)
#pragma unroll
              for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int m = tt * 16 + nrn<T>(gq, i);
                  if (m < net.n[k - 1])
                    wadd(k, neuron, m, (double)slot_of(sl)[rg_slot_dg(k - 1, L, NT) + ((size_t)tt * 4 + i) * 64 + lane]);
                }
              if (gq == 0) wadd(k, neuron, net.np[k - 1], rlo + rhi);
            }
          }
          // interval bounds in reverse: li = W relu-centre + b - |W| relu-radius, ui = ... +;
          // the sum over the neurons j of layer k is split into P parts (thread (part, m)),
          // whose partial sums go to the output rows' buffers Wr, dWr (512 contiguous
          // doubles, unused in this phase) and are added in a fixed order
          const int n16 = 16 * NT, P = kWG / n16;
          double* hpart = G.Wr;   // P x 2 x n16 <= 512
          // the cotangents that reach each neuron's interval bounds (the side that won the
          // intersection), into the slope / intercept cotangents of layer k (consumed by the
          // chord step above)
          double* dli_k = G.ds + base;
          double* dui_k = G.dt + base;
          for (int j = tid; j < nk; j += kWG) {
            const int e = base + j;
            const bool cu = G.ibl[e] < 0.0 && G.ibu[e] > 0.0;
            dli_k[j] = (cu && G.l[e] > G.ibl[e]) ? 0.0 : G.dl[e];
            dui_k[j] = (cu && G.u[e] < G.ibu[e]) ? 0.0 : G.du[e];
          }
          lds_barrier();
          {
            const int m = tid % n16, part = tid / n16;
            if (part < P) {
              double dhc = 0.0, dhr = 0.0;
              if (m < net.n[k - 1]) {
                // relu centre / radius of input m (layer k-1's final bounds)
                const double la = fmax(G.l[base - n16 + m], 0.0), ub = fmax(G.u[base - n16 + m], 0.0);
                const double hc = 0.5 * (la + ub), hr = 0.5 * (ub - la);
                const int chunk = (nk + P - 1) / P, j0 = part * chunk, j1 = min(nk, j0 + chunk);
#pragma unroll 4
                for (int j = j0; j < j1; ++j) {
                  const double dli = dli_k[j], dui = dui_k[j];
                  const double wv = (double)((const T*)net.Wn[k - 1])[(size_t)j * net.np[k - 1] + m];
                  dhc += wv * (dli + dui);
                  dhr += fabs(wv) * (dui - dli);
                  if (wg) {
                    const double sw = wv > 0.0 ? 1.0 : (wv < 0.0 ? -1.0 : 0.0);
                    wadd(k, j, m, (dli + dui) * hc + (dui - dli) * sw * hr);
                    if (m == 0) wadd(k, j, net.np[k - 1], dli + dui);
                  }
                }
              }
              hpart[(size_t)(2 * part) * n16 + m] = dhc;
              hpart[(size_t)(2 * part + 1) * n16 + m] = dhr;
            }
          }
          lds_barrier();
          for (int m = tid; m < n16; m += kWG) {
            const int e = base - n16 + m;
            double dhc = 0.0, dhr = 0.0;
            for (int part = 0; part < P; ++part) {
              dhc += hpart[(size_t)(2 * part) * n16 + m];
              dhr += hpart[(size_t)(2 * part + 1) * n16 + m];
            }
            if (G.l[e] > 0.0) G.dl[e] += 0.5 * (dhc - dhr);
            if (G.u[e] > 0.0) G.du[e] += 0.5 * (dhc + dhr);
          }
          lds_barrier();
        } else {
          // layer 1: the exact range of W_1 over the model c + P z + [I_lo, I_hi]
          for (int e = tid; e < n1 * 16; e += kWG) {
            const int j = e >> 4, z = e & 15;
            gconst<T> W = as_global((const T*)net.Wn[0] + (size_t)j * net.np[0]);
            double wpz = 0.0;
            for (int m = 0; m < n0; ++m) wpz += (double)W[m] * Pm[m * 16 + z];
            G.wps[j * 16 + z] = wpz > 0.0 ? 1 : (wpz < 0.0 ? -1 : 0);
          }
          lds_barrier();
          {
            const int m = tid >> 4, z = tid & 15;
            double dp = 0.0, dc = 0.0, dlo = 0.0, dhi = 0.0;
            if (m < n0) {
#pragma unroll 4
              for (int j = 0; j < n1; ++j) {
                const double wv = (double)((const T*)net.Wn[0])[(size_t)j * net.np[0] + m];
                const double dzc = G.dl[j] + G.du[j], dzr = G.du[j] - G.dl[j];
                dp += dzr * (double)G.wps[j * 16 + z] * wv;
                if (z == 0) {
                  dc += wv * dzc;
                  dlo += 0.5 * (wv * dzc - fabs(wv) * dzr);
                  dhi += 0.5 * (wv * dzc + fabs(wv) * dzr);
                }
              }
            }
            G.dI[16 + tid] += dp;
            if (z == 0) { G.dI[m] += dc; G.dI[272 + m] += dlo; G.dI[288 + m] += dhi; }
          }
          if (wg) {
            // dW_1[j][m] += dzc_j (c_m + mid_m) + dzr_j (sum_z sgn((W_1 P)_jz) P_mz + sgn(W_jm) rad_m)
            for (int e = tid; e < n1 * n0; e += kWG) {
              const int j = e / n0, m = e % n0;
              const double dzc = G.dl[j] + G.du[j], dzr = G.du[j] - G.dl[j];
              const double wv = (double)((const T*)net.Wn[0])[(size_t)j * net.np[0] + m];
              double sp = 0.0;
              for (int z = 0; z < 16; ++z) sp += (double)G.wps[j * 16 + z] * Pm[m * 16 + z];
              const double sw = wv > 0.0 ? 1.0 : (wv < 0.0 ? -1.0 : 0.0);
              wadd(1, j, m, dzc * (c[m] + 0.5 * (Ilo[m] + Ihi[m])) + dzr * (sp + sw * 0.5 * (Ihi[m] - Ilo[m])));
              if (m == 0) wadd(1, j, net.np[0], dzc);
            }
          }
          lds_barrier();
        }
      }
      // ---- the step's weight gradients from its row-tile records (global memory written by
      // every wave: a full barrier; the next step rewrites the records only after the
      // barriers that end this one)
      if (wg) {
        __syncthreads();
        step_wgrad<T, NT>(net, G, W, slots, wid, lane);
      }
      // ---- the incoming model's cotangent: actions, and the previous step's output
      if (tid < 16 && tid >= ns && tid < n0 && ga.du) ga.du[((size_t)b * H + t) * nx + (tid - ns)] = G.dI[tid];
      for (int e = tid; e < kTmDoubles; e += kWG) {
        int m;
        if (e < 16) m = e;
        else if (e < 272) m = (e - 16) >> 4;
        else m = (e - 272) & 15;
        const bool zok = e < 16 || e >= 272 || ((e - 16) & 15) < ns;
        G.dO[e] = (m < ns && zok) ? G.dI[e] : 0.0;
      }
      lds_barrier();
    }
    if (tid < ns) {
      if (ga.dxc) ga.dxc[(size_t)b * ns + tid] = G.dO[tid];
      if (ga.dxr) ga.dxr[(size_t)b * ns + tid] = G.dO[16 + tid * 16 + tid];
    }
    lds_barrier();
  }
  if (wglob && ga.wacc_lds) {
    // the workgroup's sums, stored once (its own region: plain stores)
    __syncthreads();
    for (size_t e = tid; e < ga.wreg_stride; e += kWG) wglob[e] = G.wacc[e];
  }
}

}  // namespace dr
