// Continuous-time flowpipes with fixed-shape Taylor models (FP64), the device side of
// Section "Propagation under Continuous-Time Analytical Dynamics" (Theorem "TM flowpipe
// step via Picard iteration", appendix Algorithm "Reachability of CT Dynamics with TM
// Flowpipe") and of the inner loop of Algorithm "Reachability of CT NN Control Systems".
//
// A model is the quasi-quadratic form of Section "Representation of Reachable Sets" over
// the generators y in [-1, 1]^m (m <= 16) of the box and the time s in [0, h]:
//     X(y, s) = c + L y + l s + s (M y) + w s^2  (+)  [lo, hi].
// One wavefront carries one box (n <= 16 state components).  Dynamics: f_i(x, u) = a_i +
// F_i x + G_i u + x^T Q_i x (degree <= 2 in the state, affine in the held input u).  A
// product keeps the monomials {1, y, s, s y, s^2} and bounds every other one over the
// domain into the interval part.  Each evaluation of f first forms every distinct
// quadratic monomial X_j X_k (j <= k) once, one per quad of lanes in chunks of 16; the
// sum of all terms (coefficient Q_ijk + Q_ikj off the diagonal) is then a product of the
// coefficient matrix with the terms' models on the FP64 matrix cores (their L and M
// parts), the scalar and interval parts on the vector units.  The step: two Picard iterations of the
// polynomial part from the seed c + S y; the remainder J validated by the Picard image
// J' = I_0 + hull(0, h range(f(p + J) - d/ds p)) inside J (widening while not), then
// refined; the step-end model c + l h + w h^2 + (L + h M) y (+) J; the remainder is then
// absorbed into the linear part (S <- S diag(1 + |S^-1| rad J), centre += mid J) when S is
// well conditioned, and a held input's model follows the change of generators.  Arithmetic is FP64 without outward
// rounding (the rounding of these steps is not covered by a margin).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"

namespace dr {

constexpr int kCtMax = 16;
constexpr int kCtLd = kCtMax + 1;                          // row stride of L, M and S in LDS (odd: rows
                                                           // read one per lane fall in distinct banks)
constexpr int kCtAug = 2 * kCtMax + 1;                     // row stride of [S | I] in the inversion
constexpr int kCtChunk = 16;                               // monomials formed per pass
constexpr int kCtPairs = kCtMax * (kCtMax + 1) / 2;        // distinct monomials x_j x_k

// A vector of `cap` models in LDS (structure of arrays; L and M are cap x 16 with row
// stride kCtLd).
struct QTL {
  double* c;
  double* L;
  double* l;
  double* M;
  double* w;
  double* lo;
  double* hi;
  __host__ __device__ static constexpr size_t bytes(int cap) { return (size_t)(5 * cap + 2 * cap * kCtLd) * sizeof(double); }
  __device__ void carve(double* base, int cap) {
    c = base; L = c + cap; l = L + cap * kCtLd; M = l + cap; w = M + cap * kCtLd;
    lo = w + cap; hi = lo + cap;
  }
};

// Range of the polynomial part over y in [-1, 1]^m, s in [0, h] (term by term), from
// the constant, the absolute sums of L and M, and the s and s^2 coefficients.
__device__ __forceinline__ void poly_range(double c, double sL, double sM, double l, double w, double h, double& lo,
                                           double& hi) {
  const double r = sL + h * sM;
  lo = c - r + fmin(0.0, l * h) + fmin(0.0, w * h * h);
  hi = c + r + fmax(0.0, l * h) + fmax(0.0, w * h * h);
}
__device__ __forceinline__ void iv_mul(double alo, double ahi, double blo, double bhi, double& lo, double& hi) {
  const double p0 = alo * blo, p1 = alo * bhi, p2 = ahi * blo, p3 = ahi * bhi;
  lo = fmin(fmin(p0, p1), fmin(p2, p3));
  hi = fmax(fmax(p0, p1), fmax(p2, p3));
}

// Sum over the four lanes of a quad (the same on each of them).
__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 1);
  return v + __shfl_xor(v, 2);
}

// dst[slot] = X_j X_k: the product truncated to the representation (the kept monomials
// exactly, the dropped ones and the interval parts bounded over the domain), with both
// factors read from LDS.  Four lanes (a quad, `part` = 0..3) form one product: each takes
// the generators 4 part .. 4 part + 3, the sums over the generators are combined over the
// quad, and every lane of the quad derives the same scalar and interval parts (part 0
// stores them).  `store` = false: the quad only takes part in the lane exchanges.
__device__ __forceinline__ void qt_product(const QTL& X, int j, int k, double h, const QTL& dst, int slot, int part,
                                           bool store) {
  const double* aL = X.L + j * kCtLd + 4 * part;
  const double* aM = X.M + j * kCtLd + 4 * part;
  const double* bL = X.L + k * kCtLd + 4 * part;
  const double* bM = X.M + k * kCtLd + 4 * part;
  const double ac = X.c[j], al = X.l[j], aw = X.w[j], alo_i = X.lo[j], ahi_i = X.hi[j];
  const double bc = X.c[k], bl = X.l[k], bw = X.w[k], blo_i = X.lo[k], bhi_i = X.hi[k];
  // (L_a y)(L_b y): y_p^2 in [0, 1], y_p y_r in [-1, 1]
  double dsum_lo = 0.0, dsum_hi = 0.0, sd = 0.0, sLa = 0.0, sLb = 0.0, sMa = 0.0, sMb = 0.0;
  double* oL = dst.L + slot * kCtLd + 4 * part;
  double* oM = dst.M + slot * kCtLd + 4 * part;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const double la = aL[p], lb = bL[p], ma = aM[p], mb = bM[p];
    sLa += fabs(la); sLb += fabs(lb); sMa += fabs(ma); sMb += fabs(mb);
    const double d = la * lb;
    dsum_lo += fmin(d, 0.0); dsum_hi += fmax(d, 0.0);
    sd += fabs(d);
    if (store) {
      oL[p] = ac * lb + bc * la;
      oM[p] = ac * mb + bc * ma + al * lb + bl * la;
    }
  }
  sLa = quad_sum(sLa); sLb = quad_sum(sLb); sMa = quad_sum(sMa); sMb = quad_sum(sMb);
  dsum_lo = quad_sum(dsum_lo); dsum_hi = quad_sum(dsum_hi); sd = quad_sum(sd);
  const double off = sLa * sLb - sd;
  double lo = dsum_lo - off, hi = dsum_hi + off;
  // s y y, s^2 y, s^2 y y, s^3, s^3 y, s^4
  const double t1 = h * (sLa * sMb + sMa * sLb);
  const double t2 = h * h * (fabs(al) * sMb + fabs(bl) * sMa + fabs(aw) * sLb + fabs(bw) * sLa);
  const double t3 = h * h * sMa * sMb;
  const double t4 = h * h * h * (fabs(aw) * sMb + fabs(bw) * sMa);
  lo -= t1 + t2 + t3 + t4; hi += t1 + t2 + t3 + t4;
  const double s3 = (al * bw + aw * bl) * h * h * h, s4 = aw * bw * h * h * h * h;
  lo += fmin(0.0, s3) + fmin(0.0, s4); hi += fmax(0.0, s3) + fmax(0.0, s4);
  // interval parts
  double alo, ahi, blo, bhi, x0, x1;
  poly_range(ac, sLa, sMa, al, aw, h, alo, ahi);
  poly_range(bc, sLb, sMb, bl, bw, h, blo, bhi);
  iv_mul(alo_i, ahi_i, blo, bhi, x0, x1); lo += x0; hi += x1;
  iv_mul(blo_i, bhi_i, alo, ahi, x0, x1); lo += x0; hi += x1;
  iv_mul(alo_i, ahi_i, blo_i, bhi_i, x0, x1); lo += x0; hi += x1;
  if (store && part == 0) {
    dst.c[slot] = ac * bc;
    dst.l[slot] = ac * bl + bc * al;
    dst.w[slot] = ac * bw + bc * aw + al * bl;
    dst.lo[slot] = lo;
    dst.hi[slot] = hi;
  }
}

struct CtDyn {
  int n, n_u;
  const double* a;     // n
  const double* F;     // n x n
  const double* G;     // n x n_u (or null)
  const double* Q;     // n x n x n (or null)
};

// Per-box LDS of the flowpipe (one wavefront): the model f is evaluated over (the Picard
// iterate, then the remainder's trial models), the held input, a chunk of quadratic
// monomials, the seed, the inversion work space and the list of monomials of the field.
struct CtLds {
  QTL X, U, P;
  double* S;        // 16 x 16 seed linear part, row stride kCtLd (the state model c + S y + [lo, hi])
  double* c;        // 16
  double* lo;       // 16
  double* hi;       // 16
  double* aux;      // 16: column scales of the preconditioning
  double* sums;     // 32: per-component sums of magnitudes (L, M) of an image
  double* aug;      // 16 x 32 (row stride kCtAug): [S | I] during the inversion, then S^-1 in the
                    // right half (in the space of the monomial chunk P)
  int* pairs;       // (j << 8) | k of the monomials x_j x_k (j <= k) with a nonzero coefficient
  int* n_pairs;
  // the held input's models come last, n_u of them (none for a flowpipe without input);
  // the inversion's [S | I] shares the monomials' space (never live together)
  static_assert(QTL::bytes(kCtChunk) >= (size_t)kCtMax * kCtAug * sizeof(double), "[S | I] must fit the chunk");
  __host__ __device__ static constexpr size_t bytes(int n_u) {
    return QTL::bytes(kCtMax) + QTL::bytes(kCtChunk) + (size_t)(kCtMax * kCtLd + 6 * kCtMax) * sizeof(double) +
           (size_t)(kCtPairs + 8) * sizeof(int) + (n_u > 0 ? QTL::bytes(n_u) : 0);
  }
  __device__ void carve(double* base, int n_u) {
    X.carve(base, kCtMax); base += QTL::bytes(kCtMax) / sizeof(double);
    P.carve(base, kCtChunk);
    aug = base; base += QTL::bytes(kCtChunk) / sizeof(double);
    S = base; base += kCtMax * kCtLd;
    c = base; base += kCtMax;
    lo = base; base += kCtMax;
    hi = base; base += kCtMax;
    aux = base; base += kCtMax;
    sums = base; base += 2 * kCtMax;
    pairs = (int*)base;
    n_pairs = pairs + kCtPairs;
    U.carve((double*)(n_pairs + 8), n_u > 0 ? n_u : 1);
  }
};

__device__ __forceinline__ void ct_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
}

// The monomials x_j x_k (j <= k, in order of j then k) whose coefficient is nonzero in
// some component (the wavefront of the box).
__device__ __forceinline__ void ct_pairs(const CtLds& C, const CtDyn& d) {
  const int lane = threadIdx.x & 63, n = d.n;
  int count = 0;
  if (d.Q) {
    for (int e0 = 0; e0 < n * n; e0 += 64) {
      const int e = e0 + lane;
      const int j = e / n, k = e % n;
      bool use = false;
      if (e < n * n && j <= k)
        for (int i = 0; i < n; ++i)
          use = use || d.Q[((size_t)i * n + j) * n + k] != 0.0 || d.Q[((size_t)i * n + k) * n + j] != 0.0;
      const unsigned long long m = __ballot(use);
      if (use) C.pairs[count + __popcll(m & ((1ull << lane) - 1ull))] = (j << 8) | k;
      count += __popcll(m);
    }
  }
  if (lane == 0) C.n_pairs[0] = count;
  ct_sync();
}

// An evaluation of f: the scalar part (c, l, w and the interval part) of component
// i = lane & 15 on every lane of the component, and the L and M coefficients in the
// output layout of the FP64 matrix cores: lane 16 g + n holds those of components
// 4 r + g (r = 0..3) at generator n.
struct QTd {
  double c, l, w, lo, hi;
  V4<double> L, M;
};

// Sum over the four lane groups of a component (bit-identical on every lane: the two
// pairwise sums commute).
__device__ __forceinline__ double group_sum(double v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}
// Sum over the 16 lanes of a lane group (butterfly: the same on every lane of the group).
__device__ __forceinline__ double row16_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  return v + __shfl_xor(v, 8);
}

// f over the models in C.X (and the held input C.U): every lane of the wavefront calls
// it.  The distinct monomials are formed first, one per quad of lanes; then the sum over
// all terms (F_ij X_j, G_ik U_k, Qs_ijk X_j X_k) is one product coefficients x term models
// on the matrix cores for the L and M parts (a 16 x 4 block of coefficients -- components
// x four terms -- against those terms' rows, 16x16x4 FP64 steps), and for the scalar and
// interval parts a per-lane sum over every fourth term (lane group g takes the terms
// 4 s + g) added over the four groups.  A lane skips the interval part of its zero terms
// (an unbounded model then stays out of the components that do not use it).  Ends with
// the wavefront synchronised.
__device__ __forceinline__ QTd ct_f(const CtLds& C, const CtDyn& d, bool ctrl, double h) {
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4, n = d.n;
  const bool act = i < n;
  const int ic = act ? i : 0;
  QTd out;
  out.c = (act && g == 0) ? d.a[ic] : 0.0;
  out.l = out.w = out.lo = out.hi = 0.0;
  out.L = V4<double>{0.0, 0.0, 0.0, 0.0};
  out.M = V4<double>{0.0, 0.0, 0.0, 0.0};
  // one matrix-core step over four terms: this lane's term (row `row` of T, coefficient
  // cf for component i; cf = 0 and no row when the lane has no term)
  auto kstep = [&](double cf, const QTL& T, int row, bool valid) {
    const int rr = valid ? row : 0;
    const double bL = valid ? T.L[rr * kCtLd + i] : 0.0, bM = valid ? T.M[rr * kCtLd + i] : 0.0;
    out.L = mfma16(cf, bL, out.L);
    out.M = mfma16(cf, bM, out.M);
    if (cf != 0.0) {
      out.c += cf * T.c[rr]; out.l += cf * T.l[rr]; out.w += cf * T.w[rr];
      const double lo = T.lo[rr], hi = T.hi[rr];
      if (cf >= 0.0) { out.lo += cf * lo; out.hi += cf * hi; }
      else { out.lo += cf * hi; out.hi += cf * lo; }
    }
  };
  // linear terms: F_ij X_j, then G_ik U_k (coefficients fetched before their steps)
  {
    double cf[kCtMax / 4];
#pragma unroll
    for (int s = 0; s < kCtMax / 4; ++s) {
      const int t = 4 * s + g;
      cf[s] = (act && t < n) ? d.F[(size_t)ic * n + t] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < kCtMax / 4; ++s)
      if (4 * s < n) kstep(cf[s], C.X, 4 * s + g, 4 * s + g < n);
  }
  if (ctrl && d.G) {
    double cf[kCtMax / 4];
#pragma unroll
    for (int s = 0; s < kCtMax / 4; ++s) {
      const int t = 4 * s + g;
      cf[s] = (act && t < d.n_u) ? d.G[(size_t)ic * d.n_u + t] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < kCtMax / 4; ++s)
      if (4 * s < d.n_u) kstep(cf[s], C.U, 4 * s + g, 4 * s + g < d.n_u);
  }
  // quadratic terms, a chunk of monomials at a time
  const int np = C.n_pairs[0];
  for (int p0 = 0; p0 < np; p0 += kCtChunk) {
    const int cnt = min(kCtChunk, np - p0);
    {
      // one quad of lanes per monomial (every quad takes part; those beyond the chunk
      // repeat its last monomial without storing it)
      const int q = lane >> 2, qq = q < cnt ? q : cnt - 1;
      const int pr = C.pairs[p0 + qq];
      qt_product(C.X, pr >> 8, pr & 255, h, C.P, qq, lane & 3, q < cnt);
    }
    double cf[kCtChunk / 4];
#pragma unroll
    for (int s = 0; s < kCtChunk / 4; ++s) {
      const int t = 4 * s + g;
      cf[s] = 0.0;
      if (act && t < cnt) {
        const int pr = C.pairs[p0 + t];
        const int j = pr >> 8, k = pr & 255;
        cf[s] = d.Q[((size_t)ic * n + j) * n + k] + (j != k ? d.Q[((size_t)ic * n + k) * n + j] : 0.0);
      }
    }
    ct_sync();
#pragma unroll
    for (int s = 0; s < kCtChunk / 4; ++s)
      if (4 * s < cnt) kstep(cf[s], C.P, 4 * s + g, 4 * s + g < cnt);
    ct_sync();
  }
  out.c = group_sum(out.c); out.l = group_sum(out.l); out.w = group_sum(out.w);
  out.lo = group_sum(out.lo); out.hi = group_sum(out.hi);
  ct_sync();
  return out;
}

// One flowpipe step of the wavefront's box (lane 16 g + i, i < n, works on component i):
// seed (C.c, C.S, C.lo, C.hi), held input C.U (if `ctrl`).  On return the step-end model
// is the new seed (not yet preconditioned), seg (per lane, for its component) the box of
// the segment, and the return value says whether a contractive remainder was found (the
// same on every lane).
__device__ __forceinline__ bool ct_step(const CtLds& C, const CtDyn& d, bool ctrl, double h, int tries, int rounds,
                                        double eps, double& seg_lo, double& seg_hi) {
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
  const int n = d.n;
  const bool act = i < n;
  // ---- polynomial Picard: g_0 = c + S y, g_{j+1} = x_0 + trunc(int f(g_j)); x_0 is
  // re-read from the seed
  if (act) {
    if (g == 0) { C.X.c[i] = C.c[i]; C.X.l[i] = 0.0; C.X.w[i] = 0.0; C.X.lo[i] = 0.0; C.X.hi[i] = 0.0; }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      C.X.L[i * kCtLd + 4 * g + q] = C.S[i * kCtLd + 4 * g + q];
      C.X.M[i * kCtLd + 4 * g + q] = 0.0;
    }
  }
  ct_sync();
  for (int it = 0; it < 2; ++it) {
    const QTd fx = ct_f(C, d, ctrl, h);
    if (act && g == 0) { C.X.l[i] = fx.c; C.X.w[i] = 0.5 * fx.l; }
    // M of component 4 r + g at generator i (rows n.. of the product are zero)
#pragma unroll
    for (int r = 0; r < 4; ++r) C.X.M[(4 * r + g) * kCtLd + i] = fx.L[r];
    ct_sync();
  }
  // p is the polynomial part of C.X from here on (the trial remainders only change its
  // interval part); d/ds p = l + M y + 2 w s
  const double I0lo = act ? C.lo[i] : 0.0, I0hi = act ? C.hi[i] : 0.0;
  double Jlo = I0lo - eps, Jhi = I0hi + eps, nlo = 0.0, nhi = 0.0;
  // the Picard image of p + J: trial model p (+) J in C.X, then f over it minus d/ds p
  auto picard_image = [&]() {
    if (act && g == 0) { C.X.lo[i] = Jlo; C.X.hi[i] = Jhi; }
    ct_sync();
    const QTd D = ct_f(C, d, ctrl, h);
    // sums of |L - M_p| and |M| over the generators, per component (matrix-core layout:
    // a lane group's 16 lanes are the generators of components 4 r + g)
    double aL[4], aM[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      aL[r] = row16_sum(fabs(D.L[r] - C.X.M[(4 * r + g) * kCtLd + i]));
      aM[r] = row16_sum(fabs(D.M[r]));
    }
    if (i == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) { C.sums[4 * r + g] = aL[r]; C.sums[kCtMax + 4 * r + g] = aM[r]; }
    }
    ct_sync();
    const double sL = C.sums[i], sM = C.sums[kCtMax + i];
    nlo = 0.0; nhi = 0.0;
    if (act) {
      const double Dc = D.c - C.X.l[i], Dl = D.l - 2.0 * C.X.w[i];
      double plo, phi;
      poly_range(Dc, sL, sM, Dl, D.w, h, plo, phi);
      nlo = I0lo + fmin(0.0, h * (plo + D.lo));
      nhi = I0hi + fmax(0.0, h * (phi + D.hi));
    }
    ct_sync();
  };
  bool ok = false;
  // an unbounded initial set has no bounded remainder
  const int ntry = __any(!(fabs(I0lo) < INFINITY) || !(fabs(I0hi) < INFINITY)) ? 0 : tries;
  for (int t = 0; t < ntry; ++t) {
    picard_image();
    const bool in = !act || (nlo >= Jlo && nhi <= Jhi);
    if (__all(in)) {
      ok = true;
      Jlo = nlo; Jhi = nhi;
      break;
    }
    const double wid = fmax(nhi - nlo, eps);
    Jlo = fmin(Jlo, nlo) - 0.5 * wid;
    Jhi = fmax(Jhi, nhi) + 0.5 * wid;
    // an unbounded remainder is no remainder: stop (the same on every lane)
    if (__any(!(fabs(Jlo) < INFINITY) || !(fabs(Jhi) < INFINITY))) break;
  }
  if (ok) {
    for (int r = 0; r < rounds; ++r) {
      picard_image();
      Jlo = fmax(Jlo, nlo); Jhi = fmin(Jhi, nhi);
    }
  } else {
    Jlo = -INFINITY; Jhi = INFINITY;
  }
  // segment box, step-end model
  double sL = 0.0, sM = 0.0;
  if (act) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double Lq = C.X.L[i * kCtLd + 4 * g + q], Mq = C.X.M[i * kCtLd + 4 * g + q];
      sL += fabs(Lq); sM += fabs(Mq);
      C.S[i * kCtLd + 4 * g + q] = Lq + h * Mq;
    }
  }
  sL = group_sum(sL); sM = group_sum(sM);
  if (act) {
    const double pc = C.X.c[i], pl = C.X.l[i], pw = C.X.w[i];
    double plo, phi;
    poly_range(pc, sL, sM, pl, pw, h, plo, phi);
    seg_lo = plo + Jlo; seg_hi = phi + Jhi;
    if (g == 0) { C.c[i] = pc + pl * h + pw * h * h; C.lo[i] = Jlo; C.hi[i] = Jhi; }
  }
  ct_sync();
  return ok;
}

// Step (A): absorb the remainder into the linear part when S is well conditioned; the
// held input follows.  The wavefront of the box: S^-1 by Gauss-Jordan with partial
// pivoting (first largest pivot) on the augmented matrix [S | I] in LDS, one column per
// lane; S^-1 is then the right half.
__device__ __forceinline__ void ct_precondition(const CtLds& C, int n, int n_u, bool ctrl) {
  const int i = threadIdx.x & 63;
  double* aug = C.aug;   // n x 2n, row stride kCtAug
  constexpr int ld = kCtAug;
  bool fin = true;
  if (i < n) {
    fin = fabs(C.lo[i]) < INFINITY && fabs(C.hi[i]) < INFINITY;
    for (int q = 0; q < n; ++q) fin = fin && fabs(C.S[i * kCtLd + q]) < INFINITY;
  }
  bool good = !__any(!fin);
  if (i < 2 * n)
    for (int r = 0; r < n; ++r) aug[r * ld + i] = i < n ? C.S[r * kCtLd + i] : (i - n == r ? 1.0 : 0.0);
  ct_sync();
  for (int col = 0; col < n && good; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(aug[r * ld + col]) > fabs(aug[piv * ld + col])) piv = r;
    const double pv = aug[piv * ld + col];
    if (!(fabs(pv) > 0.0)) { good = false; break; }
    double f[kCtMax];
    for (int r = 0; r < n; ++r) f[r] = aug[(r == col ? piv : (r == piv ? col : r)) * ld + col];
    ct_sync();
    if (i < 2 * n) {
      // swap rows col and piv, scale the pivot row, eliminate the column elsewhere
      if (piv != col) {
        const double t = aug[col * ld + i];
        aug[col * ld + i] = aug[piv * ld + i];
        aug[piv * ld + i] = t;
      }
      const double inv = 1.0 / pv;
      const double prow = aug[col * ld + i] * inv;
      aug[col * ld + i] = prow;
      for (int r = 0; r < n; ++r)
        if (r != col && f[r] != 0.0) aug[r * ld + i] -= f[r] * prow;
    }
    ct_sync();
  }
  const double* Si = aug + n;   // S^-1 (row stride ld)
  // check S^-1 S against the identity
  double err = 0.0;
  if (good) {
    for (int e = i; e < n * n; e += 64) {
      const int r = e / n, q = e % n;
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += Si[r * ld + k] * C.S[k * kCtLd + q];
      const double dv = fabs(v - (r == q ? 1.0 : 0.0));
      if (!(dv <= err)) err = dv;
    }
  }
  good = good && !__any(!(err <= 1e-9));
  if (!good) return;
  // delta_j = sum_k |Si_jk| rad_k; input extra_r = sum_j |(P_u Si)_rj| rad_j
  double Dj = 1.0;
  if (i < n) {
    double dl = 0.0;
    for (int k = 0; k < n; ++k) dl += fabs(Si[i * ld + k]) * 0.5 * (C.hi[k] - C.lo[k]);
    Dj = 1.0 + dl;
  }
  double extra = 0.0;
  if (ctrl && i < n_u) {
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += C.U.L[i * kCtLd + k] * Si[k * ld + j];
      extra += fabs(v) * 0.5 * (C.hi[j] - C.lo[j]);
    }
  }
  ct_sync();
  if (i < n) C.aux[i] = Dj;
  ct_sync();
  if (i < n) {
    C.c[i] += 0.5 * (C.lo[i] + C.hi[i]);
    for (int q = 0; q < n; ++q) C.S[i * kCtLd + q] *= C.aux[q];
    C.lo[i] = 0.0; C.hi[i] = 0.0;
  }
  if (ctrl && i < n_u) {
    for (int q = 0; q < n; ++q) C.U.L[i * kCtLd + q] *= C.aux[q];
    C.U.lo[i] -= extra; C.U.hi[i] += extra;
  }
  ct_sync();
}

// A box's state between the launches of the closed loop (FP64, global memory): the state
// model c (16), S (16 x 16, row-major), I_lo (16), I_hi (16), then the held input's model
// c_u (16), P_u (16 x 16), its interval lo (16), hi (16).
constexpr int kCtState = 608;

struct CtArgs {
  BatchDev batch;
  Scratch sc;
  CtDyn dyn;
  double h;
  int K;             // flowpipe steps per control interval
  int n_ctl;         // control intervals (without a controller: one interval of K steps each)
  int tries, rounds;
  double eps;
  double* state;     // closed loop: S x kCtState, each box's state between the launches
  double* boxes;     // S x (n_ctl K + 1) x n x 2: time points
  double* segs;      // S x n_ctl K x n x 2: segments (nullable)
  uint32_t* status;
};

// Box of the state model (c, S, lo, hi) for component i.
__device__ __forceinline__ void ct_point_box(const CtLds& C, int i, double& lo, double& hi) {
  double r = 0.0;
  for (int q = 0; q < kCtMax; ++q) r += fabs(C.S[i * kCtLd + q]);
  lo = C.c[i] - r + C.lo[i];
  hi = C.c[i] + r + C.hi[i];
}

// The seed of box b: c = centre, S = diag(radius), no remainder; writes the box of time
// point 0 (the wavefront of the box).
__device__ __forceinline__ void ct_seed(const CtLds& C, const CtArgs& ca, int b, int n0) {
  const int i = threadIdx.x & 63, n = ca.dyn.n;
  const int N = ca.n_ctl * ca.K;
  if (i < kCtMax) {
    C.c[i] = i < n ? ca.batch.xc[(size_t)b * n0 + i] : 0.0;
    C.lo[i] = 0.0; C.hi[i] = 0.0;
  }
  for (int e = i; e < kCtMax * kCtMax; e += 64) {
    const int r = e / kCtMax, q = e % kCtMax;
    C.S[r * kCtLd + q] = (r == q && r < n) ? ca.batch.xr[(size_t)b * n0 + r] : 0.0;
  }
  ct_sync();
  if (i < n) {
    double lo, hi;
    ct_point_box(C, i, lo, hi);
    double* bo = ca.boxes + (size_t)b * (N + 1) * n * 2;
    bo[i * 2 + 0] = lo; bo[i * 2 + 1] = hi;
  }
}

// K flowpipe steps from the current seed (the wavefront of the box), writing time-point
// boxes t0+1 .. t0+K and segment boxes t0 .. t0+K-1; returns false if a step found no
// contractive remainder.
__device__ __forceinline__ bool ct_steps(const CtLds& C, const CtArgs& ca, bool ctrl, int b, int t0) {
  const int lane = threadIdx.x & 63, n = ca.dyn.n;
  const int N = ca.n_ctl * ca.K;
  bool ok_all = true;
  for (int j = 0; j < ca.K; ++j) {
    double slo = 0.0, shi = 0.0;
    const bool ok = ct_step(C, ca.dyn, ctrl, ca.h, ca.tries, ca.rounds, ca.eps, slo, shi);
    ok_all = ok_all && ok;
    const int t = t0 + j, i = lane;
    if (lane < n) {
      double lo, hi;
      ct_point_box(C, i, lo, hi);
      double* bo = ca.boxes + ((size_t)b * (N + 1) + t + 1) * n * 2;
      bo[i * 2 + 0] = lo; bo[i * 2 + 1] = hi;
      if (ca.segs) {
        double* so = ca.segs + ((size_t)b * N + t) * n * 2;
        so[i * 2 + 0] = slo; so[i * 2 + 1] = shi;
      }
    }
    ct_precondition(C, n, ca.dyn.n_u, ctrl);
  }
  return ok_all;
}

}  // namespace dr
