// Continuous-time flowpipes with fixed-shape Taylor models (FP64), the device side of
// Section "Propagation under Continuous-Time Analytical Dynamics" (Theorem "TM flowpipe
// step via Picard iteration", appendix Algorithm "Reachability of CT Dynamics with TM
// Flowpipe") and of the inner loop of Algorithm "Reachability of CT NN Control Systems".
//
// A model is the quasi-quadratic form of Section "Representation of Reachable Sets" over
// the generators y in [-1, 1]^m (m <= 16) of the box and the time s in [0, h]:
//     X(y, s) = c + L y + l s + s (M y) + w s^2  (+)  [lo, hi],
// one component per lane of the first wavefront (component-parallel; n <= 16).
// Dynamics: f_i(x, u) = a_i + F_i x + G_i u + x^T Q_i x (degree <= 2 in the state, affine
// in the held input u).  Products keep the monomials {1, y, s, s y, s^2} and bound every
// other one over the domain into the interval part.  The step: two Picard iterations of
// the polynomial part from the seed c + S y; the remainder J validated by the Picard
// image J' = I_0 + hull(0, h range(f(p + J) - d/ds p)) inside J (widening while not),
// then refined; the step-end model c + l h + w h^2 + (L + h M) y (+) J; the remainder is
// then absorbed into the linear part (S <- S diag(1 + |S^-1| rad J), centre += mid J)
// when S is well conditioned, and a held input's model follows the change of generators.
// Arithmetic is FP64 without outward rounding (the rounding of these steps is not
// covered by a margin).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"

namespace dr {

constexpr int kCtMax = 16;

// One component of a model in registers.
struct QT {
  double c, L[kCtMax], l, M[kCtMax], w, lo, hi;
};

// A vector of models in LDS (structure of arrays, component-major 16 x 16 matrices).
struct QTL {
  double* c;
  double* L;
  double* l;
  double* M;
  double* w;
  double* lo;
  double* hi;
  __host__ __device__ static size_t bytes() { return (size_t)(5 * kCtMax + 2 * kCtMax * kCtMax) * sizeof(double); }
  __device__ void carve(double* base) {
    c = base; L = c + kCtMax; l = L + kCtMax * kCtMax; M = l + kCtMax; w = M + kCtMax * kCtMax;
    lo = w + kCtMax; hi = lo + kCtMax;
  }
};

__device__ __forceinline__ QT qt_get(const QTL& t, int i) {
  QT q;
  q.c = t.c[i]; q.l = t.l[i]; q.w = t.w[i]; q.lo = t.lo[i]; q.hi = t.hi[i];
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) { q.L[p] = t.L[i * kCtMax + p]; q.M[p] = t.M[i * kCtMax + p]; }
  return q;
}
__device__ __forceinline__ void qt_put(const QTL& t, int i, const QT& q) {
  t.c[i] = q.c; t.l[i] = q.l; t.w[i] = q.w; t.lo[i] = q.lo; t.hi[i] = q.hi;
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) { t.L[i * kCtMax + p] = q.L[p]; t.M[i * kCtMax + p] = q.M[p]; }
}
__device__ __forceinline__ QT qt_zero() {
  QT q;
  q.c = q.l = q.w = q.lo = q.hi = 0.0;
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) { q.L[p] = 0.0; q.M[p] = 0.0; }
  return q;
}

// Range of the polynomial part over y in [-1, 1]^m, s in [0, h] (term by term).
__device__ __forceinline__ void qt_poly_range(const QT& q, double h, double& lo, double& hi) {
  double r = 0.0;
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) r += fabs(q.L[p]) + h * fabs(q.M[p]);
  lo = q.c - r + fmin(0.0, q.l * h) + fmin(0.0, q.w * h * h);
  hi = q.c + r + fmax(0.0, q.l * h) + fmax(0.0, q.w * h * h);
}

__device__ __forceinline__ void iv_mul(double alo, double ahi, double blo, double bhi, double& lo, double& hi) {
  const double p0 = alo * blo, p1 = alo * bhi, p2 = ahi * blo, p3 = ahi * bhi;
  lo = fmin(fmin(p0, p1), fmin(p2, p3));
  hi = fmax(fmax(p0, p1), fmax(p2, p3));
}

// out += q * (a b) for scalar models a, b (the product truncated to the representation,
// the dropped monomials and the interval parts bounded over the domain).
__device__ __forceinline__ void qt_mul_acc(QT& out, const QT& a, const QT& b, double q, double h) {
  double lo = 0.0, hi = 0.0;
  // (L_a y)(L_b y): y_p^2 in [0, 1], y_p y_r in [-1, 1]
  double dsum_lo = 0.0, dsum_hi = 0.0, off = 0.0, sLa = 0.0, sLb = 0.0, sMa = 0.0, sMb = 0.0;
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) {
    sLa += fabs(a.L[p]); sLb += fabs(b.L[p]); sMa += fabs(a.M[p]); sMb += fabs(b.M[p]);
    const double d = a.L[p] * b.L[p];
    dsum_lo += fmin(d, 0.0); dsum_hi += fmax(d, 0.0);
    off -= fabs(d);
  }
  off += sLa * sLb;
  lo += dsum_lo - off; hi += dsum_hi + off;
  // s y y, s^2 y, s^2 y y, s^3, s^3 y, s^4
  const double t1 = h * (sLa * sMb + sMa * sLb);
  const double t2 = h * h * (fabs(a.l) * sMb + fabs(b.l) * sMa + fabs(a.w) * sLb + fabs(b.w) * sLa);
  const double t3 = h * h * sMa * sMb;
  const double t4 = h * h * h * (fabs(a.w) * sMb + fabs(b.w) * sMa);
  lo -= t1 + t2 + t3 + t4; hi += t1 + t2 + t3 + t4;
  const double s3 = (a.l * b.w + a.w * b.l) * h * h * h, s4 = a.w * b.w * h * h * h * h;
  lo += fmin(0.0, s3) + fmin(0.0, s4); hi += fmax(0.0, s3) + fmax(0.0, s4);
  // interval parts
  double alo, ahi, blo, bhi, x0, x1;
  qt_poly_range(a, h, alo, ahi);
  qt_poly_range(b, h, blo, bhi);
  iv_mul(a.lo, a.hi, blo, bhi, x0, x1); lo += x0; hi += x1;
  iv_mul(b.lo, b.hi, alo, ahi, x0, x1); lo += x0; hi += x1;
  iv_mul(a.lo, a.hi, b.lo, b.hi, x0, x1); lo += x0; hi += x1;
  // kept monomials, scaled by q
  out.c += q * (a.c * b.c);
  out.l += q * (a.c * b.l + b.c * a.l);
  out.w += q * (a.c * b.w + b.c * a.w + a.l * b.l);
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) {
    out.L[p] += q * (a.c * b.L[p] + b.c * a.L[p]);
    out.M[p] += q * (a.c * b.M[p] + b.c * a.M[p] + a.l * b.L[p] + b.l * a.L[p]);
  }
  const double ql = q * lo, qh = q * hi;
  out.lo += fmin(ql, qh); out.hi += fmax(ql, qh);
}

// out += F x for a scalar weight F (the interval part by its sign).
__device__ __forceinline__ void qt_axpy(QT& out, double F, const QT& x) {
  out.c += F * x.c; out.l += F * x.l; out.w += F * x.w;
#pragma unroll
  for (int p = 0; p < kCtMax; ++p) { out.L[p] += F * x.L[p]; out.M[p] += F * x.M[p]; }
  if (F >= 0.0) { out.lo += F * x.lo; out.hi += F * x.hi; }
  else { out.lo += F * x.hi; out.hi += F * x.lo; }
}

struct CtDyn {
  int n, n_u;
  const double* a;     // n
  const double* F;     // n x n
  const double* G;     // n x n_u (or null)
  const double* Q;     // n x n x n (or null)
};

// Component i of f over the state models X and the held input models U (U may be null).
__device__ __forceinline__ QT qt_f(int i, const QTL& X, const QTL* U, const CtDyn& d, double h) {
  QT out = qt_zero();
  out.c = d.a[i];
  for (int j = 0; j < d.n; ++j) {
    const double Fv = d.F[(size_t)i * d.n + j];
    if (Fv != 0.0) qt_axpy(out, Fv, qt_get(X, j));
  }
  if (U && d.G) {
    for (int k = 0; k < d.n_u; ++k) {
      const double Gv = d.G[(size_t)i * d.n_u + k];
      if (Gv != 0.0) qt_axpy(out, Gv, qt_get(*U, k));
    }
  }
  if (d.Q) {
    for (int j = 0; j < d.n; ++j)
      for (int k = 0; k < d.n; ++k) {
        const double q = d.Q[((size_t)i * d.n + j) * d.n + k];
        if (q != 0.0) qt_mul_acc(out, qt_get(X, j), qt_get(X, k), q, h);
      }
  }
  return out;
}

// Per-box LDS of the flowpipe: the seed, the Picard iterate / polynomial part, the
// model used for the remainder images, the held input, work space.
struct CtLds {
  QTL G, X, U;
  double* S;        // 16 x 16 seed linear part (the state model c + S y + [lo, hi])
  double* c;        // 16
  double* lo;       // 16
  double* hi;       // 16
  double* Si;       // 16 x 16 inverse of S (preconditioning)
  double* aux;      // 16: column scales of the preconditioning
  double* aug;      // 16 x 32: [S | I] during the inversion
  __host__ __device__ static size_t bytes() {
    return 3 * QTL::bytes() + (size_t)(2 * kCtMax * kCtMax + 4 * kCtMax + 2 * kCtMax * kCtMax) * sizeof(double);
  }
  __device__ void carve(double* base) {
    G.carve(base); base += QTL::bytes() / sizeof(double);
    X.carve(base); base += QTL::bytes() / sizeof(double);
    U.carve(base); base += QTL::bytes() / sizeof(double);
    S = base; base += kCtMax * kCtMax;
    c = base; base += kCtMax;
    lo = base; base += kCtMax;
    hi = base; base += kCtMax;
    Si = base; base += kCtMax * kCtMax;
    aux = base; base += kCtMax;
    aug = base;
  }
};

__device__ __forceinline__ void ct_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
}

// One flowpipe step on the first wavefront (lanes < n own a component): seed
// (C.c, C.S, C.lo, C.hi), held input C.U (if `ctrl`).  On return the step-end model is
// the new seed (preconditioned), seg (per lane) the box of the segment, and the return
// value says whether a contractive remainder was found (the same on every lane).
__device__ __forceinline__ bool ct_step(const CtLds& C, const CtDyn& d, bool ctrl, double h, int tries, int rounds,
                                        double eps, double& seg_lo, double& seg_hi) {
  const int i = threadIdx.x;          // component (lanes of wave 0)
  const int n = d.n;
  const bool act = i < n;
  const QTL* U = ctrl ? &C.U : nullptr;
  // ---- polynomial Picard: g_0 = c + S y, g_{j+1} = x_0 + trunc(int f(g_j))
  QT x0 = qt_zero();
  if (act) {
    x0.c = C.c[i];
#pragma unroll
    for (int p = 0; p < kCtMax; ++p) x0.L[p] = C.S[i * kCtMax + p];
    qt_put(C.G, i, x0);
  }
  ct_sync();
  for (int it = 0; it < 2; ++it) {
    QT g = qt_zero();
    if (act) {
      const QT fx = qt_f(i, C.G, U, d, h);
      g = x0;
      g.l += fx.c;
      g.w += 0.5 * fx.l;
#pragma unroll
      for (int p = 0; p < kCtMax; ++p) g.M[p] += fx.L[p];
      g.lo = 0.0; g.hi = 0.0;
    }
    ct_sync();
    if (act) qt_put(C.G, i, g);
    ct_sync();
  }
  // p is in C.G; d/ds p = l + M y + 2 w s
  QT p = act ? qt_get(C.G, i) : qt_zero();
  QT dp = qt_zero();
  dp.c = p.l; dp.l = 2.0 * p.w;
#pragma unroll
  for (int q = 0; q < kCtMax; ++q) dp.L[q] = p.M[q];
  const double I0lo = act ? C.lo[i] : 0.0, I0hi = act ? C.hi[i] : 0.0;
  auto image = [&](double Jlo, double Jhi, double& nlo, double& nhi) {
    if (act) {
      QT xj = p;
      xj.lo = Jlo; xj.hi = Jhi;
      qt_put(C.X, i, xj);
    }
    ct_sync();
    nlo = 0.0; nhi = 0.0;
    if (act) {
      QT D = qt_f(i, C.X, U, d, h);
      // D - dp (dp has no interval part)
      D.c -= dp.c; D.l -= dp.l;
#pragma unroll
      for (int q = 0; q < kCtMax; ++q) D.L[q] -= dp.L[q];
      double plo, phi;
      qt_poly_range(D, h, plo, phi);
      nlo = I0lo + fmin(0.0, h * (plo + D.lo));
      nhi = I0hi + fmax(0.0, h * (phi + D.hi));
    }
    ct_sync();
  };
  double Jlo = I0lo - eps, Jhi = I0hi + eps, nlo, nhi;
  bool ok = false;
  // an unbounded initial set has no bounded remainder
  const int ntry = __any(!(fabs(I0lo) < INFINITY) || !(fabs(I0hi) < INFINITY)) ? 0 : tries;
  for (int t = 0; t < ntry; ++t) {
    image(Jlo, Jhi, nlo, nhi);
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
      image(Jlo, Jhi, nlo, nhi);
      Jlo = fmax(Jlo, nlo); Jhi = fmin(Jhi, nhi);
    }
  } else {
    Jlo = -INFINITY; Jhi = INFINITY;
  }
  // segment box, step-end model
  if (act) {
    double plo, phi;
    qt_poly_range(p, h, plo, phi);
    seg_lo = plo + Jlo; seg_hi = phi + Jhi;
    C.c[i] = p.c + p.l * h + p.w * h * h;
#pragma unroll
    for (int q = 0; q < kCtMax; ++q) C.S[i * kCtMax + q] = p.L[q] + h * p.M[q];
    C.lo[i] = Jlo; C.hi[i] = Jhi;
  }
  ct_sync();
  return ok;
}

// Step (A): absorb the remainder into the linear part when S is well conditioned; the
// held input follows.  Wave 0: S^-1 by Gauss-Jordan with partial pivoting (first largest
// pivot) on the augmented matrix [S | I] in LDS, one column per lane.
__device__ __forceinline__ void ct_precondition(const CtLds& C, int n, int n_u, bool ctrl) {
  const int i = threadIdx.x;
  double* aug = C.aug;   // n x 2n, row stride 2 kCtMax
  constexpr int ld = 2 * kCtMax;
  bool fin = true;
  if (i < n) {
    fin = fabs(C.lo[i]) < INFINITY && fabs(C.hi[i]) < INFINITY;
    for (int q = 0; q < n; ++q) fin = fin && fabs(C.S[i * kCtMax + q]) < INFINITY;
  }
  bool good = !__any(!fin);
  if (i < 2 * n)
    for (int r = 0; r < n; ++r) aug[r * ld + i] = i < n ? C.S[r * kCtMax + i] : (i - n == r ? 1.0 : 0.0);
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
  // S^-1 and the check of S^-1 S against the identity
  double err = 0.0;
  if (good) {
    for (int e = i; e < n * n; e += 64) {
      const int r = e / n, q = e % n;
      C.Si[r * kCtMax + q] = aug[r * ld + n + q];
    }
    ct_sync();
    for (int e = i; e < n * n; e += 64) {
      const int r = e / n, q = e % n;
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += C.Si[r * kCtMax + k] * C.S[k * kCtMax + q];
      const double d = fabs(v - (r == q ? 1.0 : 0.0));
      if (!(d <= err)) err = d;
    }
  }
  good = good && !__any(!(err <= 1e-9));
  if (!good) return;
  // delta_j = sum_k |Si_jk| rad_k; input extra_r = sum_j |(P_u Si)_rj| rad_j
  double Dj = 1.0;
  if (i < n) {
    double dl = 0.0;
    for (int k = 0; k < n; ++k) dl += fabs(C.Si[i * kCtMax + k]) * 0.5 * (C.hi[k] - C.lo[k]);
    Dj = 1.0 + dl;
  }
  double extra = 0.0;
  if (ctrl && i < n_u) {
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += C.U.L[i * kCtMax + k] * C.Si[k * kCtMax + j];
      extra += fabs(v) * 0.5 * (C.hi[j] - C.lo[j]);
    }
  }
  ct_sync();
  if (i < n) C.aux[i] = Dj;
  ct_sync();
  if (i < n) {
    C.c[i] += 0.5 * (C.lo[i] + C.hi[i]);
    for (int q = 0; q < n; ++q) C.S[i * kCtMax + q] *= C.aux[q];
    C.lo[i] = 0.0; C.hi[i] = 0.0;
  }
  if (ctrl && i < n_u) {
    for (int q = 0; q < n; ++q) C.U.L[i * kCtMax + q] *= C.aux[q];
    C.U.lo[i] -= extra; C.U.hi[i] += extra;
  }
  ct_sync();
}

}  // namespace dr

namespace dr {

struct CtArgs {
  BatchDev batch;
  Scratch sc;
  CtDyn dyn;
  double h;
  int K;             // flowpipe steps per control interval
  int n_ctl;         // control intervals (without a controller: one interval of K steps each)
  int tries, rounds;
  double eps;
  double* boxes;     // S x (n_ctl K + 1) x n x 2: time points
  double* segs;      // S x n_ctl K x n x 2: segments (nullable)
  uint32_t* status;
};

// Box of the state model (c, S, lo, hi) for component i.
__device__ __forceinline__ void ct_point_box(const CtLds& C, int i, double& lo, double& hi) {
  double r = 0.0;
  for (int q = 0; q < kCtMax; ++q) r += fabs(C.S[i * kCtMax + q]);
  lo = C.c[i] - r + C.lo[i];
  hi = C.c[i] + r + C.hi[i];
}

// The seed of box b: c = centre, S = diag(radius), no remainder (wave 0).
__device__ __forceinline__ void ct_seed(const CtLds& C, const CtArgs& ca, int b, int n0) {
  const int i = threadIdx.x, n = ca.dyn.n;
  if (i < kCtMax) {
    C.c[i] = i < n ? ca.batch.xc[(size_t)b * n0 + i] : 0.0;
    C.lo[i] = 0.0; C.hi[i] = 0.0;
  }
  for (int e = i; e < kCtMax * kCtMax; e += 64) {
    const int r = e / kCtMax, q = e % kCtMax;
    C.S[e] = (r == q && r < n) ? ca.batch.xr[(size_t)b * n0 + r] : 0.0;
  }
  ct_sync();
}

// K flowpipe steps from the current seed (wave 0), writing time-point boxes t0+1 ..
// t0+K and segment boxes t0 .. t0+K-1; returns false if a step found no contractive
// remainder.
__device__ __forceinline__ bool ct_steps(const CtLds& C, const CtArgs& ca, bool ctrl, int b, int t0) {
  const int i = threadIdx.x, n = ca.dyn.n;
  const int N = ca.n_ctl * ca.K;
  bool ok_all = true;
  for (int j = 0; j < ca.K; ++j) {
    double slo = 0.0, shi = 0.0;
    const bool ok = ct_step(C, ca.dyn, ctrl, ca.h, ca.tries, ca.rounds, ca.eps, slo, shi);
    ok_all = ok_all && ok;
    const int t = t0 + j;
    if (i < n) {
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
