// af_device.hpp -- device math of the Active Flux step (gfx950).
//
// Method: Chudzik, Helzel, Porfetye, "A fully discrete truly multidimensional Active Flux
// method for the two-dimensional Euler equations", arXiv 2508.06273.
//
// Everything here is templated on the bulk type R (float or double).  Quantities that the
// method needs in FP64 whatever R is (cell averages, conserved point values, fluxes, the
// positivity tests) are written with double explicitly.
//
// Evolution operators.  EG2 (Sec. 2, eq. EG2) and EG1 (Sec. 3, the first-order operator used
// on piecewise constant data) need integrals over the circle
//   Q(theta) = P' + c' tau (cos theta, sin theta),  P' = (x - u' tau, y - v' tau),
// of the reconstruction times 1, cos, sin, cos^2, sin cos, sin^2.  The circle lies in the
// cells around the degree of freedom; the grid lines through the DOF cut it where
// cos theta = u'/c' (vertical line) and sin theta = v'/c' (horizontal line).  In cell-local
// coordinates the circle is xi = xi0 + a C, eta = eta0 + b S (C = cos, S = sin), so each
// cell's biquadratic becomes a polynomial sum d_kl C^k S^l (k, l <= 2) and the integrals are
// exact combinations of the trigonometric moments  M_ab = int C^a S^b dtheta  over the arcs
// that lie in that cell.  The moments follow from the arc end points and the arc length by
// the standard reduction formulas, so the only transcendental functions are the two arc
// angles per evaluation (an acos and an asin).  The arc set of a cell is the intersection of the circular interval
// where Q is on that side of the vertical line with the one for the horizontal line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace af {

constexpr double kPi = 3.14159265358979323846;

// FP64 arc angles.  The circle crosses a grid line at a point (c, s) of the unit circle whose
// both coordinates the evolution operators form anyway (c = u'/c' or v'/c', s = sqrt(1 - c^2)),
// and the smaller of |c| and s is at most 1/sqrt(2): the angle is an arcsine of it, plus or
// minus a multiple of pi/2.  On 0 <= x <= 1/sqrt(2), asin(x) = x + x^3 g(x^2), g taken as its
// interpolant of degree 18 at the Chebyshev points of [0, 1/2] (coefficients from
// csrc/asin_coeffs.py; at most 0.09 ulp from asin with exact evaluation), evaluated by Estrin's
// scheme: 22 operations of dependency depth 6, against about 100 for the library's acos or
// asin with its long Horner chains.
constexpr double kAsinC[19] = {
    0.16666666666666669,    0.07499999999998412,   0.04464285714665563,
    0.030381944084994415,   0.0223721770065477,    0.017352221539201188,
    0.013975730180211136,   0.01139924601483468,   0.011310924828955462,
    -0.0032941927380090922, 0.07377343868679113,   -0.2809947932275328,
    0.952265420570822,      -2.3535297860232123,   4.3847119392409954,
    -5.883233416999023,     5.436384462318588,     -3.0948547605199717,
    0.8387674099544927};
__device__ __forceinline__ double asin_small(double x) {
  constexpr const double* a = kAsinC;  // constant subscripts below: folded to immediates
  const double t = x * x, t2 = t * t, t4 = t2 * t2, t8 = t4 * t4, t16 = t8 * t8;
  const double q0 = __builtin_fma(a[1], t, a[0]), q1 = __builtin_fma(a[3], t, a[2]);
  const double q2 = __builtin_fma(a[5], t, a[4]), q3 = __builtin_fma(a[7], t, a[6]);
  const double q4 = __builtin_fma(a[9], t, a[8]), q5 = __builtin_fma(a[11], t, a[10]);
  const double q6 = __builtin_fma(a[13], t, a[12]), q7 = __builtin_fma(a[15], t, a[14]);
  const double q8 = __builtin_fma(a[17], t, a[16]);
  const double r0 = __builtin_fma(q1, t2, q0), r1 = __builtin_fma(q3, t2, q2);
  const double r2 = __builtin_fma(q5, t2, q4), r3 = __builtin_fma(q7, t2, q6);
  const double r4 = __builtin_fma(a[18], t2, q8);
  const double s0 = __builtin_fma(r1, t4, r0), s1 = __builtin_fma(r3, t4, r2);
  const double p = __builtin_fma(r4, t16, __builtin_fma(s1, t8, s0));
  return __builtin_fma(x * t, p, x);
}

template <class R> struct Math;
template <> struct Math<double> {
  static __device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
  // acos(c) and asin(c) given s = sqrt(1 - c^2), |c| <= 1
  static __device__ __forceinline__ double acos_cs(double c, double s) {
    const bool mid = __builtin_fabs(c) <= s;  // the angle lies in [pi/4, 3pi/4]
    const double r = asin_small(mid ? c : s);
    return mid ? 0.5 * kPi - r : (c > 0.0 ? r : kPi - r);
  }
  static __device__ __forceinline__ double asin_cs(double c, double s) {
    const bool mid = __builtin_fabs(c) <= s;  // |asin c| <= pi/4
    const double r = asin_small(mid ? c : s);
    return mid ? r : __builtin_copysign(0.5 * kPi - r, c);
  }
};
template <> struct Math<float> {
  // hardware square root (1 ulp) rather than the correctly rounded expansion
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float acos_cs(float c, float) { return ::acosf(c); }
  static __device__ __forceinline__ float asin_cs(float c, float) { return ::asinf(c); }
};

template <class T> __device__ __forceinline__ T mx(T a, T b) { return a > b ? a : b; }
template <class T> __device__ __forceinline__ T mn(T a, T b) { return a < b ? a : b; }
template <class T> __device__ __forceinline__ T clamp1(T a) { return mn(mx(a, T(-1)), T(1)); }
// |x| in the precision of x (__builtin_fabs alone would widen a float to double)
__device__ __forceinline__ float absr(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absr(double x) { return __builtin_fabs(x); }

// ------------------------------------------------------------------------------------------
// Ideal gas (paper Sec. 2).  P2C is written without FMA contraction so that a host that
// evaluates E = p/(gamma-1) + 0.5*rho*(u*u + v*v) in this order obtains the same bits.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void p2c(const double U[4], double g1inv, double Q[4]) {
#pragma clang fp contract(off)
  Q[0] = U[0];
  Q[1] = U[0] * U[1];
  Q[2] = U[0] * U[2];
  Q[3] = U[3] * g1inv + 0.5 * U[0] * (U[1] * U[1] + U[2] * U[2]);
}

// Admissible: rho > 0 and p > 0 (zero and NaN fail).
template <class T> __device__ __forceinline__ bool admissible(T rho, T p) {
  return rho > T(0) && p > T(0);
}

// Primitive value of conserved Q by deviation from a reference primitive state W (exact
// identity; the rounding error scales with Q - P2C(W), and Q = P2C(W) returns W bitwise).
__device__ __forceinline__ void c2p_dev(const double W[4], const double dQ[4], double gm1,
                                        double U[4]) {
  double rho = W[0] + dQ[0];
  double irho = 1.0 / rho;
  double du = (dQ[1] - W[1] * dQ[0]) * irho;
  double dv = (dQ[2] - W[2] * dQ[0]) * irho;
  double u = W[1] + du, v = W[2] + dv;
  double dkin = dQ[0] * (u * u + v * v) + W[0] * (du * (u + W[1]) + dv * (v + W[2]));
  U[0] = rho;
  U[1] = u;
  U[2] = v;
  U[3] = W[3] + gm1 * (dQ[3] - 0.5 * dkin);
}

__device__ __forceinline__ void c2p_plain(const double Q[4], double gm1, double U[4]) {
  double irho = 1.0 / Q[0];
  U[0] = Q[0];
  U[1] = Q[1] * irho;
  U[2] = Q[2] * irho;
  U[3] = gm1 * (Q[3] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2]) * irho);
}

// f(q), g(q) evaluated from primitive values, FP64.
__device__ __forceinline__ void flux_fg(const double U[4], double g1inv, double F[4],
                                        double G[4]) {
  // fused multiply-adds written out and no other contraction: every kernel that inlines this
  // gets the same bits (the batched and single-grid paths agree exactly)
#pragma clang fp contract(off)
  const double r = U[0], u = U[1], v = U[2], p = U[3];
  const double q = __builtin_fma(u, u, v * v);
  const double H = __builtin_fma(p, g1inv, __builtin_fma(0.5 * r, q, p));  // E + p
  const double ru = r * u, rv = r * v;
  F[0] = ru;
  F[1] = __builtin_fma(ru, u, p);
  F[2] = ru * v;
  F[3] = u * H;
  G[0] = rv;
  G[1] = rv * u;
  G[2] = __builtin_fma(rv, v, p);
  G[3] = v * H;
}

__device__ __forceinline__ double wave_speed(const double U[4], double gamma) {
  // c = sqrt(gamma p / rho) = gamma p / sqrt(gamma p rho): one reciprocal square root instead
  // of a division and a square root
  const double gp = gamma * U[3];
  const double c = gp * ::rsqrt(gp * U[0]);
  return mx(__builtin_fabs(U[1]), __builtin_fabs(U[2])) + c;
}

// ------------------------------------------------------------------------------------------
// Correction term of Corollary 1: C(tau) = tau^2/2 * V(U, U_x, U_y).  Returns V/2.
// ------------------------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void corr_half(const R U[4], const R Ux[4], const R Uy[4], R gamma,
                                          R out[4]) {
  R rho = U[0], u = U[1], v = U[2], p = U[3];
  R rx = Ux[0], ux = Ux[1], vx = Ux[2], px = Ux[3];
  R ry = Uy[0], uy = Uy[1], vy = Uy[2], py = Uy[3];
  R irho = (sizeof(R) == 4) ? R(__builtin_amdgcn_rcpf(float(rho))) : R(1) / rho;
  R div = ux + vy;
  R f1 = ux * ux + uy * vx;
  R f2 = uy * vx + vy * vy;
  R g1 = px * (gamma * div + ux) + py * vx;
  R g2 = py * (gamma * div + vy) + px * uy;
  R h1 = (rx * px + ry * py) * irho;
  R h2 = (rx * u + ry * v) * irho * irho;
  out[0] = R(0.5) * (rho * (f1 + f2) + u * (rx * (ux + ux + vy) + ry * vx) +
                     v * (rx * uy + ry * (ux + vy + vy)) - h1);
  out[1] = R(0.5) * (u * f1 + v * uy * div + g1 * irho - px * h2);
  out[2] = R(0.5) * (v * f2 + u * vx * div + g2 * irho - py * h2);
  out[3] = R(0.5) * (u * g1 + v * g2 + gamma * p * (f1 + f2 - h1 * irho));
}

// ------------------------------------------------------------------------------------------
// Trigonometric moments over one arc.  M[a][b] = int_arc cos^a sin^b, for a, b <= 4 except
// (4,3), (3,4), (4,4), from the end points (Ca,Sa) -> (Cb,Sb) and the arc length L >= 0.
// Reduction formulas (m + n) int c^m s^n = c^(m-1) s^(n+1) + (m-1) int c^(m-2) s^n
//                                        = -c^(m+1) s^(n-1) + (n-1) int c^m s^(n-2).
// ------------------------------------------------------------------------------------------
template <class R> struct Mom {
  R m[5][5];
};

// Brackets [F] = F(end) - F(start) of the products F = c^i s^j that the reduction formulas
// need, summed over the pieces of an arc set, and the total length L.  The moments are
// linear in these sums, so an arc set of several pieces costs one recurrence.
template <class R> struct Br {
  R L, s1, c1, cs, c2s, c3s, c4s, c5s, c2, c3, c4, c5, cs2, c2s2, c3s2, c4s2, cs3, c2s3, c3s3;
};

template <class R> __device__ __forceinline__ void br_zero(Br<R>& B) {
  B.L = B.s1 = B.c1 = B.cs = B.c2s = B.c3s = B.c4s = B.c5s = B.c2 = B.c3 = B.c4 = B.c5 = R(0);
  B.cs2 = B.c2s2 = B.c3s2 = B.c4s2 = B.cs3 = B.c2s3 = B.c3s3 = R(0);
}

// add sign * F(c, s) for every product F
template <class R> __device__ __forceinline__ void br_end(Br<R>& B, R c, R s, R sign) {
  const R c2 = c * c, c3 = c2 * c, c4 = c2 * c2, c5 = c4 * c;
  const R s2 = s * s, s3 = s2 * s;
  const R sc = sign * c, ss = sign * s, ss2 = sign * s2, ss3 = sign * s3;
  B.s1 += ss;
  B.c1 += sc;
  B.cs += sc * s;
  B.c2s += c2 * ss;
  B.c3s += c3 * ss;
  B.c4s += c4 * ss;
  B.c5s += c5 * ss;
  B.c2 += sc * c;
  B.c3 += sign * c3;
  B.c4 += sign * c4;
  B.c5 += sign * c5;
  B.cs2 += c * ss2;
  B.c2s2 += c2 * ss2;
  B.c3s2 += c3 * ss2;
  B.c4s2 += c4 * ss2;
  B.cs3 += c * ss3;
  B.c2s3 += c2 * ss3;
  B.c3s3 += c3 * ss3;
}

// one piece (Ca,Sa) -> (Cb,Sb) of length L; empty pieces (L <= 0) add nothing
template <class R>
__device__ __forceinline__ void br_piece(Br<R>& B, R Ca, R Sa, R Cb, R Sb, R L) {
  if (L > R(0)) {
    B.L += L;
    br_end(B, Cb, Sb, R(1));
    br_end(B, Ca, Sa, R(-1));
  }
}

// Moments of the circle of radius a (M'[i][j] = a^(i+j) M[i][j]) from brackets taken at the
// scaled end points (a C, a S): the reduction formulas keep their form with a^2 on the
// lower-order moment.
template <class R>
__device__ __forceinline__ void moments(const Br<R>& B, R a2, Mom<R>& M) {
  const R i2 = R(0.5), i3 = R(1) / R(3), i4 = R(0.25), i5 = R(0.2), i6 = R(1) / R(6);
  const R b2 = a2 + a2, b3 = b2 + a2;
  M.m[0][0] = B.L;
  M.m[1][0] = B.s1;
  M.m[0][1] = -B.c1;
  M.m[2][0] = (B.cs + a2 * M.m[0][0]) * i2;
  M.m[3][0] = (B.c2s + b2 * M.m[1][0]) * i3;
  M.m[4][0] = (B.c3s + b3 * M.m[2][0]) * i4;
  M.m[1][1] = -B.c2 * i2;
  M.m[2][1] = -B.c3 * i3;
  M.m[3][1] = -B.c4 * i4;
  M.m[4][1] = -B.c5 * i5;
  M.m[0][2] = (a2 * M.m[0][0] - B.cs) * i2;
  M.m[1][2] = (a2 * M.m[1][0] - B.c2s) * i3;
  M.m[2][2] = (a2 * M.m[2][0] - B.c3s) * i4;
  M.m[3][2] = (a2 * M.m[3][0] - B.c4s) * i5;
  M.m[4][2] = (a2 * M.m[4][0] - B.c5s) * i6;
  M.m[0][3] = (b2 * M.m[0][1] - B.cs2) * i3;
  M.m[1][3] = (b2 * M.m[1][1] - B.c2s2) * i4;
  M.m[2][3] = (b2 * M.m[2][1] - B.c3s2) * i5;
  M.m[3][3] = (b2 * M.m[3][1] - B.c4s2) * i6;
  M.m[0][4] = (b3 * M.m[0][2] - B.cs3) * i4;
  M.m[1][4] = (b3 * M.m[1][2] - B.c2s3) * i5;
  M.m[2][4] = (b3 * M.m[2][2] - B.c3s3) * i6;
  M.m[4][3] = M.m[3][4] = M.m[4][4] = R(0);
}

// ------------------------------------------------------------------------------------------
// Cell polynomials.  LDS holds, for every halo cell and every primitive variable, the
// monomial coefficients c_mn of xi^m eta^n (m, n <= 2) in the cell-centred frame
// (xi, eta in [-1/2, 1/2]); c_00 is the centre value U_c.
// ------------------------------------------------------------------------------------------
// Lagrange nodes W[a][b] (a: left/centre/right, b: bottom/centre/top) -> monomials.
template <class T> __device__ __forceinline__ void nodes_to_monomials(const T W[3][3], T c[9]) {
  T t[3][3];  // t[m][b]: coefficient of xi^m on node row b
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    t[0][b] = W[1][b];
    t[1][b] = W[2][b] - W[0][b];
    t[2][b] = T(2) * (W[0][b] + W[2][b]) - T(4) * W[1][b];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    c[m * 3 + 0] = t[m][1];
    c[m * 3 + 1] = t[m][2] - t[m][0];
    c[m * 3 + 2] = T(2) * (t[m][0] + t[m][2]) - T(4) * t[m][1];
  }
}

// Substitute xi = xi0 + a C, eta = eta0 + a S into sum c_mn xi^m eta^n.  The result is
// sum e_kl (aC)^k (aS)^l; the powers of the radius a are carried by the moments (those of the
// circle of radius a), so the substitution itself needs no multiplication by a.  Both local
// coordinates are in units of dx (the y-coefficients are stored premultiplied by (dx/dy)^n).
// c00 is the constant coefficient (already a deviation); `ch` points at c_01 of one variable
// of one cell in LDS, the coefficients c_01 .. c_22 `stride` apart.
template <class R>
__device__ __forceinline__ void circle_shift(R c00, const R* __restrict__ ch, int stride, R xi0,
                                             R eta0, R d[9]) {
  R e[9];
  const R x2 = xi0 + xi0, y2 = eta0 + eta0;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    R c0 = n == 0 ? c00 : ch[(n - 1) * stride];
    R c1 = ch[(3 + n - 1) * stride], c2 = ch[(6 + n - 1) * stride];
    e[0 * 3 + n] = c0 + xi0 * (c1 + xi0 * c2);
    e[1 * 3 + n] = c1 + x2 * c2;
    e[2 * 3 + n] = c2;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R e0 = e[k * 3 + 0], e1 = e[k * 3 + 1], e2 = e[k * 3 + 2];
    d[k * 3 + 0] = e0 + eta0 * (e1 + eta0 * e2);
    d[k * 3 + 1] = e1 + y2 * e2;
    d[k * 3 + 2] = e2;
  }
}

// Polynomial value at (xi, eta) with constant coefficient c00 (see circle_shift).
template <class R>
__device__ __forceinline__ R poly_eval(R c00, const R* __restrict__ ch, int stride, R xi, R eta) {
  R r0 = c00 + eta * (ch[0 * stride] + eta * ch[1 * stride]);
  R r1 = ch[2 * stride] + eta * (ch[3 * stride] + eta * ch[4 * stride]);
  R r2 = ch[5 * stride] + eta * (ch[6 * stride] + eta * ch[7 * stride]);
  return r0 + xi * (r1 + xi * r2);
}

// Accumulators of the circle integrals of the deviations dp, du, dv from the linearisation
// state:  Ip = int dp, IpC = int dp C, IpS = int dp S, Jr = int (du C + dv S),
// Ju = int (du (2C^2 - 1/2) + 2 dv S C) = 2 Ua - Ub / 2,
// Jv = int (2 du S C + dv (2 S^2 - 1/2)) = 2 Va - Vb / 2, with Ua = int (du C^2 + dv S C),
// Ub = int du, Va = int (du S C + dv S^2), Vb = int dv (no per-arc moment combinations).
// With scaled moments IpC, IpS, Jr hold a times and Ua, Va a^2 times their values.
template <class R> struct Acc {
  R Ip, IpC, IpS, Jr, Ua, Ub, Va, Vb;
};

// Arc (-alpha, alpha) from (m, -s) to (m, s), symmetric in S: the moments with odd b vanish.
// Arc (beta, pi - beta) from (q, w) to (-q, w), symmetric in C: the moments with odd a vanish.
// Scaled moments of the circle of radius a, from the scaled end points ma = a m, sa = a s
// (qa = a q, wa = a w) and a2 = a^2: the reduction formulas above with the brackets of these
// end points written out.
template <class R>
__device__ __forceinline__ void moments_sym_x(R ma, R sa, R alpha, R a2, Mom<R>& M) {
  const R i3 = R(1) / R(3), i5 = R(0.2), i6 = R(1) / R(6);
  const R s2 = sa + sa;
  const R m1s = ma * s2, m2s = ma * m1s, m3s = ma * m2s, m4s = ma * m3s, m5s = ma * m4s;
  const R sa2 = sa * sa;
  const R b2 = a2 + a2, b3 = b2 + a2;
  M.m[0][0] = alpha + alpha;
  M.m[1][0] = s2;
  M.m[2][0] = R(0.5) * m1s + a2 * alpha;
  M.m[3][0] = (m2s + b2 * M.m[1][0]) * i3;
  M.m[4][0] = (m3s + b3 * M.m[2][0]) * R(0.25);
  M.m[0][2] = a2 * alpha - R(0.5) * m1s;
  M.m[1][2] = (a2 * M.m[1][0] - m2s) * i3;
  M.m[2][2] = (a2 * M.m[2][0] - m3s) * R(0.25);
  M.m[3][2] = (a2 * M.m[3][0] - m4s) * i5;
  M.m[4][2] = (a2 * M.m[4][0] - m5s) * i6;
  M.m[0][4] = (b3 * M.m[0][2] - m1s * sa2) * R(0.25);
  M.m[1][4] = (b3 * M.m[1][2] - m2s * sa2) * i5;
  M.m[2][4] = (b3 * M.m[2][2] - m3s * sa2) * i6;
}
template <class R>
__device__ __forceinline__ void moments_sym_y(R qa, R wa, R L, R a2, Mom<R>& M) {
  const R i3 = R(1) / R(3), i5 = R(0.2), i6 = R(1) / R(6);
  const R q2 = qa * qa, q3 = q2 * qa, q5 = q3 * q2, w2 = wa * wa;
  const R qw = qa * wa, q3w = q3 * wa;
  const R b2 = a2 + a2, b3 = b2 + a2;
  M.m[0][0] = L;
  M.m[0][1] = qa + qa;
  M.m[2][0] = R(0.5) * (a2 * L) - qw;
  M.m[4][0] = (b3 * M.m[2][0] - R(2) * q3w) * R(0.25);
  M.m[2][1] = R(2) * q3 * i3;
  M.m[4][1] = R(2) * q5 * i5;
  M.m[0][2] = R(0.5) * (a2 * L) + qw;
  M.m[2][2] = (a2 * M.m[2][0] + R(2) * q3w) * R(0.25);
  M.m[4][2] = (a2 * M.m[4][0] + R(2) * q5 * wa) * i6;
  M.m[0][3] = (R(2) * b2 * qa + R(2) * qw * wa) * i3;
  M.m[2][3] = (b2 * M.m[2][1] + R(2) * q3w * wa) * i5;
  M.m[0][4] = (b3 * M.m[0][2] + R(2) * qw * w2) * R(0.25);
  M.m[2][4] = (b3 * M.m[2][2] + R(2) * q3w * w2) * i6;
}

// Per-variable contractions with the moments of one arc set.  SYM = 1 (odd-b moments zero),
// 2 (odd-a moments zero) or 3 (full circle: both) drops the terms that vanish identically;
// SYM = 0 keeps all.
template <int SYM> __device__ __forceinline__ constexpr bool nz(int a, int b) {
  return SYM == 1 ? (b % 2 == 0)
                  : (SYM == 2 ? (a % 2 == 0) : (SYM == 3 ? (a % 2 == 0 && b % 2 == 0) : true));
}
template <int SYM, class R>
__device__ __forceinline__ void contract_p(const R d[9], const Mom<R>& M, Acc<R>& A) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const R x = d[k * 3 + l];
      if (nz<SYM>(k, l)) A.Ip += x * M.m[k][l];
      if (nz<SYM>(k + 1, l)) A.IpC += x * M.m[k + 1][l];
      if (nz<SYM>(k, l + 1)) A.IpS += x * M.m[k][l + 1];
    }
}
template <int SYM, class R>
__device__ __forceinline__ void contract_u(const R d[9], const Mom<R>& M, Acc<R>& A) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const R x = d[k * 3 + l];
      if (nz<SYM>(k + 1, l)) A.Jr += x * M.m[k + 1][l];
      if (nz<SYM>(k + 2, l)) A.Ua += x * M.m[k + 2][l];
      if (nz<SYM>(k, l)) A.Ub += x * M.m[k][l];
      if (nz<SYM>(k + 1, l + 1)) A.Va += x * M.m[k + 1][l + 1];
    }
}
template <int SYM, class R>
__device__ __forceinline__ void contract_v(const R d[9], const Mom<R>& M, Acc<R>& A) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const R x = d[k * 3 + l];
      if (nz<SYM>(k, l + 1)) A.Jr += x * M.m[k][l + 1];
      if (nz<SYM>(k + 1, l + 1)) A.Ua += x * M.m[k + 1][l + 1];
      if (nz<SYM>(k, l + 2)) A.Va += x * M.m[k][l + 2];
      if (nz<SYM>(k, l)) A.Vb += x * M.m[k][l];
    }
}

// Scaled moments of the full circle (SYM = 3: only even powers of C and S survive):
// int C^a S^b over [0, 2pi] = 2pi, pi, pi, 3pi/4, pi/4, 3pi/4, pi/8, pi/8 for
// (0,0),(2,0),(0,2),(4,0),(2,2),(0,4),(4,2),(2,4).
template <class R> __device__ __forceinline__ void full_moments(Mom<R>& M, R a) {
  const R pi = R(kPi), a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
  M.m[0][0] = R(2) * pi;
  M.m[2][0] = M.m[0][2] = pi * a2;
  M.m[4][0] = M.m[0][4] = R(0.75) * pi * a4;
  M.m[2][2] = R(0.25) * pi * a4;
  M.m[4][2] = M.m[2][4] = R(0.125) * pi * a6;
}

}  // namespace af
