// FP64 CPU oracle for the vortex-particle hot path — TEST INFRASTRUCTURE ONLY.
//
// This file is the plain, slow reference against which the HIP library is checked.
// Only the test-suite, the smoke check and the benchmark's CPU-baseline leg load it;
// the product path never links or calls it, and it shares no code, header or constant
// with the GPU library.
//
// What it computes (paper: Fu & Laurendeau, "Nonlinear Unsteady Vortex-Lattice
// Vortex-Particle Method with Adaptive Wake Conversion", Sec. II.B, Eqs. 2-5, and
// Sec. II.A for the Vatistas-cored segments):
//
//   * particle field  w(x) = sum_j Gamma_j zeta_sigma(x - x_j)                 (Eq. 2)
//     with the 3-D Gaussian zeta_sigma(rho) = (2 pi sigma^2)^(-3/2) exp(-rho^2/2) (Eq. 3)
//   * velocity (Biot-Savart of that field, Eq. 4's right-hand side)
//         u_i = sum_{j != i} g(s) Gamma_j x r,  r = x_i - x_j, s = |r|
//         g(s) = q(rho) / (4 pi s^3),  q(rho) = erf(rho/sqrt2) - c0 rho exp(-rho^2/2)
//     q is the fraction of a unit Gaussian blob inside radius rho, c0 = sqrt(2/pi).
//   * stretching, transposed scheme (first term of Eq. 5, (Gamma_i . grad^T) u):
//         dGamma_i/dt = sum_{j != i} [ g Gamma_i x Gamma_j + h (Gamma_i . (Gamma_j x r)) r ]
//     h(s) = g'(s)/s.  Classical option (Gamma_i . grad) u:
//         sum_{j != i} [ g Gamma_j x Gamma_i + h (r . Gamma_i) (Gamma_j x r) ]
//   * velocity gradient J_i[a][b] = d u_a / d x_b at the targets (sources held fixed):
//         J = sum_{j != i} [ g [Gamma_j]_x + h (Gamma_j x r) r^T ]
//     where [w]_x is the cross-product matrix ([w]_x y = w x y).  The stretching of Eq. 5
//     is J^T Gamma_i (transposed) or J Gamma_i (classical).
//   * viscous term of Eq. 5, nu lap(Gamma_i), by particle strength exchange (PSE) with the
//     Gaussian of Eq. 3 as the exchange kernel (Sec. II.B names PSE):
//         dGamma_i/dt = sum_{j != i} (2 nu_ij / sigma_ij^2) (V_i Gamma_j - V_j Gamma_i) zeta_{sigma_ij}(|r|)
//     V = particle volume (an input), sigma_ij^2 = (sigma_i^2 + sigma_j^2)/2 and
//     nu_ij = nu + (nu_t,i + nu_t,j)/2 (symmetric in i, j, so sum_i dGamma_i/dt = 0).
//   * Vreman's sub-grid eddy viscosity (Sec. II.B, C_V = 0.07) from J, filter width sigma_i:
//         nu_t = C_V sqrt(B_beta / (alpha_ab alpha_ab)),  alpha_ab = d u_b / d x_a = J[b][a],
//         beta_ab = sigma^2 sum_m alpha_ma alpha_mb,
//         B_beta = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2  (0 where alpha = 0).
//   * straight-segment velocity with a Vatistas core (Sec. II.A): finite-segment
//     Biot-Savart multiplied by d^2 / (d^(2n) + rc^(2n))^(1/n), d = distance to the line.
//   * low-storage third-order Runge-Kutta (Williamson 2N-storage, Sec. II.B) for
//     (x_i, Gamma_i), and the loss L = sum_c (u_c . z)^2 on control points.
//   * forward-mode tangents of all of the above on dual numbers (gradient oracle).
//
// Kernel weights are evaluated exactly as defined: for rho >= 1 the closed form with
// std::erf/std::exp; for rho < 1 the Taylor series of q(rho)/rho^3 (and of the derived
// weights) in rho^2, because the closed form cancels catastrophically there.  There is
// no far-field shortcut.  Per-target sums use Neumaier compensation, and the file is
// compiled with -ffp-contract=off.
//
// Readings where the paper is silent (see the design notes): source-sigma rule by
// default, symmetric rule sigma_ij^2 = (sigma_i^2 + sigma_j^2)/2 as an option; self pair
// excluded by index; Vatistas exponent n given by the caller (2 by default); segments
// with a vanishing arm or length contribute nothing.

#include <array>
#include <cmath>
#include <cstdlib>
#include <map>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

const double kPi = 3.14159265358979323846264338327950288;
const double kC0 = 0.79788456080286535587989211986876373;  // sqrt(2/pi)
const double kInvSqrt2 = 0.70710678118654752440084436210484903;
const double kTwoOverSqrtPi = 1.12837916709551257389615890312154517;

// ---------------------------------------------------------------- dual numbers
// Forward-mode scalar: value v and one directional derivative d.
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline bool operator<(Dual a, double b) { return a.v < b; }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
inline Dual dsqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, s > 0 ? a.d / (2 * s) : 0.0); }
inline double dsqrt(double a) { return std::sqrt(a); }
inline Dual dexp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline double dexp(double a) { return std::exp(a); }
inline Dual derf(Dual a) { return Dual(std::erf(a.v), kTwoOverSqrtPi * std::exp(-a.v * a.v) * a.d); }
inline double derf(double a) { return std::erf(a); }
inline Dual dpow(Dual a, double p) {  // a > 0
    double r = std::pow(a.v, p);
    return Dual(r, p * std::pow(a.v, p - 1.0) * a.d);
}
inline double dpow(double a, double p) { return std::pow(a, p); }

// Hyper-dual scalar: value v, derivatives a and b along two directions, and the mixed second
// derivative ab.  A function f of one argument maps x to
//   (f, f' x.a, f' x.b, f' x.ab + f'' x.a x.b).
struct HDual {
    double v, a, b, ab;
    HDual() : v(0), a(0), b(0), ab(0) {}
    HDual(double x) : v(x), a(0), b(0), ab(0) {}
    HDual(double x, double da, double db, double dab) : v(x), a(da), b(db), ab(dab) {}
};
inline HDual chain(const HDual& x, double f, double f1, double f2) {
    return HDual(f, f1 * x.a, f1 * x.b, f1 * x.ab + f2 * x.a * x.b);
}
inline HDual operator+(HDual x, HDual y) { return HDual(x.v + y.v, x.a + y.a, x.b + y.b, x.ab + y.ab); }
inline HDual operator-(HDual x, HDual y) { return HDual(x.v - y.v, x.a - y.a, x.b - y.b, x.ab - y.ab); }
inline HDual operator-(HDual x) { return HDual(-x.v, -x.a, -x.b, -x.ab); }
inline HDual operator*(HDual x, HDual y) {
    return HDual(x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b,
                 x.ab * y.v + x.a * y.b + x.b * y.a + x.v * y.ab);
}
inline HDual operator/(HDual x, HDual y) {
    const double r = 1.0 / y.v;
    return x * chain(y, r, -r * r, 2.0 * r * r * r);
}
inline HDual& operator+=(HDual& x, HDual y) { x = x + y; return x; }
inline bool operator<(HDual x, double y) { return x.v < y; }
inline double val(HDual x) { return x.v; }
inline HDual dsqrt(HDual x) {
    const double s = std::sqrt(x.v);
    if (!(s > 0)) return HDual(s, 0, 0, 0);
    return chain(x, s, 0.5 / s, -0.25 / (s * x.v));
}
inline HDual dpow(HDual x, double p) {  // x > 0
    return chain(x, std::pow(x.v, p), p * std::pow(x.v, p - 1.0), p * (p - 1.0) * std::pow(x.v, p - 2.0));
}

// ---------------------------------------------------------------- compensated sum
// Neumaier's variant of Kahan summation, applied separately to value and tangent.
struct Neumaier {
    double s = 0, c = 0;
    void add(double x) {
        double t = s + x;
        if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    double get() const { return s + c; }
};
template <class T> struct Acc;
template <> struct Acc<double> {
    Neumaier a;
    void add(double x) { a.add(x); }
    double get() const { return a.get(); }
};
template <> struct Acc<Dual> {
    Neumaier a, b;
    void add(Dual x) { a.add(x.v); b.add(x.d); }
    Dual get() const { return Dual(a.get(), b.get()); }
};
template <> struct Acc<HDual> {
    Neumaier v, a, b, ab;
    void add(HDual x) { v.add(x.v); a.add(x.a); b.add(x.b); ab.add(x.ab); }
    HDual get() const { return HDual(v.get(), a.get(), b.get(), ab.get()); }
};

template <class T> struct V3 { T x, y, z; };
template <class T> inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> inline T dot(const V3<T>& a, const V3<T>& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class T> inline V3<T> sub(const V3<T>& a, const V3<T>& b) {
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}

// ---------------------------------------------------------------- kernel weights
// Dimensionless weights of the Gaussian blob as functions of rho (Eq. 3):
//   Gw = q/rho^3,  Hw = (rho q' - 3 q)/rho^5,  Kw = (rho^2 q'' - 7 rho q' + 15 q)/rho^7
// so that g = Gw/(4 pi sigma^3), h = g'/s = Hw/(4 pi sigma^5), k = h'/s = Kw/(4 pi sigma^7).
// For rho < 1 the Taylor series in t = rho^2 (20 terms); otherwise the closed form.
// Taylor series: q(rho) = c0 sum_n (-1)^n rho^(2n+3) / ((2n+3) 2^n n!).
const int kSeriesTerms = 20;

template <class T>
void weights(T rho, T* Gw, T* Hw, T* Kw) {
    if (rho < 1.0) {
        T t = rho * rho;
        T sg(0.0), sh(0.0), sk(0.0);
        // a_n = 1 / (2^n n!)
        double a[kSeriesTerms + 1];
        a[0] = 1.0;
        for (int n = 1; n <= kSeriesTerms; ++n) a[n] = a[n - 1] / (2.0 * n);
        // Sum from the highest term down (terms decrease in magnitude for t < 1).
        for (int n = kSeriesTerms; n >= 0; --n) {
            double sgn = (n % 2) ? -1.0 : 1.0;
            double cg = sgn * a[n] / (2 * n + 3);
            sg = sg * t + T(cg);
            if (n >= 1) sh = sh * t + T(cg * 2.0 * n);
            if (n >= 2) sk = sk * t + T(cg * 4.0 * n * (n - 1));
        }
        *Gw = T(kC0) * sg;
        *Hw = T(kC0) * sh;
        *Kw = T(kC0) * sk;
    } else {
        T e = dexp(T(-0.5) * rho * rho);
        T q = derf(rho * T(kInvSqrt2)) - T(kC0) * rho * e;
        T r2 = rho * rho;
        T r3 = r2 * rho;
        T r5 = r3 * r2;
        T r7 = r5 * r2;
        *Gw = q / r3;
        *Hw = (T(kC0) * r3 * e - T(3.0) * q) / r5;
        *Kw = (T(15.0) * q - T(kC0) * e * (T(5.0) * r3 + r5)) / r7;
    }
}

// g, h (and k) at separation s for core size sigma.
template <class T>
void ghk(T s, T sigma, T* g, T* h, T* k) {
    T rho = s / sigma;
    T Gw, Hw, Kw;
    weights(rho, &Gw, &Hw, &Kw);
    T s2 = sigma * sigma;
    T s3 = s2 * sigma;
    T s5 = s3 * s2;
    T s7 = s5 * s2;
    T f = T(1.0 / (4.0 * kPi));
    *g = f * Gw / s3;
    *h = f * Hw / s5;
    if (k) *k = f * Kw / s7;
}

template <class T> inline V3<T> load3(const T* a, int64_t ld, int64_t i) {
    return {a[i], a[ld + i], a[2 * ld + i]};
}

// ---------------------------------------------------------------- particle sums
// u_t and dGamma_t/dt at every target t from every source j (Eqs. 2-5).
// Arrays are [3][n] (component-major).  gam_t == nullptr: velocity only.
// excl[t] = index of the source that is the same particle as target t (skipped), or -1.
template <class T>
void eval_pairs(int64_t ns, const T* xs, const T* gs, const double* sgs,
                int64_t nt, const T* xt, const T* gt, const double* sgt,
                const int64_t* excl, int scheme, int sigma_rule, T* u, T* dg) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        V3<T> xi = load3(xt, nt, t);
        V3<T> Gi = {T(0.0), T(0.0), T(0.0)};
        if (gt) Gi = load3(gt, nt, t);
        Acc<T> au[3], ad[3];
        for (int64_t j = 0; j < ns; ++j) {
            if (excl && excl[t] == j) continue;
            V3<T> xj = load3(xs, ns, j);
            V3<T> Gj = load3(gs, ns, j);
            V3<T> r = sub(xi, xj);
            T s = dsqrt(dot(r, r));
            double sig = sgs[j];
            if (sigma_rule == 1) sig = std::sqrt(0.5 * (sgt[t] * sgt[t] + sgs[j] * sgs[j]));
            T g, h;
            ghk<T>(s, T(sig), &g, &h, nullptr);
            V3<T> v = cross(Gj, r);
            au[0].add(g * v.x);
            au[1].add(g * v.y);
            au[2].add(g * v.z);
            if (gt) {
                V3<T> term;
                if (scheme == 0) {  // transposed
                    V3<T> c = cross(Gi, Gj);
                    T tau = dot(Gi, v);
                    term = {g * c.x + h * tau * r.x, g * c.y + h * tau * r.y, g * c.z + h * tau * r.z};
                } else {  // classical
                    V3<T> c = cross(Gj, Gi);
                    T rg = dot(r, Gi);
                    term = {g * c.x + h * rg * v.x, g * c.y + h * rg * v.y, g * c.z + h * rg * v.z};
                }
                ad[0].add(term.x);
                ad[1].add(term.y);
                ad[2].add(term.z);
            }
        }
        for (int c = 0; c < 3; ++c) {
            u[c * nt + t] = au[c].get();
            if (gt) dg[c * nt + t] = ad[c].get();
        }
    }
}

// ---------------------------------------------------------------- segments
// Velocity at targets induced by straight vortex segments A->B with circulation gam
// (Sec. II.A: Biot-Savart of the vortex-ring edges with the Vatistas core).
template <class T>
void eval_segments(int64_t nseg, const double* A, const double* B, const double* gam,
                   double rc, int vn, int64_t nt, const T* xt, T* u) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        V3<T> P = load3(xt, nt, t);
        Acc<T> au[3];
        for (int64_t k = 0; k < nseg; ++k) {
            V3<T> a = {T(A[k]), T(A[nseg + k]), T(A[2 * nseg + k])};
            V3<T> b = {T(B[k]), T(B[nseg + k]), T(B[2 * nseg + k])};
            V3<T> r1 = sub(P, a), r2 = sub(P, b), r0 = sub(b, a);
            T L0 = dsqrt(dot(r0, r0)), L1 = dsqrt(dot(r1, r1)), L2 = dsqrt(dot(r2, r2));
            double eps = 1e-12 * std::fmax(val(L0), 1.0);
            if (val(L0) < eps || val(L1) < eps || val(L2) < eps) continue;
            V3<T> c = cross(r1, r2);
            T c2 = dot(c, c);
            T L02 = L0 * L0;
            T d2 = c2 / L02;
            T den;
            if (rc == 0.0) den = c2;
            else if (vn == 1) den = L02 * (d2 + T(rc * rc));
            else den = L02 * dpow(dpow(d2, double(vn)) + T(std::pow(rc * rc, double(vn))), 1.0 / vn);
            if (val(den) == 0.0) continue;
            V3<T> e = {r1.x / L1 - r2.x / L2, r1.y / L1 - r2.y / L2, r1.z / L1 - r2.z / L2};
            T f = T(gam[k] / (4.0 * kPi)) * dot(r0, e) / den;
            au[0].add(f * c.x);
            au[1].add(f * c.y);
            au[2].add(f * c.z);
        }
        for (int c = 0; c < 3; ++c) u[c * nt + t] = au[c].get();
    }
}

// ---------------------------------------------------------------- segments acting on particles
// A fixed lattice of straight segments (blade rings or frozen wake lines) adds its velocity
// and its share of the stretching to the particles' right-hand side (Sec. II.B: the
// particles move with, and are stretched by, the total velocity).
struct Lattice {
    int64_t nseg = 0;
    const double* A = nullptr;
    const double* B = nullptr;
    const double* gam = nullptr;
    double rc = 0.0;
    int vn = 2;
};

// J[(3a+b) nt + t] = d u_a / d x_b of the segments at nt points, by forward mode.
void segment_jacobian(const Lattice& L, int64_t nt, const double* xt, double* J) {
    std::vector<Dual> X(3 * size_t(nt)), U(3 * size_t(nt));
    for (int b = 0; b < 3; ++b) {
        for (int c = 0; c < 3; ++c)
            for (int64_t t = 0; t < nt; ++t) X[c * nt + t] = Dual(xt[c * nt + t], c == b ? 1.0 : 0.0);
        eval_segments<Dual>(L.nseg, L.A, L.B, L.gam, L.rc, L.vn, nt, X.data(), U.data());
        for (int a = 0; a < 3; ++a)
            for (int64_t t = 0; t < nt; ++t) J[(3 * a + b) * nt + t] = U[a * nt + t].d;
    }
}

// J as above and M[(3a+b) nt + t] = d/dx_b (w_t . grad) u_a, the derivative of J's column
// sum along w_t (hyper-dual: direction a = e_b, direction b = w_t).
void segment_jacobian_and_hessian(const Lattice& L, int64_t nt, const double* xt, const double* w, double* J,
                                  double* M) {
    std::vector<HDual> X(3 * size_t(nt)), U(3 * size_t(nt));
    for (int b = 0; b < 3; ++b) {
        for (int c = 0; c < 3; ++c)
            for (int64_t t = 0; t < nt; ++t)
                X[c * nt + t] = HDual(xt[c * nt + t], c == b ? 1.0 : 0.0, w[c * nt + t], 0.0);
        eval_segments<HDual>(L.nseg, L.A, L.B, L.gam, L.rc, L.vn, nt, X.data(), U.data());
        for (int a = 0; a < 3; ++a)
            for (int64_t t = 0; t < nt; ++t) {
                J[(3 * a + b) * nt + t] = U[a * nt + t].a;
                M[(3 * a + b) * nt + t] = U[a * nt + t].ab;
            }
    }
}

// fx += u_seg(x), fg += J^T G (scheme 0, transposed) or J G (scheme 1, classical).
void add_segment_rhs(const Lattice& L, int64_t n, const double* x, const double* G, int scheme, double* fx,
                     double* fg) {
    std::vector<double> u(3 * n), J(9 * n);
    eval_segments<double>(L.nseg, L.A, L.B, L.gam, L.rc, L.vn, n, x, u.data());
    segment_jacobian(L, n, x, J.data());
    for (int64_t t = 0; t < n; ++t)
        for (int c = 0; c < 3; ++c) {
            fx[c * n + t] += u[c * n + t];
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                s += (scheme == 0 ? J[(3 * a + c) * n + t] : J[(3 * c + a) * n + t]) * G[a * n + t];
            fg[c * n + t] += s;
        }
}

// Tangent form: x and G carry tangents; the tangent of J along x's tangent comes from the
// hyper-dual pass (M with w = x.d).
void add_segment_rhs(const Lattice& L, int64_t n, const Dual* x, const Dual* G, int scheme, Dual* fx, Dual* fg) {
    std::vector<Dual> u(3 * n);
    eval_segments<Dual>(L.nseg, L.A, L.B, L.gam, L.rc, L.vn, n, x, u.data());
    std::vector<double> xv(3 * n), xd(3 * n), J(9 * n), Jd(9 * n);
    for (int64_t i = 0; i < 3 * n; ++i) { xv[i] = x[i].v; xd[i] = x[i].d; }
    segment_jacobian_and_hessian(L, n, xv.data(), xd.data(), J.data(), Jd.data());
    for (int64_t t = 0; t < n; ++t)
        for (int c = 0; c < 3; ++c) {
            fx[c * n + t] += u[c * n + t];
            Dual s;
            for (int a = 0; a < 3; ++a) {
                const int64_t k = (scheme == 0 ? (3 * a + c) : (3 * c + a)) * n + t;
                s += Dual(J[k], Jd[k]) * G[a * n + t];
            }
            fg[c * n + t] += s;
        }
}

// ---------------------------------------------------------------- RK3 program
// Williamson's low-storage third-order scheme, 2N-storage form:
//   Q <- a_k Q + dt F(Y);  Y <- Y + b_k Q,   k = 1..3,
// a = (0, -5/9, -153/128), b = (1/3, 15/16, 8/15), Y = (x, Gamma), F = (u, dGamma/dt).
const double kRkA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double kRkB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

// Storage model of the program (how the GPU programs in FP32 store their numbers):
//   0  every quantity in FP64 (the exact program);
//   1  each evaluation reads the state rounded to FP32 and its results are rounded to FP32
//      (an FP32 result that a second contribution is added to is rounded again), the state
//      and the registers stay FP64;
//   2  as 1, and the registers and the state are rounded to FP32 after every update.
// Rounding acts on values only: a tangent passes through it unchanged (the derivative of the
// program in which rounding is the identity).
inline double r32(double v) { return double(float(v)); }
inline Dual r32(Dual v) { return Dual(double(float(v.v)), v.d); }

template <class T>
void rk3_program(int64_t n, T* x, T* G, const double* sig, int nsteps, double dt, int scheme,
                 int sigma_rule, int64_t m, const double* y, T* uc, T* loss, const Lattice& lat,
                 int storage) {
    std::vector<T> qx(3 * n), qg(3 * n), fx(3 * n), fg(3 * n), xe(3 * n), ge(3 * n);
    std::vector<int64_t> excl(n);
    for (int64_t i = 0; i < n; ++i) excl[i] = i;
    auto round_all = [](std::vector<T>& v) { for (T& e : v) e = r32(e); };
    // the evaluation input: the state itself, or its FP32 copy
    auto eval_input = [&]() {
        for (int64_t i = 0; i < 3 * n; ++i) {
            xe[i] = storage ? r32(x[i]) : x[i];
            ge[i] = storage ? r32(G[i]) : G[i];
        }
    };
    for (int step = 0; step < nsteps; ++step) {
        for (int64_t i = 0; i < 3 * n; ++i) { qx[i] = T(0.0); qg[i] = T(0.0); }
        for (int k = 0; k < 3; ++k) {
            eval_input();
            eval_pairs<T>(n, xe.data(), ge.data(), sig, n, xe.data(), ge.data(), sig, excl.data(), scheme,
                          sigma_rule, fx.data(), fg.data());
            if (storage) { round_all(fx); round_all(fg); }
            if (lat.nseg > 0) {
                add_segment_rhs(lat, n, xe.data(), ge.data(), scheme, fx.data(), fg.data());
                if (storage) { round_all(fx); round_all(fg); }
            }
            for (int64_t i = 0; i < 3 * n; ++i) {
                qx[i] = T(kRkA[k]) * qx[i] + T(dt) * fx[i];
                qg[i] = T(kRkA[k]) * qg[i] + T(dt) * fg[i];
                if (storage == 2) { qx[i] = r32(qx[i]); qg[i] = r32(qg[i]); }
                x[i] = x[i] + T(kRkB[k]) * qx[i];
                G[i] = G[i] + T(kRkB[k]) * qg[i];
                if (storage == 2) { x[i] = r32(x[i]); G[i] = r32(G[i]); }
            }
        }
    }
    if (m > 0) {
        eval_input();
        std::vector<T> yt(3 * m);
        for (int64_t i = 0; i < 3 * m; ++i) yt[i] = T(y[i]);
        eval_pairs<T>(n, xe.data(), ge.data(), sig, m, yt.data(), nullptr, nullptr, nullptr, 0, 0, uc, nullptr);
        if (storage)
            for (int64_t i = 0; i < 3 * m; ++i) uc[i] = r32(uc[i]);
        if (lat.nseg > 0) {
            std::vector<T> us(3 * m);
            eval_segments<T>(lat.nseg, lat.A, lat.B, lat.gam, lat.rc, lat.vn, m, yt.data(), us.data());
            for (int64_t i = 0; i < 3 * m; ++i) uc[i] = storage ? r32(uc[i] + us[i]) : uc[i] + us[i];
        }
        Acc<T> l;
        for (int64_t c = 0; c < m; ++c) l.add(uc[2 * m + c] * uc[2 * m + c]);
        *loss = l.get();
    } else {
        *loss = T(0.0);
    }
}

// ---------------------------------------------------------------- velocity gradient
// Levi-Civita symbol eps_{abc}.
inline double levi(int a, int b, int c) {
    if (a == b || b == c || a == c) return 0.0;
    return ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1)) ? 1.0
                                                                                                        : -1.0;
}

// J[(3a+b) nt + t] = d u_a / d x_b at target t.  Differentiating g(s) eps_{acd} Gamma_c r_d
// with respect to x_b (r = x - x_j, ds/dx_b = r_b / s) gives
//     g eps_{acb} Gamma_c + (g'(s)/s) r_b eps_{acd} Gamma_c r_d.
void eval_gradient(int64_t ns, const double* xs, const double* gs, const double* sgs, int64_t nt,
                   const double* xt, const double* sgt, const int64_t* excl, int sigma_rule, double* J) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        V3<double> xi = load3(xt, nt, t);
        Neumaier acc[9];
        for (int64_t j = 0; j < ns; ++j) {
            if (excl && excl[t] == j) continue;
            V3<double> xj = load3(xs, ns, j);
            V3<double> Gj = load3(gs, ns, j);
            V3<double> r = sub(xi, xj);
            double s = std::sqrt(dot(r, r));
            double sig = sgs[j];
            if (sigma_rule == 1) sig = std::sqrt(0.5 * (sgt[t] * sgt[t] + sgs[j] * sgs[j]));
            double g, h;
            ghk<double>(s, sig, &g, &h, nullptr);
            const double G[3] = {Gj.x, Gj.y, Gj.z};
            const double R[3] = {r.x, r.y, r.z};
            V3<double> v = cross(Gj, r);
            const double Vv[3] = {v.x, v.y, v.z};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double rot = 0.0;
                    for (int c = 0; c < 3; ++c) rot += levi(a, c, b) * G[c];
                    acc[3 * a + b].add(g * rot + h * Vv[a] * R[b]);
                }
        }
        for (int k = 0; k < 9; ++k) J[k * nt + t] = acc[k].get();
    }
}

// ---------------------------------------------------------------- Vreman eddy viscosity
double vreman(const double* Jt, double delta, double cv) {
    // alpha_ab = d u_b / d x_a
    double al[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) al[a][b] = Jt[3 * b + a];
    double aa = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) aa += al[a][b] * al[a][b];
    if (aa == 0.0) return 0.0;
    double be[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double sum = 0.0;
            for (int m = 0; m < 3; ++m) sum += al[m][a] * al[m][b];
            be[a][b] = delta * delta * sum;
        }
    double B = be[0][0] * be[1][1] - be[0][1] * be[0][1] + be[0][0] * be[2][2] - be[0][2] * be[0][2] +
               be[1][1] * be[2][2] - be[1][2] * be[1][2];
    if (B < 0.0) B = 0.0;  // B_beta >= 0 in exact arithmetic (principal minors of a Gram matrix)
    return cv * std::sqrt(B / aa);
}

// ---------------------------------------------------------------- PSE diffusion
// zeta_sigma(s) = (2 pi sigma^2)^(-3/2) exp(-s^2 / (2 sigma^2))  (Eq. 3)
double zeta(double s, double sigma) {
    const double s2 = sigma * sigma;
    return std::exp(-0.5 * s * s / s2) / std::pow(2.0 * kPi * s2, 1.5);
}

// Targets: tgt[k] for k < nt (tgt == nullptr: every particle, nt == n); result row k of dg [3][nt].
void eval_pse(int64_t n, const double* x, const double* G, const double* sg, const double* vol,
              const double* nut, double nu, int64_t nt, const int64_t* tgt, double* dg) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt ? tgt[k] : k;
        V3<double> xi = load3(x, n, i);
        V3<double> Gi = load3(G, n, i);
        Neumaier acc[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            V3<double> xj = load3(x, n, j);
            V3<double> Gj = load3(G, n, j);
            V3<double> r = sub(xi, xj);
            const double s = std::sqrt(dot(r, r));
            const double sig2 = 0.5 * (sg[i] * sg[i] + sg[j] * sg[j]);
            const double nij = nu + (nut ? 0.5 * (nut[i] + nut[j]) : 0.0);
            const double w = 2.0 * nij / sig2 * zeta(s, std::sqrt(sig2));
            acc[0].add(w * (vol[i] * Gj.x - vol[j] * Gi.x));
            acc[1].add(w * (vol[i] * Gj.y - vol[j] * Gi.y));
            acc[2].add(w * (vol[i] * Gj.z - vol[j] * Gi.z));
        }
        for (int c = 0; c < 3; ++c) dg[c * nt + k] = acc[c].get();
    }
}

template <class T> void set_threads(int nth) {
    if (nth > 0) omp_set_num_threads(nth);
}

// ---------------------------------------------------------------- Cartesian FMM
// The far field of the particle sum with the singular kernel (the Gaussian differs from it
// by less than 2e-9 beyond 7 core radii), as the Laplace vector potential
//   psi(y) = sum_j Gamma_j G(y - x_j),  G(r) = 1/(4 pi |r|),  u = curl psi,
//   J_ae = d u_a / d y_e = eps_abc d_e d_b psi_c,
// expanded in Cartesian Taylor series of total order p (Sec. II.B names a Cartesian FMM):
//   multipole  M_k = sum_j Gamma_j (x_j - c)^k / k!                          (P2M)
//   shift      M_k(c') = sum_{m <= k} M_m(c) (c - c')^(k-m) / (k-m)!           (M2M)
//   local      L_n = sum_{|k| <= p-|n|} (-1)^|k| D_{n+k}(c_t - c_s) M_k        (M2L)
//              with D_m = d^m G, so psi(y) ~ sum_n L_n (y - c_t)^n / n!
//   shift      L_n(c') = sum_{m >= n, |m| <= p} L_m(c) (c' - c)^(m-n) / (m-n)! (L2L)
//   evaluate   d_b psi = sum_n L_{n+e_b} a^n / n!, d_e d_b psi likewise        (L2P)
// on a uniform octree of depth `level` over the particles' bounding cube: the leaves'
// 27-neighbourhoods are summed directly with the exact Gaussian kernel (P2P, self pair
// excluded), and at each level from 2 down every cell takes M2L from the children of its
// parent's neighbours that are not its own neighbours.  Derivatives of 1/|R| come from the
// Taylor expansion of 1/|R + h| in h, built by composing polynomials:
//   1/|R + h| = |R|^-1 (1 + w)^(-1/2),  w = (2 R.h + |h|^2)/|R|^2,
//   (1 + w)^(-1/2) = sum_m binom(-1/2, m) w^m,
// whose coefficient of h^n is D_n / n! of 1/|R|.

// Multi-indices with |n| <= P: by total degree, then decreasing n_x, then decreasing n_y.
struct Terms {
    int P = 0;
    std::vector<std::array<int, 3>> idx;
    std::vector<int> pos;  // (a (P+1) + b)(P+1) + c -> position, -1 beyond P
    explicit Terms(int P_) : P(P_), pos(size_t(P_ + 1) * (P_ + 1) * (P_ + 1), -1) {
        for (int d = 0; d <= P; ++d)
            for (int a = d; a >= 0; --a)
                for (int b = d - a; b >= 0; --b) {
                    const int c = d - a - b;
                    pos[(size_t(a) * (P + 1) + b) * (P + 1) + c] = int(idx.size());
                    idx.push_back({a, b, c});
                }
    }
    int at(int a, int b, int c) const {
        if (a < 0 || b < 0 || c < 0 || a + b + c > P) return -1;
        return pos[(size_t(a) * (P + 1) + b) * (P + 1) + c];
    }
    int size() const { return int(idx.size()); }
};

inline double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// Product of two polynomials in h (coefficients by Terms), truncated at total degree P.
std::vector<double> poly_mul(const std::vector<double>& a, const std::vector<double>& b, const Terms& T) {
    std::vector<double> out(T.size(), 0.0);
    std::vector<int> nzb;
    for (int j = 0; j < T.size(); ++j)
        if (b[j] != 0.0) nzb.push_back(j);
    for (int i = 0; i < T.size(); ++i) {
        if (a[i] == 0.0) continue;
        const auto& ni = T.idx[i];
        for (int j : nzb) {
            const auto& nj = T.idx[j];
            const int k = T.at(ni[0] + nj[0], ni[1] + nj[1], ni[2] + nj[2]);
            if (k >= 0) out[k] += a[i] * b[j];
        }
    }
    return out;
}

// Taylor coefficients of 1/|R + h| up to total degree Q (T.P == Q): D_n(R)/n! of 1/|R|.
std::vector<double> inv_r_taylor(const double R[3], const Terms& T) {
    const int Q = T.P;
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    std::vector<double> w(T.size(), 0.0), acc(T.size(), 0.0), wp(T.size(), 0.0);
    for (int a = 0; a < 3; ++a) {
        int e[3] = {0, 0, 0};
        e[a] = 1;
        if (Q >= 1) w[T.at(e[0], e[1], e[2])] = 2.0 * R[a] / r2;
        e[a] = 2;
        if (Q >= 2) w[T.at(e[0], e[1], e[2])] = 1.0 / r2;
    }
    acc[0] = 1.0;
    wp[0] = 1.0;
    double binom = 1.0;
    for (int m = 1; m <= Q; ++m) {
        wp = poly_mul(wp, w, T);
        binom *= (-0.5 - (m - 1)) / m;
        for (int i = 0; i < T.size(); ++i) acc[i] += binom * wp[i];
    }
    const double ir = 1.0 / std::sqrt(r2);
    for (double& v : acc) v *= ir;
    return acc;
}

struct FmmCell {
    int64_t key;            // (ix << 40) | (iy << 20) | iz at its level
    double c[3];            // centre
    std::vector<double> M;  // 3 x terms (component-major)
    std::vector<double> L;
};

inline int64_t cell_key(int64_t ix, int64_t iy, int64_t iz) { return (ix << 40) | (iy << 20) | iz; }
inline void key_coords(int64_t k, int64_t* i) { i[0] = k >> 40; i[1] = (k >> 20) & 0xFFFFF; i[2] = k & 0xFFFFF; }

void fmm_eval(int64_t n, const double* x, const double* G, const double* sig, int level, int p, int scheme,
              double* u, double* dg, double* Jout) {
    const Terms T(p);
    const int nt = T.size();
    // root cube: bounding box centre, half of the largest extent
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = hi[d] = n > 0 ? x[d * n] : 0.0;
        for (int64_t i = 1; i < n; ++i) {
            lo[d] = std::fmin(lo[d], x[d * n + i]);
            hi[d] = std::fmax(hi[d], x[d * n + i]);
        }
    }
    double H = 0.0, c0[3];
    for (int d = 0; d < 3; ++d) {
        c0[d] = 0.5 * (lo[d] + hi[d]);
        H = std::fmax(H, 0.5 * (hi[d] - lo[d]));
    }
    if (!(H > 0.0)) H = 1.0;
    double corner[3];
    for (int d = 0; d < 3; ++d) corner[d] = c0[d] - H;
    auto width = [&](int l) { return std::ldexp(2.0 * H, -l); };
    const int64_t side = int64_t(1) << level;
    // leaves
    std::vector<int64_t> leaf_of(n);
    std::map<int64_t, std::vector<int64_t>> leaves;
    const double wL = width(level);
    for (int64_t i = 0; i < n; ++i) {
        int64_t ic[3];
        for (int d = 0; d < 3; ++d) {
            int64_t v = int64_t(std::floor((x[d * n + i] - corner[d]) / wL));
            ic[d] = v < 0 ? 0 : (v >= side ? side - 1 : v);
        }
        leaf_of[i] = cell_key(ic[0], ic[1], ic[2]);
        leaves[leaf_of[i]].push_back(i);
    }
    // cells of every level
    std::vector<std::map<int64_t, FmmCell>> lev(level + 1);
    for (const auto& kv : leaves) {
        int64_t ic[3];
        key_coords(kv.first, ic);
        for (int l = level; l >= 0; --l) {
            const int sh = level - l;
            const int64_t k = cell_key(ic[0] >> sh, ic[1] >> sh, ic[2] >> sh);
            if (lev[l].count(k)) continue;
            FmmCell C;
            C.key = k;
            for (int d = 0; d < 3; ++d) C.c[d] = corner[d] + (double((&ic[0])[d] >> sh) + 0.5) * width(l);
            C.M.assign(3 * nt, 0.0);
            C.L.assign(3 * nt, 0.0);
            lev[l][k] = C;
        }
    }
    // P2M
    for (auto& kv : lev[level]) {
        FmmCell& C = kv.second;
        for (int64_t i : leaves[kv.first]) {
            const double a[3] = {x[i] - C.c[0], x[n + i] - C.c[1], x[2 * n + i] - C.c[2]};
            for (int t = 0; t < nt; ++t) {
                const auto& k = T.idx[t];
                const double mono = std::pow(a[0], k[0]) * std::pow(a[1], k[1]) * std::pow(a[2], k[2]) /
                                    (factorial(k[0]) * factorial(k[1]) * factorial(k[2]));
                for (int d = 0; d < 3; ++d) C.M[d * nt + t] += G[d * n + i] * mono;
            }
        }
    }
    // M2M
    for (int l = level - 1; l >= 0; --l) {
        for (auto& kv : lev[l + 1]) {
            const FmmCell& Ch = kv.second;
            int64_t ic[3];
            key_coords(Ch.key, ic);
            FmmCell& Pa = lev[l][cell_key(ic[0] >> 1, ic[1] >> 1, ic[2] >> 1)];
            const double dlt[3] = {Ch.c[0] - Pa.c[0], Ch.c[1] - Pa.c[1], Ch.c[2] - Pa.c[2]};
            for (int t = 0; t < nt; ++t) {
                const auto& k = T.idx[t];
                for (int s = 0; s < nt; ++s) {
                    const auto& m = T.idx[s];
                    if (m[0] > k[0] || m[1] > k[1] || m[2] > k[2]) continue;
                    const int q[3] = {k[0] - m[0], k[1] - m[1], k[2] - m[2]};
                    const double f = std::pow(dlt[0], q[0]) * std::pow(dlt[1], q[1]) * std::pow(dlt[2], q[2]) /
                                     (factorial(q[0]) * factorial(q[1]) * factorial(q[2]));
                    for (int d = 0; d < 3; ++d) Pa.M[d * nt + t] += Ch.M[d * nt + s] * f;
                }
            }
        }
    }
    // M2L (levels 2 .. level)
    const Terms T2(2 * p);
    for (int l = 2; l <= level; ++l) {
        std::map<int64_t, std::vector<double>> dcache;  // offset -> D_m / 4 pi, |m| <= 2p
        std::vector<int64_t> keys;
        for (const auto& kv : lev[l]) keys.push_back(kv.first);
#pragma omp parallel for schedule(dynamic)
        for (size_t ci = 0; ci < keys.size(); ++ci) {
            FmmCell& C = lev[l].at(keys[ci]);
            int64_t ic[3];
            key_coords(C.key, ic);
            for (int64_t dx = -1; dx <= 1; ++dx)
                for (int64_t dy = -1; dy <= 1; ++dy)
                    for (int64_t dz = -1; dz <= 1; ++dz) {
                        const int64_t px = (ic[0] >> 1) + dx, py = (ic[1] >> 1) + dy, pz = (ic[2] >> 1) + dz;
                        const int64_t ps = int64_t(1) << (l - 1);
                        if (px < 0 || py < 0 || pz < 0 || px >= ps || py >= ps || pz >= ps) continue;
                        for (int ch = 0; ch < 8; ++ch) {
                            const int64_t sx = 2 * px + (ch >> 2), sy = 2 * py + ((ch >> 1) & 1),
                                          sz = 2 * pz + (ch & 1);
                            if (std::llabs(sx - ic[0]) <= 1 && std::llabs(sy - ic[1]) <= 1 &&
                                std::llabs(sz - ic[2]) <= 1)
                                continue;
                            auto it = lev[l].find(cell_key(sx, sy, sz));
                            if (it == lev[l].end()) continue;
                            const FmmCell& S = it->second;
                            const int64_t off = cell_key(sx - ic[0] + 8, sy - ic[1] + 8, sz - ic[2] + 8);
                            std::vector<double> D;
#pragma omp critical(fmm_dcache)
                            {
                                auto dit = dcache.find(off);
                                if (dit != dcache.end()) D = dit->second;
                            }
                            if (D.empty()) {
                                // offset of the centres, canonically (integer offset) x (cell width)
                                const double R[3] = {double(ic[0] - sx) * width(l), double(ic[1] - sy) * width(l),
                                                     double(ic[2] - sz) * width(l)};
                                D = inv_r_taylor(R, T2);
                                for (int t = 0; t < T2.size(); ++t) {
                                    const auto& m = T2.idx[t];
                                    D[t] *= factorial(m[0]) * factorial(m[1]) * factorial(m[2]) / (4.0 * kPi);
                                }
#pragma omp critical(fmm_dcache)
                                dcache[off] = D;
                            }
                            for (int tn = 0; tn < nt; ++tn) {
                                const auto& nn = T.idx[tn];
                                const int dn = nn[0] + nn[1] + nn[2];
                                for (int tk = 0; tk < nt; ++tk) {
                                    const auto& k = T.idx[tk];
                                    const int dk = k[0] + k[1] + k[2];
                                    if (dn + dk > p) continue;
                                    const double Dv = D[T2.at(nn[0] + k[0], nn[1] + k[1], nn[2] + k[2])];
                                    const double sgn = (dk & 1) ? -1.0 : 1.0;
                                    for (int d = 0; d < 3; ++d) C.L[d * nt + tn] += sgn * Dv * S.M[d * nt + tk];
                                }
                            }
                        }
                    }
        }
    }
    // L2L (parents at levels 2 .. level-1)
    for (int l = 2; l < level; ++l) {
        for (auto& kv : lev[l + 1]) {
            FmmCell& Ch = kv.second;
            int64_t ic[3];
            key_coords(Ch.key, ic);
            const FmmCell& Pa = lev[l].at(cell_key(ic[0] >> 1, ic[1] >> 1, ic[2] >> 1));
            const double dlt[3] = {Ch.c[0] - Pa.c[0], Ch.c[1] - Pa.c[1], Ch.c[2] - Pa.c[2]};
            for (int tn = 0; tn < nt; ++tn) {
                const auto& nn = T.idx[tn];
                for (int tm = 0; tm < nt; ++tm) {
                    const auto& m = T.idx[tm];
                    if (m[0] < nn[0] || m[1] < nn[1] || m[2] < nn[2]) continue;
                    const int q[3] = {m[0] - nn[0], m[1] - nn[1], m[2] - nn[2]};
                    const double f = std::pow(dlt[0], q[0]) * std::pow(dlt[1], q[1]) * std::pow(dlt[2], q[2]) /
                                     (factorial(q[0]) * factorial(q[1]) * factorial(q[2]));
                    for (int d = 0; d < 3; ++d) Ch.L[d * nt + tn] += Pa.L[d * nt + tm] * f;
                }
            }
        }
    }
    // L2P and P2P
    std::vector<int64_t> leaf_keys;
    for (const auto& kv : leaves) leaf_keys.push_back(kv.first);
    for (int64_t i = 0; i < 3 * n; ++i) u[i] = dg[i] = 0.0;
    if (Jout)
        for (int64_t i = 0; i < 9 * n; ++i) Jout[i] = 0.0;
#pragma omp parallel for schedule(dynamic)
    for (size_t li = 0; li < leaf_keys.size(); ++li) {
        const std::vector<int64_t>& tg = leaves.at(leaf_keys[li]);
        const FmmCell& C = lev[level].at(leaf_keys[li]);
        int64_t ic[3];
        key_coords(leaf_keys[li], ic);
        // near field: the 27 neighbouring leaves, exact kernel
        std::vector<int64_t> src;
        for (int64_t dx = -1; dx <= 1; ++dx)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dz = -1; dz <= 1; ++dz) {
                    auto it = leaves.find(cell_key(ic[0] + dx, ic[1] + dy, ic[2] + dz));
                    if (ic[0] + dx < 0 || ic[1] + dy < 0 || ic[2] + dz < 0 || it == leaves.end()) continue;
                    src.insert(src.end(), it->second.begin(), it->second.end());
                }
        for (int64_t i : tg) {
            const double xi[3] = {x[i], x[n + i], x[2 * n + i]};
            const double Gi[3] = {G[i], G[n + i], G[2 * n + i]};
            Neumaier au[3], ad[3], aj[9];
            for (int64_t j : src) {
                if (j == i) continue;
                const double r[3] = {xi[0] - x[j], xi[1] - x[n + j], xi[2] - x[2 * n + j]};
                const double Gj[3] = {G[j], G[n + j], G[2 * n + j]};
                const double s = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double g, h;
                ghk<double>(s, sig[j], &g, &h, nullptr);
                const double v[3] = {Gj[1] * r[2] - Gj[2] * r[1], Gj[2] * r[0] - Gj[0] * r[2],
                                     Gj[0] * r[1] - Gj[1] * r[0]};
                for (int a = 0; a < 3; ++a) au[a].add(g * v[a]);
                if (Jout)  // J += g [Gamma_j]x + h (Gamma_j x r) r^T
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            double gx = 0.0;
                            for (int c = 0; c < 3; ++c) gx += levi(a, c, b) * Gj[c];
                            aj[3 * a + b].add(g * gx + h * v[a] * r[b]);
                        }
                if (scheme == 0) {
                    const double cgg[3] = {Gi[1] * Gj[2] - Gi[2] * Gj[1], Gi[2] * Gj[0] - Gi[0] * Gj[2],
                                           Gi[0] * Gj[1] - Gi[1] * Gj[0]};
                    const double tau = Gi[0] * v[0] + Gi[1] * v[1] + Gi[2] * v[2];
                    for (int a = 0; a < 3; ++a) ad[a].add(g * cgg[a] + h * tau * r[a]);
                } else {
                    const double cgg[3] = {Gj[1] * Gi[2] - Gj[2] * Gi[1], Gj[2] * Gi[0] - Gj[0] * Gi[2],
                                           Gj[0] * Gi[1] - Gj[1] * Gi[0]};
                    const double rg = r[0] * Gi[0] + r[1] * Gi[1] + r[2] * Gi[2];
                    for (int a = 0; a < 3; ++a) ad[a].add(g * cgg[a] + h * rg * v[a]);
                }
            }
            // far field from the local expansion (levels >= 2 only)
            double gp[3][3] = {{0}}, hp[3][3][3] = {{{0}}};  // d_b psi_c, d_e d_b psi_c
            if (level >= 2) {
                const double a[3] = {xi[0] - C.c[0], xi[1] - C.c[1], xi[2] - C.c[2]};
                for (int tn = 0; tn < nt; ++tn) {
                    const auto& nn = T.idx[tn];
                    const double mono = std::pow(a[0], nn[0]) * std::pow(a[1], nn[1]) * std::pow(a[2], nn[2]) /
                                        (factorial(nn[0]) * factorial(nn[1]) * factorial(nn[2]));
                    for (int b = 0; b < 3; ++b) {
                        int e1[3] = {nn[0], nn[1], nn[2]};
                        e1[b] += 1;
                        const int t1 = T.at(e1[0], e1[1], e1[2]);
                        if (t1 < 0) continue;
                        for (int c = 0; c < 3; ++c) gp[b][c] += C.L[c * nt + t1] * mono;
                        for (int e = 0; e < 3; ++e) {
                            int e2[3] = {e1[0], e1[1], e1[2]};
                            e2[e] += 1;
                            const int t2 = T.at(e2[0], e2[1], e2[2]);
                            if (t2 < 0) continue;
                            for (int c = 0; c < 3; ++c) hp[e][b][c] += C.L[c * nt + t2] * mono;
                        }
                    }
                }
            }
            double uf[3] = {0, 0, 0}, J[3][3] = {{0}};
            for (int aa = 0; aa < 3; ++aa)
                for (int b = 0; b < 3; ++b)
                    for (int c = 0; c < 3; ++c) {
                        const double e = levi(aa, b, c);
                        if (e == 0.0) continue;
                        uf[aa] += e * gp[b][c];
                        for (int ee = 0; ee < 3; ++ee) J[aa][ee] += e * hp[ee][b][c];
                    }
            for (int a = 0; a < 3; ++a) {
                double sf = 0.0;
                for (int b = 0; b < 3; ++b) sf += (scheme == 0 ? J[b][a] : J[a][b]) * Gi[b];
                u[a * n + i] = au[a].get() + uf[a];
                dg[a * n + i] = ad[a].get() + sf;
                if (Jout)
                    for (int b = 0; b < 3; ++b) Jout[(3 * a + b) * n + i] = aj[3 * a + b].get() + J[a][b];
            }
        }
    }
}

}  // namespace

// ================================================================ C entry points
// All arrays are component-major [3][n] double.  Return 0 on success, nonzero on a bad
// argument.  nthreads <= 0 keeps the OpenMP default.
extern "C" {

int orc_weights(double rho, double* Gw, double* Hw, double* Kw) {
    if (!(rho >= 0.0)) return 1;
    weights<double>(rho, Gw, Hw, Kw);
    return 0;
}

int orc_ghk(double s, double sigma, double* g, double* h, double* k) {
    if (!(s >= 0.0) || !(sigma > 0.0)) return 1;
    ghk<double>(s, sigma, g, h, k);
    return 0;
}

int orc_eval(int64_t ns, const double* xs, const double* gs, const double* sgs, int64_t nt,
             const double* xt, const double* gt, const double* sgt, const int64_t* excl,
             int scheme, int sigma_rule, double* u, double* dg, int nthreads) {
    if (ns < 0 || nt < 0 || !xs || !gs || !sgs || !xt || !u) return 1;
    if (gt && !dg) return 1;
    if (sigma_rule == 1 && !sgt) return 1;
    if (scheme < 0 || scheme > 1 || sigma_rule < 0 || sigma_rule > 1) return 1;
    set_threads<double>(nthreads);
    eval_pairs<double>(ns, xs, gs, sgs, nt, xt, gt, sgt, excl, scheme, sigma_rule, u, dg);
    return 0;
}

// Tangent of orc_eval: (xs_d, gs_d) is the direction on the sources, (xt_d, gt_d) on
// the targets; with self evaluation pass the same direction for both.
int orc_eval_jvp(int64_t ns, const double* xs, const double* gs, const double* sgs,
                 const double* xs_d, const double* gs_d, int64_t nt, const double* xt,
                 const double* gt, const double* sgt, const double* xt_d, const double* gt_d,
                 const int64_t* excl, int scheme, int sigma_rule, double* u, double* dg,
                 double* u_d, double* dg_d, int nthreads) {
    if (ns < 0 || nt < 0 || !xs || !gs || !sgs || !xt || !u || !xs_d || !gs_d || !xt_d || !u_d)
        return 1;
    if (gt && (!dg || !gt_d || !dg_d)) return 1;
    if (sigma_rule == 1 && !sgt) return 1;
    set_threads<double>(nthreads);
    std::vector<Dual> Xs(3 * ns), Gs(3 * ns), Xt(3 * nt), Gt(gt ? 3 * nt : 0), U(3 * nt),
        D(gt ? 3 * nt : 0);
    for (int64_t i = 0; i < 3 * ns; ++i) { Xs[i] = Dual(xs[i], xs_d[i]); Gs[i] = Dual(gs[i], gs_d[i]); }
    for (int64_t i = 0; i < 3 * nt; ++i) {
        Xt[i] = Dual(xt[i], xt_d[i]);
        if (gt) Gt[i] = Dual(gt[i], gt_d[i]);
    }
    eval_pairs<Dual>(ns, Xs.data(), Gs.data(), sgs, nt, Xt.data(), gt ? Gt.data() : nullptr, sgt,
                     excl, scheme, sigma_rule, U.data(), gt ? D.data() : nullptr);
    for (int64_t i = 0; i < 3 * nt; ++i) {
        u[i] = U[i].v; u_d[i] = U[i].d;
        if (gt) { dg[i] = D[i].v; dg_d[i] = D[i].d; }
    }
    return 0;
}

int orc_segments(int64_t nseg, const double* A, const double* B, const double* gam, double rc,
                 int vn, int64_t nt, const double* xt, double* u, int nthreads) {
    if (nseg < 0 || nt < 0 || !xt || !u || (nseg > 0 && (!A || !B || !gam))) return 1;
    if (!(rc >= 0.0) || vn < 1) return 1;
    set_threads<double>(nthreads);
    eval_segments<double>(nseg, A, B, gam, rc, vn, nt, xt, u);
    return 0;
}

// Velocity gradient of the segments at the targets, J [9][nt] (J[(3a+b) nt + t] = du_a/dx_b),
// by forward-mode differentiation of the segment law along each coordinate of the targets.
int orc_segments_gradient(int64_t nseg, const double* A, const double* B, const double* gam, double rc, int vn,
                          int64_t nt, const double* xt, double* J, int nthreads) {
    if (nseg < 0 || nt < 0 || !xt || !J || (nseg > 0 && (!A || !B || !gam))) return 1;
    if (!(rc >= 0.0) || vn < 1) return 1;
    set_threads<double>(nthreads);
    std::vector<Dual> X(3 * size_t(nt)), U(3 * size_t(nt));
    for (int b = 0; b < 3; ++b) {
        for (int c = 0; c < 3; ++c)
            for (int64_t t = 0; t < nt; ++t) X[c * nt + t] = Dual(xt[c * nt + t], c == b ? 1.0 : 0.0);
        eval_segments<Dual>(nseg, A, B, gam, rc, vn, nt, X.data(), U.data());
        for (int a = 0; a < 3; ++a)
            for (int64_t t = 0; t < nt; ++t) J[(3 * a + b) * nt + t] = U[a * nt + t].d;
    }
    return 0;
}

// Vector-Jacobian product of the segments' velocity and stretching at particles (x, G)
// [3][nt] with seeds ubar, dbar [3][nt] (dbar may be null):
//   L = sum_t ubar_t . u(x_t) + dbar_t . s_t,  s = J^T G (scheme 0) or J G (scheme 1),
//   xbar = J^T ubar + sum_a w2_a M[a][.],  M = d/dx (w1 . grad) u,
//   (w1, w2) = (dbar, G) for scheme 0 and (G, dbar) for scheme 1,
//   Gbar = J dbar (scheme 0) or J^T dbar (scheme 1).
int orc_segments_vjp(int64_t nseg, const double* A, const double* B, const double* gam, double rc, int vn,
                     int64_t nt, const double* xt, const double* gt, const double* ubar, const double* dbar,
                     int scheme, double* xbar, double* gbar, int nthreads) {
    if (nseg < 0 || nt < 0 || !xt || !ubar || !xbar || (nseg > 0 && (!A || !B || !gam))) return 1;
    if (!(rc >= 0.0) || vn < 1 || scheme < 0 || scheme > 1) return 1;
    if (dbar && (!gt || !gbar)) return 1;
    set_threads<double>(nthreads);
    Lattice lat;
    lat.nseg = nseg; lat.A = A; lat.B = B; lat.gam = gam; lat.rc = rc; lat.vn = vn;
    std::vector<double> J(9 * nt), M(9 * nt, 0.0), zero(3 * nt, 0.0);
    const double* w1 = !dbar ? zero.data() : (scheme == 0 ? dbar : gt);
    const double* w2 = !dbar ? zero.data() : (scheme == 0 ? gt : dbar);
    segment_jacobian_and_hessian(lat, nt, xt, w1, J.data(), M.data());
    for (int64_t t = 0; t < nt; ++t)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                s += J[(3 * a + b) * nt + t] * ubar[a * nt + t] + w2[a * nt + t] * M[(3 * a + b) * nt + t];
            xbar[b * nt + t] = s;
            if (dbar) {
                double g = 0.0;
                for (int c = 0; c < 3; ++c)
                    g += (scheme == 0 ? J[(3 * b + c) * nt + t] : J[(3 * c + b) * nt + t]) * dbar[c * nt + t];
                gbar[b * nt + t] = g;
            }
        }
    return 0;
}

// Runs nsteps RK3 steps from (x, G) in place, then the control-point velocity uc [3][m]
// and the loss sum_c uc_z^2.
// Optional fixed lattice: nseg segments A -> B [3][nseg] of strength gs, core rc, exponent vn
// (nseg = 0: particles only).
int orc_rk3_program(int64_t n, double* x, double* G, const double* sig, int nsteps, double dt,
                    int scheme, int sigma_rule, int64_t m, const double* y, double* uc,
                    double* loss, int nthreads, int64_t nseg, const double* A, const double* B,
                    const double* gs, double rc, int vn, int storage) {
    if (n < 0 || m < 0 || nsteps < 0 || !x || !G || !sig || !loss || (m > 0 && (!y || !uc)))
        return 1;
    if (storage < 0 || storage > 2) return 1;
    if (nseg < 0 || (nseg > 0 && (!A || !B || !gs || !(rc >= 0.0) || vn < 1))) return 1;
    set_threads<double>(nthreads);
    Lattice lat;
    lat.nseg = nseg; lat.A = A; lat.B = B; lat.gam = gs; lat.rc = rc; lat.vn = vn;
    rk3_program<double>(n, x, G, sig, nsteps, dt, scheme, sigma_rule, m, y, uc, loss, lat, storage);
    return 0;
}

// Directional derivative of the program's loss along (xd, Gd) at (x, G); x and G are left
// unchanged.  Returns loss and dloss.
int orc_rk3_program_jvp(int64_t n, const double* x, const double* G, const double* sig,
                        const double* xd, const double* Gd, int nsteps, double dt, int scheme,
                        int sigma_rule, int64_t m, const double* y, double* loss,
                        double* dloss, int nthreads, int64_t nseg, const double* A, const double* B,
                        const double* gs, double rc, int vn, int storage) {
    if (n < 0 || m < 0 || nsteps < 0 || !x || !G || !sig || !xd || !Gd || !loss || !dloss)
        return 1;
    if (storage < 0 || storage > 2) return 1;
    if (m > 0 && !y) return 1;
    if (nseg < 0 || (nseg > 0 && (!A || !B || !gs || !(rc >= 0.0) || vn < 1))) return 1;
    set_threads<double>(nthreads);
    Lattice lat;
    lat.nseg = nseg; lat.A = A; lat.B = B; lat.gam = gs; lat.rc = rc; lat.vn = vn;
    std::vector<Dual> X(3 * n), Gm(3 * n), UC(3 * (m > 0 ? m : 1));
    for (int64_t i = 0; i < 3 * n; ++i) { X[i] = Dual(x[i], xd[i]); Gm[i] = Dual(G[i], Gd[i]); }
    Dual L;
    rk3_program<Dual>(n, X.data(), Gm.data(), sig, nsteps, dt, scheme, sigma_rule, m, y, UC.data(), &L, lat,
                      storage);
    *loss = L.v;
    *dloss = L.d;
    return 0;
}

// FP64 diagnostics of one evaluation (invariants of Eq. 1):
// out[0..2] = sum Gamma_i, out[3..5] = sum dGamma_i/dt, out[6..8] = impulse 1/2 sum x_i x Gamma_i,
// out[9..11] = its rate 1/2 sum (u_i x Gamma_i + x_i x dGamma_i/dt), out[12] = number of
// non-finite entries among x, Gamma, u, dGamma/dt.
// Velocity gradient J [9][nt] (row-major 3x3 per target: J[(3a+b) nt + t] = du_a/dx_b).
int orc_gradient(int64_t ns, const double* xs, const double* gs, const double* sgs, int64_t nt,
                 const double* xt, const double* sgt, const int64_t* excl, int sigma_rule, double* J,
                 int nthreads) {
    if (ns < 0 || nt < 0 || !xs || !gs || !sgs || !xt || !J) return 1;
    if (sigma_rule < 0 || sigma_rule > 1 || (sigma_rule == 1 && !sgt)) return 1;
    set_threads<double>(nthreads);
    eval_gradient(ns, xs, gs, sgs, nt, xt, sgt, excl, sigma_rule, J);
    return 0;
}

// Vreman eddy viscosity nu_t[n] from J [9][n] with filter width sigma[n].
int orc_vreman(int64_t n, const double* J, const double* sigma, double cv, double* nut) {
    if (n < 0 || !J || !sigma || !nut || !(cv >= 0.0)) return 1;
    for (int64_t i = 0; i < n; ++i) {
        double Jt[9];
        for (int k = 0; k < 9; ++k) Jt[k] = J[k * n + i];
        nut[i] = vreman(Jt, sigma[i], cv);
    }
    return 0;
}

// PSE diffusion dGamma/dt [3][n] of one particle set; nut may be NULL (no eddy viscosity).
int orc_pse(int64_t n, const double* x, const double* G, const double* sigma, const double* vol,
            const double* nut, double nu, double* dg, int nthreads) {
    if (n < 0 || !x || !G || !sigma || !vol || !dg || !(nu >= 0.0)) return 1;
    set_threads<double>(nthreads);
    eval_pse(n, x, G, sigma, vol, nut, nu, n, nullptr, dg);
    return 0;
}

// The same at the particles tgt[0..nt) only (each summed over all n particles); dg [3][nt].
int orc_pse_at(int64_t n, const double* x, const double* G, const double* sigma, const double* vol,
               const double* nut, double nu, int64_t nt, const int64_t* tgt, double* dg, int nthreads) {
    if (n < 0 || nt < 0 || !x || !G || !sigma || !vol || !dg || !tgt || !(nu >= 0.0)) return 1;
    for (int64_t k = 0; k < nt; ++k)
        if (tgt[k] < 0 || tgt[k] >= n) return 1;
    set_threads<double>(nthreads);
    eval_pse(n, x, G, sigma, vol, nut, nu, nt, tgt, dg);
    return 0;
}

int orc_diagnostics(int64_t n, const double* x, const double* G, const double* u, const double* dg,
                    double* out) {
    if (n < 0 || !x || !G || !u || !dg || !out) return 1;
    Neumaier acc[12];
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        V3<double> xi = load3(x, n, i), Gi = load3(G, n, i), ui = load3(u, n, i), di = load3(dg, n, i);
        V3<double> p = cross(xi, Gi);
        V3<double> a = cross(ui, Gi);
        V3<double> b = cross(xi, di);
        double vals[12] = {Gi.x, Gi.y, Gi.z, di.x, di.y, di.z, 0.5 * p.x, 0.5 * p.y, 0.5 * p.z,
                           0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z)};
        for (int c = 0; c < 12; ++c) acc[c].add(vals[c]);
        const double* all[4] = {x, G, u, dg};
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c)
                if (!std::isfinite(all[k][c * n + i])) ++bad;
    }
    for (int c = 0; c < 12; ++c) out[c] = acc[c].get();
    out[12] = double(bad);
    return 0;
}


// Cartesian FMM evaluation of the self-interaction of n particles (velocity and stretching,
// scheme 0 transposed / 1 classical; optionally the velocity gradient J [9][n], row 3a + b =
// du_a/dx_b) on a uniform octree of depth `level` (0..10) with expansions of order `order`
// (1..20).
int orc_fmm(int64_t n, const double* x, const double* G, const double* sig, int level, int order, int scheme,
            double* u, double* dg, double* J, int nthreads) {
    if (n < 0 || (n > 0 && (!x || !G || !sig || !u || !dg))) return 1;
    if (level < 0 || level > 10 || order < 1 || order > 20 || scheme < 0 || scheme > 1) return 1;
    set_threads<double>(nthreads);
    fmm_eval(n, x, G, sig, level, order, scheme, u, dg, J);
    return 0;
}

// Taylor coefficients of 1/|R + h| in h up to total degree Q, in the oracle's multi-index
// order (by degree, then decreasing n_x, then decreasing n_y); idx receives the multi-indices.
int orc_inv_r_taylor(const double* R, int Q, double* coef, int* idx) {
    if (!R || !coef || !idx || Q < 0 || Q > 40) return 1;
    const Terms T(Q);
    const std::vector<double> c = inv_r_taylor(R, T);
    for (int t = 0; t < T.size(); ++t) {
        coef[t] = c[t];
        for (int d = 0; d < 3; ++d) idx[3 * t + d] = T.idx[t][d];
    }
    return 0;
}
}  // extern "C"
