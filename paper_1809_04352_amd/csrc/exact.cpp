// Exact labels of single points (eq. 2) for the host arbitration of the
// classification.  Every comparison of the label is a polynomial in the input
// doubles -- centres, radii, probe radius and the point's coordinates -- up to
// square roots, which are removed by squaring under sign analysis.  Each sign
// is first taken from an FP64 evaluation with a rigorous running error bound
// (Ap below); only when the bound does not decide it is the same polynomial
// evaluated exactly in dyadic big-integer arithmetic (Dy below).
//
// The label (section 1: the SES bounds the union of probe balls that overlap
// no atom; eq. 2), with s_i = r_i + rho taken exactly:
//   1. |x - c_i|^2 <= r_i^2 for some atom               -> inside;
//   2. |x - c_i|^2 >= s_i^2 for every atom (x is in A)   -> outside;
//   3. otherwise outside iff an admissible candidate (a point of A) lies
//      strictly within rho: a concave probe position, the radial projection
//      onto an SAS sphere, or the nearest point of an SAS circle.
// The polynomial forms (all denominators are positive and cleared):
//   face i, neighbour k: admissible iff N sqrt(D) - L >= 0 with D = |x - c_i|^2,
//     N = s_i^2 + |c_k - c_i|^2 - s_k^2, L = 2 s_i (x - c_i).(c_k - c_i);
//   circle (i, j): v = c_j - c_i, Dv = |v|^2, A = s_i^2 - s_j^2 + Dv; with
//     W = 2 Dv (x - c_i) - A v (= 2 Dv (x - o)), R2s = 4 Dv s_i^2 - A^2
//     (= 4 Dv R^2) and B2s = Dv |W|^2 - (W.v)^2 (= 4 Dv^3 b^2), the nearest
//     circle point is within rho iff |W|^2 + Dv R2s - 4 Dv^2 rho^2 <
//     2 sqrt(R2s B2s); it is admissible against k iff
//     Nk sqrt(|Wp|^2) + 2 (Ok.Wp) sqrt(Dv R2s) >= 0 with
//     Ok = 2 Dv (c_i - c_k) + A v, Nk = |Ok|^2 + Dv R2s - 4 Dv^2 s_k^2 and
//     Wp = Dv W - (W.v) v (a positive multiple of the in-plane part of x - o;
//     on the axis, where every circle point is equally near, a fixed
//     direction perpendicular to v instead);
//   probe (i < j < k, side sigma): a = c_j - c_i, b = c_k - c_i, m = a x b,
//     M2 = |m|^2, Z = (s_i^2 - s_j^2 + |a|^2)(b x m) + (s_i^2 - s_k^2 + |b|^2)(m x a)
//     (= 2 M2 z, z the point of the radical line with m.z = 0), E =
//     2 M2 (x - c_i) - Z, Ts = 4 M2^2 s_i^2 - |Z|^2; then x is strictly within
//     rho of the probe iff (|E|^2 + Ts - 4 M2^2 rho^2) sqrt(M2) -
//     2 sigma (m.E) sqrt(Ts) < 0.
#include "exact.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace eses {

namespace {

// ----------------------------------------------------------------- Ap
// FP64 value with a bound on its rounding error: for an expression of +, -
// and * over exact doubles, |computed - exact| <= gamma_{d} * a, where a is
// the same expression over absolute values and d the depth of the operation
// tree (gamma_k = k u / (1 - k u)).  The sign is certain when |v| exceeds
// twice that bound (a itself is rounded, by less than gamma_d relative).
struct Ap {
    double v, a;
    int d;
};

inline Ap ap(double x) { return {x, std::fabs(x), 0}; }
inline Ap operator+(const Ap &x, const Ap &y) { return {x.v + y.v, x.a + y.a, std::max(x.d, y.d) + 1}; }
inline Ap operator-(const Ap &x, const Ap &y) { return {x.v - y.v, x.a + y.a, std::max(x.d, y.d) + 1}; }
inline Ap operator*(const Ap &x, const Ap &y) { return {x.v * y.v, x.a * y.a, x.d + y.d + 1}; }
inline Ap operator-(const Ap &x) { return {-x.v, x.a, x.d}; }

// Sign of x, or ok = false when the bound does not decide it (or the
// magnitudes leave the range where the bound holds).
inline int sign_of(const Ap &x, bool &ok) {
    const double u = 1.1102230246251565e-16;
    const double k = x.d + 2;
    const double gam = k * u / (1.0 - k * u);
    if (!(x.a < 1e290) || (x.a != 0.0 && x.a < 1e-280)) {
        ok = false;
        return 0;
    }
    const double bound = 2.0 * gam * x.a;
    if (x.v > bound) return 1;
    if (x.v < -bound) return -1;
    if (x.a == 0.0) return 0;  // an exact zero: every term was zero
    ok = false;
    return 0;
}

// ----------------------------------------------------------------- Dy
// Dyadic number sign * mag * 2^exp with an arbitrary-precision magnitude
// (32-bit limbs, least significant first; zero has no limbs).
struct Dy {
    int sign = 0;
    int64_t exp = 0;
    std::vector<uint32_t> mag;
};

void trim(std::vector<uint32_t> &m) {
    while (!m.empty() && m.back() == 0) m.pop_back();
}

Dy dy(double x) {
    Dy r;
    if (x == 0.0) return r;
    int e = 0;
    double f = std::frexp(std::fabs(x), &e);  // x = f 2^e, f in [0.5, 1)
    uint64_t m = (uint64_t)std::ldexp(f, 53);
    int64_t ex = (int64_t)e - 53;
    while ((m & 1u) == 0) {
        m >>= 1;
        ++ex;
    }
    r.sign = x < 0 ? -1 : 1;
    r.exp = ex;
    r.mag = {(uint32_t)m, (uint32_t)(m >> 32)};
    trim(r.mag);
    return r;
}

std::vector<uint32_t> shl(const std::vector<uint32_t> &m, int64_t bits) {
    if (m.empty() || bits == 0) return m;
    const int64_t limbs = bits / 32;
    const int b = (int)(bits % 32);
    std::vector<uint32_t> r((size_t)limbs, 0u);
    r.reserve(m.size() + (size_t)limbs + 1);
    uint32_t carry = 0;
    for (uint32_t w : m) {
        r.push_back(b ? (w << b) | carry : w);
        carry = b ? w >> (32 - b) : 0;
    }
    if (carry) r.push_back(carry);
    return r;
}

int cmp_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t q = a.size(); q-- > 0;)
        if (a[q] != b[q]) return a[q] < b[q] ? -1 : 1;
    return 0;
}

std::vector<uint32_t> add_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    const std::vector<uint32_t> &x = a.size() >= b.size() ? a : b;
    const std::vector<uint32_t> &y = a.size() >= b.size() ? b : a;
    std::vector<uint32_t> r(x.size() + 1, 0u);
    uint64_t c = 0;
    for (size_t q = 0; q < x.size(); ++q) {
        c += (uint64_t)x[q] + (q < y.size() ? y[q] : 0u);
        r[q] = (uint32_t)c;
        c >>= 32;
    }
    r[x.size()] = (uint32_t)c;
    trim(r);
    return r;
}

// a - b for |a| >= |b|.
std::vector<uint32_t> sub_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    std::vector<uint32_t> r(a.size(), 0u);
    int64_t br = 0;
    for (size_t q = 0; q < a.size(); ++q) {
        int64_t t = (int64_t)a[q] - (q < b.size() ? b[q] : 0u) - br;
        br = t < 0 ? 1 : 0;
        r[q] = (uint32_t)(t + (br << 32));
    }
    trim(r);
    return r;
}

Dy operator*(const Dy &x, const Dy &y) {
    Dy r;
    if (!x.sign || !y.sign) return r;
    r.sign = x.sign * y.sign;
    r.exp = x.exp + y.exp;
    r.mag.assign(x.mag.size() + y.mag.size(), 0u);
    for (size_t i = 0; i < x.mag.size(); ++i) {
        uint64_t c = 0;
        for (size_t j = 0; j < y.mag.size(); ++j) {
            uint64_t t = (uint64_t)x.mag[i] * y.mag[j] + r.mag[i + j] + c;
            r.mag[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        size_t k = i + y.mag.size();
        while (c) {
            uint64_t t = (uint64_t)r.mag[k] + c;
            r.mag[k] = (uint32_t)t;
            c = t >> 32;
            ++k;
        }
    }
    trim(r.mag);
    return r;
}

Dy operator+(const Dy &x, const Dy &y) {
    if (!x.sign) return y;
    if (!y.sign) return x;
    const int64_t e = std::min(x.exp, y.exp);
    std::vector<uint32_t> a = shl(x.mag, x.exp - e), b = shl(y.mag, y.exp - e);
    Dy r;
    r.exp = e;
    if (x.sign == y.sign) {
        r.sign = x.sign;
        r.mag = add_mag(a, b);
    } else {
        const int c = cmp_mag(a, b);
        if (c == 0) return Dy();
        r.sign = c > 0 ? x.sign : y.sign;
        r.mag = c > 0 ? sub_mag(a, b) : sub_mag(b, a);
    }
    return r;
}

Dy operator-(const Dy &x) {
    Dy r = x;
    r.sign = -r.sign;
    return r;
}

Dy operator-(const Dy &x, const Dy &y) { return x + (-y); }

inline int sign_of(const Dy &x, bool &) { return x.sign; }

// ---------------------------------------------------------- vectors
template <class T>
struct V3 {
    T x, y, z;
};

template <class T>
T num(double v);
template <>
Ap num<Ap>(double v) { return ap(v); }
template <>
Dy num<Dy>(double v) { return dy(v); }

template <class T>
V3<T> vec(const double *p) {
    return {num<T>(p[0]), num<T>(p[1]), num<T>(p[2])};
}
template <class T>
V3<T> operator-(const V3<T> &a, const V3<T> &b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T>
V3<T> operator+(const V3<T> &a, const V3<T> &b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T>
V3<T> operator*(const T &s, const V3<T> &a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T>
T dot(const V3<T> &a, const V3<T> &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
V3<T> cross(const V3<T> &a, const V3<T> &b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Sign of a sqrt(X) + b sqrt(Y) for X, Y >= 0.
template <class T>
int sqrt2_sign(const T &a, const T &X, const T &b, const T &Y, bool &ok) {
    const int sX = sign_of(X, ok), sY = sign_of(Y, ok);
    const int sa = sX > 0 ? sign_of(a, ok) : 0;
    const int sb = sY > 0 ? sign_of(b, ok) : 0;
    if (!ok) return 0;
    if (sa == 0) return sb;
    if (sb == 0) return sa;
    if (sa == sb) return sa;
    const int d = sign_of(a * a * X - b * b * Y, ok);
    return sa * d;
}

// ------------------------------------------------------ predicates
// Each returns a sign (or a boolean) and clears ok when an FP64 evaluation
// cannot certify it.

// sign(|x - c|^2 - q^2) with q = r + k rho (k = 0, 1, 2).
template <class T>
int ball_sign(const double *x, const double *c, double r, double rho, int k, bool &ok) {
    V3<T> e = vec<T>(x) - vec<T>(c);
    T q = num<T>(r);
    for (int t = 0; t < k; ++t) q = q + num<T>(rho);
    return sign_of(dot(e, e) - q * q, ok);
}

// Face of atom i admissible against neighbour k (see the header comment).
template <class T>
int face_cut_sign(const double *x, const double *ci, double ri, const double *ck, double rk,
                  double rho, bool &ok) {
    V3<T> e = vec<T>(x) - vec<T>(ci);
    V3<T> v = vec<T>(ck) - vec<T>(ci);
    T si = num<T>(ri) + num<T>(rho), sk = num<T>(rk) + num<T>(rho);
    T D = dot(e, e);
    T N = si * si + dot(v, v) - sk * sk;
    T L = num<T>(2.0) * si * dot(e, v);
    T one = num<T>(1.0);
    return sqrt2_sign(N, D, -L, one, ok);
}

template <class T>
struct Circle {
    V3<T> v, ci;
    T Dv, A, R2s;
};

template <class T>
Circle<T> circle(const double *ci, double ri, const double *cj, double rj, double rho) {
    Circle<T> c;
    c.ci = vec<T>(ci);
    c.v = vec<T>(cj) - c.ci;
    T si = num<T>(ri) + num<T>(rho), sj = num<T>(rj) + num<T>(rho);
    c.Dv = dot(c.v, c.v);
    c.A = si * si - sj * sj + c.Dv;
    c.R2s = num<T>(4.0) * c.Dv * si * si - c.A * c.A;
    return c;
}

// The SAS spheres of i and j meet in a circle: (s_i - s_j)^2 < Dv < (s_i + s_j)^2.
template <class T>
bool circle_exists(const double *ci, double ri, const double *cj, double rj, double rho,
                   bool &ok) {
    V3<T> v = vec<T>(cj) - vec<T>(ci);
    T Dv = dot(v, v);
    T si = num<T>(ri) + num<T>(rho), sj = num<T>(rj) + num<T>(rho);
    T dm = si - sj, dp = si + sj;
    const int a = sign_of(Dv - dm * dm, ok);
    const int b = sign_of(dp * dp - Dv, ok);
    return a > 0 && b > 0;
}

// The nearest circle point within rho of x (strictly).
template <class T>
bool circle_within(const Circle<T> &c, const double *x, double rho, bool &ok) {
    V3<T> W = (num<T>(2.0) * c.Dv) * (vec<T>(x) - c.ci) - c.A * c.v;
    T Wv = dot(W, c.v);
    T B2s = c.Dv * dot(W, W) - Wv * Wv;
    T r = num<T>(rho);
    T P = dot(W, W) + c.Dv * c.R2s - num<T>(4.0) * c.Dv * c.Dv * r * r;
    T one = num<T>(1.0);
    // 2 sqrt(R2s B2s) - P > 0
    return sqrt2_sign(num<T>(2.0), c.R2s * B2s, -P, one, ok) > 0;
}

// Admissibility of the nearest circle point against atom k; axis: 0-2 picks
// the fixed perpendicular direction used on the circle's axis, -1 the
// direction of x.
template <class T>
int circle_cut_sign(const Circle<T> &c, const double *x, int axis, const double *ck, double rk,
                    double rho, bool &ok) {
    V3<T> Wp;
    if (axis < 0) {
        V3<T> W = (num<T>(2.0) * c.Dv) * (vec<T>(x) - c.ci) - c.A * c.v;
        Wp = c.Dv * W - dot(W, c.v) * c.v;
    } else {
        double e[3] = {0.0, 0.0, 0.0};
        e[axis] = 1.0;
        V3<T> E = vec<T>(e);
        Wp = c.Dv * E - dot(E, c.v) * c.v;
    }
    V3<T> Ok = (num<T>(2.0) * c.Dv) * (c.ci - vec<T>(ck)) + c.A * c.v;
    T sk = num<T>(rk) + num<T>(rho);
    T Nk = dot(Ok, Ok) + c.Dv * c.R2s - num<T>(4.0) * c.Dv * c.Dv * sk * sk;
    return sqrt2_sign(Nk, dot(Wp, Wp), num<T>(2.0) * dot(Ok, Wp), c.Dv * c.R2s, ok);
}

// The circle's in-plane offset of x vanishes (x on the axis).
template <class T>
bool on_axis(const Circle<T> &c, const double *x, bool &ok) {
    V3<T> W = (num<T>(2.0) * c.Dv) * (vec<T>(x) - c.ci) - c.A * c.v;
    T Wv = dot(W, c.v);
    return sign_of(c.Dv * dot(W, W) - Wv * Wv, ok) == 0;
}

// x strictly within rho of the probe position (i, j, k, sigma).
template <class T>
bool probe_within_t(const double *x, const double *ci, double ri, const double *cj, double rj,
                    const double *ck, double rk, int sigma, double rho, bool &ok) {
    V3<T> Ci = vec<T>(ci);
    V3<T> a = vec<T>(cj) - Ci, b = vec<T>(ck) - Ci;
    V3<T> m = cross(a, b);
    T M2 = dot(m, m);
    T r = num<T>(rho);
    T si = num<T>(ri) + r, sj = num<T>(rj) + r, sk = num<T>(rk) + r;
    T A = si * si - sj * sj + dot(a, a);
    T B = si * si - sk * sk + dot(b, b);
    V3<T> Z = A * cross(b, m) + B * cross(m, a);
    V3<T> E = (num<T>(2.0) * M2) * (vec<T>(x) - Ci) - Z;
    T Ts = num<T>(4.0) * M2 * M2 * si * si - dot(Z, Z);
    T P = dot(E, E) + Ts - num<T>(4.0) * M2 * M2 * r * r;
    T mE = dot(m, E);
    T q = sigma > 0 ? -(num<T>(2.0) * mE) : num<T>(2.0) * mE;
    return sqrt2_sign(P, M2, q, Ts, ok) < 0;
}

// Evaluate with the certified FP64 form first, exactly when it cannot decide.
#define CERTIFIED(call_ap, call_dy)   \
    [&]() {                           \
        bool ok_ = true;              \
        auto res_ = call_ap;          \
        if (ok_) return res_;         \
        bool ok2_ = true;             \
        (void)ok2_;                   \
        return call_dy;               \
    }()

}  // namespace

int exact_sign_sqrt2(double a, double X, double b, double Y) {
    bool ok = true;
    int s = sqrt2_sign(ap(a), ap(X), ap(b), ap(Y), ok);
    if (ok) return s;
    ok = true;
    return sqrt2_sign(dy(a), dy(X), dy(b), dy(Y), ok);
}

ExactMolecule::ExactMolecule(const double *centres, const double *radii, int64_t n, double rho,
                             const int32_t *probe_atoms, const int8_t *probe_sign, int64_t nprobe)
    : c_(centres, centres + 3 * n), r_(radii, radii + n), rho_(rho), n_(n) {
    smax_ = 0.0;
    double hi[3];
    for (int a = 0; a < 3; ++a) {
        lo_[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i) {
        smax_ = std::max(smax_, r_[i] + rho);
        for (int a = 0; a < 3; ++a) {
            lo_[a] = std::min(lo_[a], c_[3 * i + a]);
            hi[a] = std::max(hi[a], c_[3 * i + a]);
        }
    }
    cell_ = 2.0 * smax_ + 1e-6;
    long long nc = 1;
    for (;;) {
        nc = 1;
        for (int a = 0; a < 3; ++a) {
            nc_[a] = (int)std::floor((hi[a] - lo_[a]) / cell_) + 1;
            nc *= nc_[a];
        }
        if (nc <= 4 * n + 64) break;
        cell_ *= 1.5;
    }
    cstart_.assign((size_t)nc + 1, 0);
    std::vector<int> cid((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int q[3];
        for (int a = 0; a < 3; ++a)
            q[a] = std::min(nc_[a] - 1, std::max(0, (int)std::floor((c_[3 * i + a] - lo_[a]) / cell_)));
        cid[(size_t)i] = q[0] + nc_[0] * (q[1] + nc_[1] * q[2]);
        ++cstart_[(size_t)cid[(size_t)i] + 1];
    }
    for (long long q = 0; q < nc; ++q) cstart_[(size_t)q + 1] += cstart_[(size_t)q];
    catom_.assign((size_t)n, 0);
    std::vector<int> fill(cstart_.begin(), cstart_.end() - 1);
    for (int64_t i = 0; i < n; ++i) catom_[(size_t)fill[(size_t)cid[(size_t)i]]++] = (int)i;

    pa_.assign(probe_atoms, probe_atoms + 3 * nprobe);
    ps_.assign((size_t)nprobe, 0);
    pp_.assign((size_t)(3 * nprobe), 0.0);
    for (int64_t v = 0; v < nprobe; ++v) {
        ps_[(size_t)v] = probe_sign[v];
        // FP64 position for the reach filter only: the equidistant point of
        // the three SAS spheres on the chosen side (Cramer's rule on the
        // radical planes and the plane through the centres)
        const double *ci = &c_[3 * (size_t)pa_[3 * v]], *cj = &c_[3 * (size_t)pa_[3 * v + 1]],
                     *ck = &c_[3 * (size_t)pa_[3 * v + 2]];
        const double si = r_[(size_t)pa_[3 * v]] + rho, sj = r_[(size_t)pa_[3 * v + 1]] + rho,
                     sk = r_[(size_t)pa_[3 * v + 2]] + rho;
        double a[3], b[3], m[3], bm[3], ma[3];
        for (int t = 0; t < 3; ++t) {
            a[t] = cj[t] - ci[t];
            b[t] = ck[t] - ci[t];
        }
        m[0] = a[1] * b[2] - a[2] * b[1];
        m[1] = a[2] * b[0] - a[0] * b[2];
        m[2] = a[0] * b[1] - a[1] * b[0];
        bm[0] = b[1] * m[2] - b[2] * m[1];
        bm[1] = b[2] * m[0] - b[0] * m[2];
        bm[2] = b[0] * m[1] - b[1] * m[0];
        ma[0] = m[1] * a[2] - m[2] * a[1];
        ma[1] = m[2] * a[0] - m[0] * a[2];
        ma[2] = m[0] * a[1] - m[1] * a[0];
        const double M2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        const double A = si * si - sj * sj + (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        const double B = si * si - sk * sk + (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double z[3], zz = 0.0;
        for (int t = 0; t < 3; ++t) {
            z[t] = (A * bm[t] + B * ma[t]) / (2.0 * M2);
            zz += z[t] * z[t];
        }
        const double T = std::sqrt(std::max(0.0, (si * si - zz) / M2)) * (probe_sign[v] > 0 ? 1 : -1);
        for (int t = 0; t < 3; ++t) pp_[(size_t)(3 * v + t)] = ci[t] + z[t] + T * m[t];
    }
    // probes listed under each of their atoms
    pstart_.assign((size_t)n + 1, 0);
    for (int64_t v = 0; v < nprobe; ++v)
        for (int t = 0; t < 3; ++t) ++pstart_[(size_t)pa_[3 * v + t] + 1];
    for (int64_t i = 0; i < n; ++i) pstart_[(size_t)i + 1] += pstart_[(size_t)i];
    plist_.assign((size_t)pstart_[(size_t)n], 0);
    std::vector<int> pf(pstart_.begin(), pstart_.end() - 1);
    for (int64_t v = 0; v < nprobe; ++v)
        for (int t = 0; t < 3; ++t) plist_[(size_t)pf[(size_t)pa_[3 * v + t]]++] = (int)v;
}

void ExactMolecule::near(const double x[3], double reach, std::vector<int> &out) const {
    out.clear();
    int a0[3], a1[3];
    for (int a = 0; a < 3; ++a) {
        a0[a] = std::min(nc_[a] - 1, std::max(0, (int)std::floor((x[a] - reach - lo_[a]) / cell_)));
        a1[a] = std::min(nc_[a] - 1, std::max(0, (int)std::floor((x[a] + reach - lo_[a]) / cell_)));
    }
    for (int k = a0[2]; k <= a1[2]; ++k)
        for (int j = a0[1]; j <= a1[1]; ++j)
            for (int i = a0[0]; i <= a1[0]; ++i) {
                const int cidx = i + nc_[0] * (j + nc_[1] * k);
                for (int q = cstart_[(size_t)cidx]; q < cstart_[(size_t)cidx + 1]; ++q) {
                    const int t = catom_[(size_t)q];
                    const double *c = &c_[3 * (size_t)t];
                    const double d2 = (x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) +
                                      (x[2] - c[2]) * (x[2] - c[2]);
                    if (d2 < (reach + 1e-6) * (reach + 1e-6)) out.push_back(t);
                }
            }
}

// SAS neighbours of i (a superset: centre distance below s_i + s_k + 1e-6).
const std::vector<int> &ExactMolecule::nbrs(int i) {
    auto it = nbr_.find(i);
    if (it != nbr_.end()) return it->second;
    std::vector<int> cand;
    near(&c_[3 * (size_t)i], r_[(size_t)i] + rho_ + smax_, cand);
    std::vector<int> out;
    const double *ci = &c_[3 * (size_t)i];
    for (int k : cand) {
        if (k == i) continue;
        const double *ck = &c_[3 * (size_t)k];
        const double d = std::sqrt((ci[0] - ck[0]) * (ci[0] - ck[0]) + (ci[1] - ck[1]) * (ci[1] - ck[1]) +
                                   (ci[2] - ck[2]) * (ci[2] - ck[2]));
        if (d < r_[(size_t)i] + r_[(size_t)k] + 2.0 * rho_ + 1e-6) out.push_back(k);
    }
    std::sort(out.begin(), out.end());
    return nbr_.emplace(i, std::move(out)).first->second;
}

bool ExactMolecule::probe_within(int v, const double x[3]) {
    const int i = pa_[3 * (size_t)v], j = pa_[3 * (size_t)v + 1], k = pa_[3 * (size_t)v + 2];
    const double *ci = &c_[3 * (size_t)i], *cj = &c_[3 * (size_t)j], *ck = &c_[3 * (size_t)k];
    return CERTIFIED(probe_within_t<Ap>(x, ci, r_[i], cj, r_[j], ck, r_[k], ps_[v], rho_, ok_),
                     probe_within_t<Dy>(x, ci, r_[i], cj, r_[j], ck, r_[k], ps_[v], rho_, ok2_));
}

// Face of atom i: within rho of x (|x - c_i| < s_i + rho) and admissible.
bool ExactMolecule::face_candidate(int i, const double x[3]) {
    const double *ci = &c_[3 * (size_t)i];
    const int w = CERTIFIED(ball_sign<Ap>(x, ci, r_[i], rho_, 2, ok_),
                            ball_sign<Dy>(x, ci, r_[i], rho_, 2, ok2_));
    if (w >= 0) return false;
    for (int k : nbrs(i)) {
        const double *ck = &c_[3 * (size_t)k];
        const int s = CERTIFIED(face_cut_sign<Ap>(x, ci, r_[i], ck, r_[k], rho_, ok_),
                                face_cut_sign<Dy>(x, ci, r_[i], ck, r_[k], rho_, ok2_));
        if (s < 0) return false;
    }
    return true;
}

bool ExactMolecule::circle_candidate(int i, int j, const double x[3]) {
    const double *ci = &c_[3 * (size_t)i], *cj = &c_[3 * (size_t)j];
    const bool ex = CERTIFIED(circle_exists<Ap>(ci, r_[i], cj, r_[j], rho_, ok_),
                              circle_exists<Dy>(ci, r_[i], cj, r_[j], rho_, ok2_));
    if (!ex) return false;
    int stage = 0;  // which evaluation decided: 0 FP64, 1 exact
    bool within, axis_pt;
    {
        bool ok = true;
        Circle<Ap> c = circle<Ap>(ci, r_[i], cj, r_[j], rho_);
        within = circle_within(c, x, rho_, ok);
        axis_pt = ok && within ? on_axis(c, x, ok) : false;
        if (!ok) stage = 1;
    }
    if (stage == 1) {
        bool ok = true;
        Circle<Dy> c = circle<Dy>(ci, r_[i], cj, r_[j], rho_);
        within = circle_within(c, x, rho_, ok);
        axis_pt = within ? on_axis(c, x, ok) : false;
    }
    if (!within) return false;
    int axis = -1;
    if (axis_pt) {
        const double v[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
        axis = 0;
        for (int a = 1; a < 3; ++a)
            if (std::fabs(v[a]) < std::fabs(v[axis])) axis = a;
    }
    Circle<Ap> ca = circle<Ap>(ci, r_[i], cj, r_[j], rho_);
    Circle<Dy> cd;
    bool have_dy = false;
    for (int k : nbrs(i)) {
        if (k == j) continue;
        const double *ck = &c_[3 * (size_t)k];
        bool ok = true;
        int s = circle_cut_sign(ca, x, axis, ck, r_[k], rho_, ok);
        if (!ok) {
            if (!have_dy) {
                cd = circle<Dy>(ci, r_[i], cj, r_[j], rho_);
                have_dy = true;
            }
            ok = true;
            s = circle_cut_sign(cd, x, axis, ck, r_[k], rho_, ok);
        }
        if (s < 0) return false;
    }
    return true;
}

int ExactMolecule::label(const double x[3]) {
    std::vector<int> at;
    near(x, smax_ + rho_, at);
    bool inU = false;
    std::vector<int> reach;  // atoms within s_i + rho of x (faces, circles)
    for (int i : at) {
        const double *ci = &c_[3 * (size_t)i];
        const int v = CERTIFIED(ball_sign<Ap>(x, ci, r_[i], rho_, 0, ok_),
                                ball_sign<Dy>(x, ci, r_[i], rho_, 0, ok2_));
        if (v <= 0) return 1;
        const int u = CERTIFIED(ball_sign<Ap>(x, ci, r_[i], rho_, 1, ok_),
                                ball_sign<Dy>(x, ci, r_[i], rho_, 1, ok2_));
        if (u < 0) inU = true;
        reach.push_back(i);
    }
    if (!inU) return 0;
    // concave probe positions of the atoms within reach (a probe within rho
    // of x touches atoms within s + rho of x)
    for (int i : reach)
        for (int q = pstart_[(size_t)i]; q < pstart_[(size_t)i + 1]; ++q) {
            const int v = plist_[(size_t)q];
            const double *p = &pp_[3 * (size_t)v];
            const double d2 = (x[0] - p[0]) * (x[0] - p[0]) + (x[1] - p[1]) * (x[1] - p[1]) +
                              (x[2] - p[2]) * (x[2] - p[2]);
            if (d2 > (rho_ + 1e-6) * (rho_ + 1e-6)) continue;
            if (probe_within(v, x)) return 0;
        }
    for (int i : reach)
        if (face_candidate(i, x)) return 0;
    for (int i : reach)
        for (int j : nbrs(i)) {
            if (j <= i) continue;
            if (std::find(reach.begin(), reach.end(), j) == reach.end()) continue;
            if (circle_candidate(i, j, x)) return 0;
        }
    return 1;
}

}  // namespace eses
