// su2.h -- SU(2) algebra for the SU(2) variant of the method (the field and
// particle equations of Sec. II.A and III.B for N_c = 2).
//
// A link is a unit quaternion U = w + i (a . sigma), stored as (w, a1, a2,
// a3); an algebra element X = X^a T^a with T^a = sigma^a / 2 is its real
// 3-vector of components.  Products, transports, the commutator and the
// exponential then have short closed forms:
//   (w1, a)(w2, b)  = (w1 w2 - a.b, w1 b + w2 a - a x b)
//   U X U^+         = (w^2 - |a|^2) X + 2 (a.X) a - 2 w (a x X)
//   i[A, B]         = -A x B
//   exp(i e X)      = (cos r, sin(r)/r * e X / 2),  r = e |X| / 2
//   Proj[M]         = 2 a for M = (w, a) (also for sums of links)
#pragma once
#include "su3.h"

namespace cpic {

template <typename T> struct q4 {
    T w, x, y, z;
};
template <typename T> struct v3 {
    T v[3];
};

template <typename T> CPIC_HD q4<T> qmul(const q4<T>& p, const q4<T>& q)
{
    return {p.w * q.w - p.x * q.x - p.y * q.y - p.z * q.z,
            p.w * q.x + q.w * p.x - (p.y * q.z - p.z * q.y),
            p.w * q.y + q.w * p.y - (p.z * q.x - p.x * q.z),
            p.w * q.z + q.w * p.z - (p.x * q.y - p.y * q.x)};
}
template <typename T> CPIC_HD q4<T> qadj(const q4<T>& p) { return {p.w, -p.x, -p.y, -p.z}; }
template <typename T> CPIC_HD q4<T> qadd(const q4<T>& p, const q4<T>& q)
{
    return {p.w + q.w, p.x + q.x, p.y + q.y, p.z + q.z};
}
template <typename T> CPIC_HD q4<T> qsub(const q4<T>& p, const q4<T>& q)
{
    return {p.w - q.w, p.x - q.x, p.y - q.y, p.z - q.z};
}
template <typename T> CPIC_HD q4<T> qone() { return {T(1), T(0), T(0), T(0)}; }
// Proj[M] = 2 (vector part)
template <typename T> CPIC_HD v3<T> qproj(const q4<T>& p) { return {{T(2) * p.x, T(2) * p.y, T(2) * p.z}}; }

// U X U^+ (transport_adj: U^+ X U, i.e. the same with a -> -a)
template <typename T> CPIC_HD v3<T> qtransport(const q4<T>& u, const v3<T>& X, bool adjoint = false)
{
    const T s = adjoint ? T(-1) : T(1);
    const T ax = s * u.x, ay = s * u.y, az = s * u.z;
    const T c0 = u.w * u.w - (ax * ax + ay * ay + az * az);
    const T d = T(2) * (ax * X.v[0] + ay * X.v[1] + az * X.v[2]);
    const T cx = ay * X.v[2] - az * X.v[1], cy = az * X.v[0] - ax * X.v[2], cz = ax * X.v[1] - ay * X.v[0];
    return {{c0 * X.v[0] + d * ax - T(2) * u.w * cx, c0 * X.v[1] + d * ay - T(2) * u.w * cy,
             c0 * X.v[2] + d * az - T(2) * u.w * cz}};
}
// i[A, B] = -A x B
template <typename T> CPIC_HD v3<T> vicomm(const v3<T>& A, const v3<T>& B)
{
    return {{-(A.v[1] * B.v[2] - A.v[2] * B.v[1]), -(A.v[2] * B.v[0] - A.v[0] * B.v[2]),
             -(A.v[0] * B.v[1] - A.v[1] * B.v[0])}};
}
template <typename T> CPIC_HD T vdot(const v3<T>& a, const v3<T>& b)
{
    return a.v[0] * b.v[0] + a.v[1] * b.v[1] + a.v[2] * b.v[2];
}
// exp(i e X^a T^a)
template <typename T> CPIC_HD q4<T> qexpi(const v3<T>& X, T e)
{
    const T hx = T(0.5) * e * X.v[0], hy = T(0.5) * e * X.v[1], hz = T(0.5) * e * X.v[2];
    const T r2 = hx * hx + hy * hy + hz * hz;
    const T r = T(sqrt(r2));
    // sin(r)/r by its series where r is small enough for three terms to be exact to rounding
    const T sinc = r2 < T(sizeof(T) == 8 ? 1e-4 : 1e-2) ? T(1) - r2 / T(6) * (T(1) - r2 / T(20) * (T(1) - r2 / T(42)))
                                                        : T(sin(r) / r);
    return {T(cos(r)), sinc * hx, sinc * hy, sinc * hz};
}
// rescale to unit norm (rounding drift of single-precision links)
template <typename T> CPIC_HD q4<T> qnormalize(const q4<T>& p)
{
    const T n = T(1) / T(sqrt(p.w * p.w + p.x * p.x + p.y * p.y + p.z * p.z));
    return {p.w * n, p.x * n, p.y * n, p.z * n};
}

}  // namespace cpic
