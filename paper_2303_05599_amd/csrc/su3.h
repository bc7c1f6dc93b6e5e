// su3.h -- SU(3) arithmetic for the CPIC kernels (device and host), templated
// on the storage/compute type T (double or float).
//
// Algebra elements X = X^a T^a (T^a = lambda^a / 2, Gell-Mann basis of
// Appendix B.1) are carried as their 8 real components; links as 3x3 complex
// matrices.  Everything here is written for register-resident use inside one
// thread: no shared state, no allocation.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#define CPIC_HD __host__ __device__ __forceinline__

namespace cpic {

template <typename T> struct cx {
    T re, im;
};
template <typename T> struct m3 {
    cx<T> e[9];  // row-major
};
template <typename T> struct a8 {
    T v[8];
};

template <typename T> constexpr T kInvSqrt3 = T(0.57735026918962576451);
template <typename T> constexpr T kSqrt3Half = T(0.86602540378443864676);

// fused multiply-add in the operand type (host and device)
CPIC_HD float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
CPIC_HD double fmaT(double a, double b, double c) { return ::fma(a, b, c); }

// ---------------------------------------------------------------- complex
template <typename T> CPIC_HD cx<T> cmul(cx<T> a, cx<T> b)
{
    return {fmaT(a.re, b.re, -a.im * b.im), fmaT(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
template <typename T> CPIC_HD cx<T> cmulc(cx<T> a, cx<T> b)
{
    return {fmaT(a.re, b.re, a.im * b.im), fmaT(a.im, b.re, -a.re * b.im)};
}
// conj(a) * b
template <typename T> CPIC_HD cx<T> ccmul(cx<T> a, cx<T> b)
{
    return {fmaT(a.re, b.re, a.im * b.im), fmaT(a.re, b.im, -a.im * b.re)};
}

// ---------------------------------------------------------------- 3x3
// Complex multiply-accumulate chains written as explicit fused multiply-adds
// (four per complex product): the compiler does not contract a*b - c*d + acc
// into two FMAs on its own.
// acc += a * b
template <typename T> CPIC_HD void cmac(cx<T>& acc, cx<T> a, cx<T> b)
{
    acc.re = fmaT(a.re, b.re, acc.re);
    acc.re = fmaT(-a.im, b.im, acc.re);
    acc.im = fmaT(a.re, b.im, acc.im);
    acc.im = fmaT(a.im, b.re, acc.im);
}
// acc += a * conj(b)
template <typename T> CPIC_HD void cmacc(cx<T>& acc, cx<T> a, cx<T> b)
{
    acc.re = fmaT(a.re, b.re, acc.re);
    acc.re = fmaT(a.im, b.im, acc.re);
    acc.im = fmaT(a.im, b.re, acc.im);
    acc.im = fmaT(-a.re, b.im, acc.im);
}
// acc += conj(a) * b
template <typename T> CPIC_HD void ccmac(cx<T>& acc, cx<T> a, cx<T> b)
{
    acc.re = fmaT(a.re, b.re, acc.re);
    acc.re = fmaT(a.im, b.im, acc.re);
    acc.im = fmaT(a.re, b.im, acc.im);
    acc.im = fmaT(-a.im, b.re, acc.im);
}

// C = A B
template <typename T> CPIC_HD m3<T> mul(const m3<T>& A, const m3<T>& B)
{
    m3<T> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<T> acc = cmul(A.e[3 * i], B.e[j]);
            cmac(acc, A.e[3 * i + 1], B.e[3 + j]);
            cmac(acc, A.e[3 * i + 2], B.e[6 + j]);
            C.e[3 * i + j] = acc;
        }
    return C;
}
// C = A B^+
template <typename T> CPIC_HD m3<T> mul_adj(const m3<T>& A, const m3<T>& B)
{
    m3<T> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<T> acc = cmulc(A.e[3 * i], B.e[3 * j]);
            cmacc(acc, A.e[3 * i + 1], B.e[3 * j + 1]);
            cmacc(acc, A.e[3 * i + 2], B.e[3 * j + 2]);
            C.e[3 * i + j] = acc;
        }
    return C;
}
// C = A^+ B
template <typename T> CPIC_HD m3<T> adj_mul(const m3<T>& A, const m3<T>& B)
{
    m3<T> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<T> acc = ccmul(A.e[i], B.e[j]);
            ccmac(acc, A.e[3 + i], B.e[3 + j]);
            ccmac(acc, A.e[6 + i], B.e[6 + j]);
            C.e[3 * i + j] = acc;
        }
    return C;
}
template <typename T> CPIC_HD m3<T> adj(const m3<T>& A)
{
    m3<T> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) C.e[3 * i + j] = {A.e[3 * j + i].re, -A.e[3 * j + i].im};
    return C;
}
template <typename T> CPIC_HD m3<T> identity()
{
    m3<T> C;
#pragma unroll
    for (int k = 0; k < 9; k++) C.e[k] = {T(0), T(0)};
    C.e[0].re = C.e[4].re = C.e[8].re = T(1);
    return C;
}

// ---------------------------------------------------------------- algebra
template <typename T> CPIC_HD a8<T> azero()
{
    a8<T> r;
#pragma unroll
    for (int a = 0; a < 8; a++) r.v[a] = T(0);
    return r;
}
template <typename T> CPIC_HD void axpy(a8<T>& y, T s, const a8<T>& x)
{
#pragma unroll
    for (int a = 0; a < 8; a++) y.v[a] = fmaT(s, x.v[a], y.v[a]);
}
template <typename T> CPIC_HD T dot(const a8<T>& x, const a8<T>& y)
{
    T s = x.v[0] * y.v[0];
#pragma unroll
    for (int a = 1; a < 8; a++) s = fmaT(x.v[a], y.v[a], s);
    return s;
}

// Hermitian matrix sum_a x^a T^a
template <typename T> CPIC_HD m3<T> herm(const a8<T>& x)
{
    const T h = T(0.5);
    const T d8 = x.v[7] * kInvSqrt3<T>;
    m3<T> H;
    H.e[0] = {h * (x.v[2] + d8), 0};
    H.e[4] = {h * (-x.v[2] + d8), 0};
    H.e[8] = {-d8, 0};
    H.e[1] = {h * x.v[0], -h * x.v[1]};
    H.e[3] = {h * x.v[0], h * x.v[1]};
    H.e[2] = {h * x.v[3], -h * x.v[4]};
    H.e[6] = {h * x.v[3], h * x.v[4]};
    H.e[5] = {h * x.v[5], -h * x.v[6]};
    H.e[7] = {h * x.v[5], h * x.v[6]};
    return H;
}
// components 2 Re Tr(T^a M) of a Hermitian matrix, from its upper triangle
template <typename T> CPIC_HD a8<T> herm_comp(cx<T> m00, cx<T> m11, cx<T> m22, cx<T> m01, cx<T> m02, cx<T> m12)
{
    a8<T> r;
    r.v[0] = T(2) * m01.re;
    r.v[1] = T(-2) * m01.im;
    r.v[2] = m00.re - m11.re;
    r.v[3] = T(2) * m02.re;
    r.v[4] = T(-2) * m02.im;
    r.v[5] = T(2) * m12.re;
    r.v[6] = T(-2) * m12.im;
    r.v[7] = (m00.re + m11.re - T(2) * m22.re) * kInvSqrt3<T>;
    return r;
}
template <typename T> CPIC_HD a8<T> herm_comp(const m3<T>& M) { return herm_comp(M.e[0], M.e[4], M.e[8], M.e[1], M.e[2], M.e[5]); }

// Proj[M]^a = 2 Im Tr(T^a M): the traceless Hermitian part of -i (M - M^+)/2,
// the generator part of M (the "[.]_ah" projection of Sec. II.A, III.B).
template <typename T> CPIC_HD a8<T> proj(const m3<T>& M)
{
    a8<T> r;
    r.v[0] = M.e[3].im + M.e[1].im;
    r.v[1] = M.e[1].re - M.e[3].re;
    r.v[2] = M.e[0].im - M.e[4].im;
    r.v[3] = M.e[6].im + M.e[2].im;
    r.v[4] = M.e[2].re - M.e[6].re;
    r.v[5] = M.e[7].im + M.e[5].im;
    r.v[6] = M.e[5].re - M.e[7].re;
    r.v[7] = (M.e[0].im + M.e[4].im - T(2) * M.e[8].im) * kInvSqrt3<T>;
    return r;
}
// Proj[A B^+] without forming the diagonal real parts
template <typename T> CPIC_HD a8<T> proj_mul_adj(const m3<T>& A, const m3<T>& B)
{
    return proj(mul_adj(A, B));
}

// U X U^+ (forward parallel transport of an algebra element)
template <typename T> CPIC_HD a8<T> transport(const m3<T>& U, const a8<T>& x)
{
    m3<T> A = mul(U, herm(x));
    cx<T> m[6];  // 00 11 22 01 02 12 of A U^+
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int i = ii[q], j = jj[q];
        cx<T> acc = cmulc(A.e[3 * i], U.e[3 * j]);
        cmacc(acc, A.e[3 * i + 1], U.e[3 * j + 1]);
        cmacc(acc, A.e[3 * i + 2], U.e[3 * j + 2]);
        m[q] = acc;
    }
    return herm_comp(m[0], m[1], m[2], m[3], m[4], m[5]);
}
// U^+ X U (backward parallel transport)
template <typename T> CPIC_HD a8<T> transport_adj(const m3<T>& U, const a8<T>& x)
{
    m3<T> A = mul(herm(x), U);  // X U
    cx<T> m[6];                 // of U^+ (X U)
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int i = ii[q], j = jj[q];
        cx<T> acc = ccmul(U.e[i], A.e[j]);
        ccmac(acc, U.e[3 + i], A.e[3 + j]);
        ccmac(acc, U.e[6 + i], A.e[6 + j]);
        m[q] = acc;
    }
    return herm_comp(m[0], m[1], m[2], m[3], m[4], m[5]);
}

// (i [A, B])^c = -f_abc A^a B^b, with the nonzero f_abc of Table I.
template <typename T> CPIC_HD a8<T> icomm(const a8<T>& A, const a8<T>& B)
{
    a8<T> C = azero<T>();
    // each triple (a,b,c,f): C^c -= f (A^a B^b - A^b B^a), and cyclic
#define CPIC_F(a, b, c, f)                                                          \
    {                                                                               \
        const T ff = (f);                                                           \
        C.v[c] = fmaT(-ff, fmaT(A.v[a], B.v[b], -A.v[b] * B.v[a]), C.v[c]);           \
        C.v[a] = fmaT(-ff, fmaT(A.v[b], B.v[c], -A.v[c] * B.v[b]), C.v[a]);           \
        C.v[b] = fmaT(-ff, fmaT(A.v[c], B.v[a], -A.v[a] * B.v[c]), C.v[b]);           \
    }
    CPIC_F(0, 1, 2, T(1));
    CPIC_F(0, 3, 6, T(0.5));
    CPIC_F(0, 4, 5, T(-0.5));
    CPIC_F(1, 3, 5, T(0.5));
    CPIC_F(1, 4, 6, T(0.5));
    CPIC_F(2, 3, 4, T(0.5));
    CPIC_F(2, 5, 6, T(-0.5));
    CPIC_F(3, 4, 7, kSqrt3Half<T>);
    CPIC_F(5, 6, 7, kSqrt3Half<T>);
#undef CPIC_F
    return C;
}

// exp(i eps X) for X = x^a T^a, by the Cayley-Hamilton reduction
// Y^3 = c1 Y + c0 (Y = eps X traceless Hermitian, c1 = Tr Y^2 / 2,
// c0 = det Y) applied to the exponential series: exp(iY) = f0 + f1 Y + f2 Y^2.
// Large arguments are halved s times and the result squared back.
template <typename T> CPIC_HD m3<T> expi(const a8<T>& x, T eps)
{
    a8<T> y;
#pragma unroll
    for (int a = 0; a < 8; a++) y.v[a] = eps * x.v[a];
    T c1 = T(0.25) * dot(y, y);
    int s = 0;
    while (c1 > T(3)) {  // eigenvalues bounded by sqrt(4 c1 / 3) <= 2
#pragma unroll
        for (int a = 0; a < 8; a++) y.v[a] *= T(0.5);
        c1 *= T(0.25);
        s++;
    }
    m3<T> Y = herm(y);
    m3<T> Y2 = mul(Y, Y);
    // c0 = det Y = Tr(Y^3) / 3 (real)
    T tr3 = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) tr3 += Y.e[3 * i + k].re * Y2.e[3 * k + i].re - Y.e[3 * i + k].im * Y2.e[3 * k + i].im;
    const T c0 = tr3 / T(3);
    // Y^k = a_k + b_k Y + d_k Y^2; exp(iY) = sum_k i^k / k! Y^k
    T ak = 1, bk = 0, dk = 0, fac = 1;
    T f0r = 1, f0i = 0, f1r = 0, f1i = 0, f2r = 0, f2i = 0;
    constexpr int K = sizeof(T) == 8 ? 28 : 16;
#pragma unroll
    for (int k = 1; k <= K; k++) {
        T an = c0 * dk, bn = fmaT(c1, dk, ak), dn = bk;
        ak = an; bk = bn; dk = dn;
        fac = fac / T(k);
        const int ph = k & 3;  // i^k = 1, i, -1, -i
        const T sg = (ph < 2) ? fac : -fac;
        if (ph & 1) {
            f0i = fmaT(sg, ak, f0i); f1i = fmaT(sg, bk, f1i); f2i = fmaT(sg, dk, f2i);
        } else {
            f0r = fmaT(sg, ak, f0r); f1r = fmaT(sg, bk, f1r); f2r = fmaT(sg, dk, f2r);
        }
    }
    m3<T> R;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        cx<T> yv = Y.e[q], y2 = Y2.e[q];
        R.e[q] = {fmaT(f1r, yv.re, fmaT(-f1i, yv.im, fmaT(f2r, y2.re, -f2i * y2.im))),
                  fmaT(f1r, yv.im, fmaT(f1i, yv.re, fmaT(f2r, y2.im, f2i * y2.re)))};
    }
    R.e[0].re += f0r; R.e[0].im += f0i;
    R.e[4].re += f0r; R.e[4].im += f0i;
    R.e[8].re += f0r; R.e[8].im += f0i;
    for (int q = 0; q < s; q++) R = mul(R, R);
    return R;
}

// Generator of a link: the traceless Hermitian X with exp(iX) = U up to a
// centre element (the traceless part of -i log U, principal branch), found
// by the fixed-point iteration X <- X + Proj[exp(-iX/2) U exp(-iX/2)] from
// X = Proj[U].  For commuting X and U the error e (per eigenphase) maps to
// e - sin e, so the iteration converges cubically from any eigenphase in
// (-pi, pi); the symmetric splitting keeps the leading commutator out of
// the correction.  Stops when the correction is below tol or after maxit.
template <typename T> CPIC_HD a8<T> link_generator(const m3<T>& U, T tol, int maxit)
{
    a8<T> X = proj(U);
    for (int k = 0; k < maxit; k++) {
        const m3<T> H = expi(X, T(-0.5));
        const a8<T> D = proj(mul(mul(H, U), H));
        T m = 0;
#pragma unroll
        for (int a = 0; a < 8; a++) {
            X.v[a] += D.v[a];
            m = fmax(m, fabs(D.v[a]));
        }
        if (m <= tol) break;
    }
    return X;
}

// nearest-SU(3) style projection used to remove rounding drift: Gram-Schmidt
// on rows 1 and 2, row 3 = conj(r1 x r2) (unit determinant by construction)
template <typename T> CPIC_HD m3<T> reunitarize(const m3<T>& W)
{
    m3<T> R;
    T n0 = 0;
#pragma unroll
    for (int j = 0; j < 3; j++) n0 += W.e[j].re * W.e[j].re + W.e[j].im * W.e[j].im;
    T r0 = T(1) / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; j++) R.e[j] = {W.e[j].re * r0, W.e[j].im * r0};
    cx<T> ip = {0, 0};
#pragma unroll
    for (int j = 0; j < 3; j++) {
        cx<T> t = ccmul(R.e[j], W.e[3 + j]);
        ip.re += t.re; ip.im += t.im;
    }
    T n1 = 0;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        cx<T> t = cmul(ip, R.e[j]);
        R.e[3 + j] = {W.e[3 + j].re - t.re, W.e[3 + j].im - t.im};
        n1 += R.e[3 + j].re * R.e[3 + j].re + R.e[3 + j].im * R.e[3 + j].im;
    }
    T r1 = T(1) / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; j++) R.e[3 + j] = {R.e[3 + j].re * r1, R.e[3 + j].im * r1};
    // r3 = conj(r1 x r2)
    auto crs = [&](int a, int b) {
        cx<T> p = cmul(R.e[a], R.e[3 + b]), q = cmul(R.e[b], R.e[3 + a]);
        return cx<T>{p.re - q.re, -(p.im - q.im)};
    };
    R.e[6] = crs(1, 2);
    R.e[7] = crs(2, 0);
    R.e[8] = crs(0, 1);
    return R;
}

}  // namespace cpic
