// wong.h -- one test particle's step at t_n (Sec. III.B), as the lane that
// owns the particle takes it: the nearest grid point, the CPIC colour
// rotation for the cells crossed since t_{n-1} ([eq:colorrotnum]), the
// explicit Euler step of the Wong equations in Milne coordinates once the
// charge has been contracted with the six colour fields at the cell, and the
// particle's momentum-broadening terms ([eq:mombroad]) on recording steps.
// Shared by the gather push (push.hip) and the tile push of the fused step
// (fused.hip), which differ only in where the fields at the cell come from.
#pragma once
#include "cellfields.h"

namespace cpic {

// components of A^+ Q A
template <typename T> __device__ __forceinline__ a8<T> rotate(const m3<T>& A, const a8<T>& Q) { return transport_adj(A, Q); }

// Replace the spectrum of Q by the sorted spectrum of Q0 (keeps the
// eigenvectors): restores both classical Casimirs exactly.  Written with
// compile-time indices only (no private arrays indexed at run time).
template <typename T> __device__ __forceinline__ void null_vector(const m3<T>& H, T l, cx<T>* v)
{
    // rows of H - l: the cross product of two rows is orthogonal to both;
    // keep the largest of the three choices
    cx<T> m[9];
#pragma unroll
    for (int q = 0; q < 9; q++) m[q] = H.e[q];
    m[0].re -= l; m[4].re -= l; m[8].re -= l;
    T best = T(-1);
#pragma unroll
    for (int pr = 0; pr < 3; pr++) {
        const int ra = pr == 2 ? 1 : 0, rb = pr == 0 ? 1 : 2;
        cx<T> c[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const cx<T> u = cmul(m[3 * ra + j1], m[3 * rb + j2]), w = cmul(m[3 * ra + j2], m[3 * rb + j1]);
            c[j] = {u.re - w.re, u.im - w.im};
        }
        const T nn = c[0].re * c[0].re + c[0].im * c[0].im + c[1].re * c[1].re + c[1].im * c[1].im +
                     c[2].re * c[2].re + c[2].im * c[2].im;
        const bool take = nn > best;
        best = take ? nn : best;
#pragma unroll
        for (int j = 0; j < 3; j++) v[j] = take ? c[j] : v[j];
    }
}
template <typename T> __device__ a8<T> renorm_charge(const a8<T>& Q, const double* eig0)
{
    const m3<T> H = herm(Q);
    const T p = T(0.25) * dot(Q, Q);  // Tr H^2 / 2
    if (!(p > T(0))) return Q;
    // det H
    const cx<T> d0 = cmul(H.e[4], H.e[8]), d1 = cmul(H.e[5], H.e[7]);
    const cx<T> e0 = cmul(H.e[3], H.e[8]), e1 = cmul(H.e[5], H.e[6]);
    const cx<T> f0 = cmul(H.e[3], H.e[7]), f1 = cmul(H.e[4], H.e[6]);
    const T det = cmul(H.e[0], {d0.re - d1.re, d0.im - d1.im}).re - cmul(H.e[1], {e0.re - e1.re, e0.im - e1.im}).re +
                  cmul(H.e[2], {f0.re - f1.re, f0.im - f1.im}).re;
    const T r = sqrt(p / T(3));
    T arg = det / (T(2) * r * r * r);
    arg = arg > T(1) ? T(1) : (arg < T(-1) ? T(-1) : arg);
    const T th = acos(arg) / T(3);
    // roots 2r cos(th - 2 pi k/3) with th in [0, pi/3]: k = 0 largest,
    // k = 1 middle, k = 2 smallest
    const T mid = T(2) * r * cos(th - T(2.0943951023931954923));
    const T lo = T(2) * r * cos(th - T(4.1887902047863909846));
    cx<T> v0[3], v1[3], v2[3];
    null_vector(H, lo, v0);
    null_vector(H, mid, v1);
    T n0 = 0;
#pragma unroll
    for (int j = 0; j < 3; j++) n0 += v0[j].re * v0[j].re + v0[j].im * v0[j].im;
    const T i0 = T(1) / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; j++) { v0[j].re *= i0; v0[j].im *= i0; }
    cx<T> ip = {0, 0};
#pragma unroll
    for (int j = 0; j < 3; j++) { const cx<T> q = ccmul(v0[j], v1[j]); ip.re += q.re; ip.im += q.im; }
    T n1 = 0;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const cx<T> q = cmul(ip, v0[j]);
        v1[j].re -= q.re; v1[j].im -= q.im;
        n1 += v1[j].re * v1[j].re + v1[j].im * v1[j].im;
    }
    const T i1 = T(1) / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; j++) { v1[j].re *= i1; v1[j].im *= i1; }
#pragma unroll
    for (int j = 0; j < 3; j++) {  // v2 = conj(v0 x v1)
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const cx<T> u = cmul(v0[j1], v1[j2]), w = cmul(v0[j2], v1[j1]);
        v2[j] = {u.re - w.re, -(u.im - w.im)};
    }
    // Q' = sum_k eig0_k v_k v_k^+, only the upper triangle is needed
    const T l0 = T(eig0[0]), l1 = T(eig0[1]), l2 = T(eig0[2]);
    auto ent = [&](int i, int j) {
        const cx<T> a = cmulc(v0[i], v0[j]), b = cmulc(v1[i], v1[j]), c = cmulc(v2[i], v2[j]);
        return cx<T>{l0 * a.re + l1 * b.re + l2 * c.re, l0 * a.im + l1 * b.im + l2 * c.im};
    };
    return herm_comp(ent(0, 0), ent(1, 1), ent(2, 2), ent(0, 1), ent(0, 2), ent(1, 2));
}


// The owner lane's copy of a particle during the step.
template <typename T> struct Particle {
    a8<T> Q;
    T x, y, eta, px, py, pe, pt_ode;
    int nx, ny;  // nearest grid point at t_n
};

// the nearest grid point at t_n (static particles keep their cell)
template <typename T>
__device__ __forceinline__ void particle_cell(const View<T>& R, const View<int>& C, uint32_t po, uint32_t pi, int N,
                                              bool is_static, Particle<T>& s)
{
    s.x = 0;
    s.y = 0;
    if (is_static) {
        s.nx = bld_i(C, pi, 0);
        s.ny = bld_i(C, pi, 1);
        return;
    }
    s.x = bld(R, po, PX_);
    s.y = bld(R, po, PY_);
    const int nx = (int)floor(s.x + T(0.5)), ny = (int)floor(s.y + T(0.5));
    s.nx = nx >= N ? nx - N : nx;
    s.ny = ny >= N ? ny - N : ny;
}

// Loads the charge and the momenta and, from the second push step on, rotates
// the charge with the links crossed since the last step (x first, then y from
// the new column) and with the rapidity Wilson line exp(i deta phi) at the
// cell, all at t_n from the buffer set A; in single precision the charge is
// renormalised on reunitarisation steps.  SPLIT: scheduling barriers between
// the two link loads (keeps the registers of the eight-wave push low).
template <typename T, bool LOGQ, bool SPLIT>
__device__ __forceinline__ void particle_load_rotate(const View<T>& A, const View<T>& R, const View<int>& C,
                                                     uint32_t po, uint32_t pi, const Cell& cell, const PushArgs& a,
                                                     int n, bool live, bool renorm, int* err, Particle<T>& s)
{
    const int N = a.N;
#pragma unroll
    for (int q = 0; q < 8; q++) s.Q.v[q] = bld(R, po, PQ0 + q);
    s.px = bld(R, po, PPX);
    s.py = bld(R, po, PPY);
    s.pe = bld(R, po, PPETA);
    s.eta = bld(R, po, PETA_);
    s.pt_ode = a.is_static ? T(0) : bld(R, po, PPTAU);
    if (!LOGQ && !a.is_static && live && n > a.sc.n_form) {
        const int cx = bld_i(C, pi, 0), cy = bld_i(C, pi, 1);
        const T deta = bld(R, po, PDETA);
        int dx = s.nx - cx, dy = s.ny - cy;
        dx = dx > N / 2 ? dx - N : (dx < -N / 2 ? dx + N : dx);
        dy = dy > N / 2 ? dy - N : (dy < -N / 2 ? dy + N : dy);
        if (dx < -1 || dx > 1) atomicAdd(err, 1);
        if (dy < -1 || dy > 1) atomicAdd(err, 1);
        m3<T> Lx, Ly;
        if (dx != 0) Lx = vU(A, (uint32_t)(cy * N + (dx > 0 ? cx : wrap(cx - 1, N))) * (uint32_t)sizeof(T), 0);
        if (SPLIT) {
            if (dx == 1) s.Q = rotate(Lx, s.Q);
            else if (dx == -1) s.Q = transport(Lx, s.Q);
            CPIC_PHASE();
        }
        if (dy != 0) Ly = vU(A, (uint32_t)((dy > 0 ? cy : wrap(cy - 1, N)) * N + s.nx) * (uint32_t)sizeof(T), 1);
        const a8<T> ph = vA(A, cell.s, kCompPhi);
        if (!SPLIT) {
            if (dx == 1) s.Q = rotate(Lx, s.Q);
            else if (dx == -1) s.Q = transport(Lx, s.Q);  // U Q U^+
        }
        if (dy == 1) s.Q = rotate(Ly, s.Q);
        else if (dy == -1) s.Q = transport(Ly, s.Q);
        if (SPLIT) CPIC_PHASE();
        if (deta != T(0)) s.Q = rotate(expi(ph, deta), s.Q);
    }
    // charges are renormalised in single precision only (double-precision
    // contexts never schedule it); leaving it out of the double kernel
    // also keeps its trigonometric calls from needing scratch memory
    if constexpr (sizeof(T) == 4 && !LOGQ)
        if (!a.is_static && renorm && live) s.Q = renorm_charge(s.Q, a.q0eig);
}

// The Euler step with f[j] = Q . (field j at the cell) (job order E_x, E_y,
// E_eta, B_x, B_y, B_eta), the stores of the new record, and on recording
// steps the particle's four broadening terms in double precision (obs).
// Static particles integrate only the momentum (p^z in the PPETA slot).
template <typename T, bool LOGQ>
__device__ __forceinline__ void particle_update(const View<T>& A, const View<T>& R, const View<int>& C, uint32_t po,
                                                uint32_t pi, const Cell& cell, const PushArgs& a, int n,
                                                bool renorm, bool record, const T (&f)[6], Particle<T>& s,
                                                double (&obs)[4])
{
    const int N = a.N;
    const T dt = T(a.sc.dt), t = T(n * a.sc.dt);
    T px = s.px, py = s.py, pe = s.pe, eta = s.eta;
    if (a.is_static) {
        px += dt * f[0];
        py += dt * f[1];
        pe += dt * f[2];  // p^z of the static branch
        bst(R, po, PPX, px); bst(R, po, PPY, py); bst(R, po, PPETA, pe);
    } else {
        const T e1 = f[0], e2 = f[1], ee = f[2], b1 = f[3], b2 = f[4], be = f[5];
        const T mh = T(a.mhat);
        const T ptau = sqrt(px * px + py * py + (t * pe) * (t * pe) + mh * mh);
        const T v1 = px / ptau, v2 = py / ptau, vl = t * pe / ptau;
        const T npx = px + dt * (e1 + be * v2 - b2 * vl);
        const T npy = py + dt * (e2 - be * v1 + b1 * vl);
        const T npe = n > 0 ? pe + dt * (ee - b1 * v2 + b2 * v1 - T(2) * pe) / t : pe;
        // p^tau from its own equation of motion [eq:ptaueq] (Euler, with the
        // integrated value on the right-hand side), started from the
        // constraint at the formation step
        const T pt = n == a.sc.n_form ? ptau : s.pt_ode;
        const T npt = pt + dt * (ee * t * pe + e1 * px + e2 * py - t * pe * pe) / pt;
        if constexpr (LOGQ) {
            // Q_{n+1} = Q_n + dt i[Q_n, M_n]
            CPIC_PHASE();
            const int lx = min((int)floor(s.x), N - 1), ly = min((int)floor(s.y), N - 1);
            constexpr T tol = sizeof(T) == 8 ? T(1e-15) : T(1e-7);
            const a8<T> gx = link_generator(vU(A, (uint32_t)(s.ny * N + lx) * (uint32_t)sizeof(T), 0), tol, 50);
            const a8<T> gy = link_generator(vU(A, (uint32_t)(ly * N + s.nx) * (uint32_t)sizeof(T), 1), tol, 50);
            const a8<T> ph = vA(A, cell.s, kCompPhi);
            const T veta = pe / ptau;
            a8<T> M;
#pragma unroll
            for (int c = 0; c < 8; c++) M.v[c] = v1 * gx.v[c] + v2 * gy.v[c] + veta * ph.v[c];
            const a8<T> dq = icomm(s.Q, M);
#pragma unroll
            for (int c = 0; c < 8; c++) s.Q.v[c] += dt * dq.v[c];
        }
        T xn = s.x + dt * v1, yn = s.y + dt * v2;
        if (xn >= T(N)) xn -= T(N); else if (xn < T(0)) xn += T(N);
        if (yn >= T(N)) yn -= T(N); else if (yn < T(0)) yn += T(N);
        const T deta = dt * pe / ptau;
        eta += deta;
        px = npx; py = npy; pe = npe;
        bst(R, po, PX_, xn); bst(R, po, PY_, yn); bst(R, po, PETA_, eta);
        bst(R, po, PPX, px); bst(R, po, PPY, py); bst(R, po, PPETA, pe); bst(R, po, PDETA, deta);
        bst(R, po, PPTAU, npt);
        bst_i(C, pi, 0, s.nx);
        bst_i(C, pi, 1, s.ny);
        if (LOGQ || n > a.sc.n_form || renorm) {
#pragma unroll
            for (int q = 0; q < 8; q++) bst(R, po, PQ0 + q, s.Q.v[q]);
        }
    }
    if (record) {
        const T ux0 = bld(R, po, PUX0), uy0 = bld(R, po, PUY0), pt0 = bld(R, po, PPT0);
        const double dpx = px, dpy = py, tn = (double)(n + 1) * a.sc.dt;
        double pz;
        if (a.is_static) {
            pz = pe;
        } else {
            const double dpe = pe, et = eta;
            const double ptn = sqrt(dpx * dpx + dpy * dpy + (tn * dpe) * (tn * dpe) + a.mhat * a.mhat);
            pz = ptn * sinh(et) + tn * dpe * cosh(et);
        }
        const double par = dpx * (double)ux0 + dpy * (double)uy0;
        const double perp = -dpx * (double)uy0 + dpy * (double)ux0;
        const double p02 = (double)pt0 * (double)pt0;
        obs[0] += dpx * dpx + dpy * dpy - p02;
        obs[1] += pz * pz;
        obs[2] += par * par - p02;
        obs[3] += perp * perp;
    }
}

}  // namespace cpic
