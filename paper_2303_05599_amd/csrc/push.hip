// push.hip -- the Wong / CPIC particle push (Sec. III.B) and the momentum
// broadening sums [eq:mombroad].
//
// One thread owns one test particle (structure-of-arrays records).  At time
// t_n it (1) rotates its colour charge with the links it crossed since t_{n-1}
// and with the rapidity Wilson line, (2) reads the colour-electric and
// -magnetic fields at its nearest grid point from U(n), phi(n), E(n +- 1/2),
// pi(n +- 1/2), (3) takes one explicit Euler step.  On recording steps the
// block writes double-precision partial sums of the broadening; a second
// small kernel adds the block partials in a fixed order.
#include "internal.h"
#include "reduce.h"
#include "su3.h"
#include "bufio.h"

namespace cpic {

__device__ __forceinline__ int wrap(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

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

// compiler barrier between phases: keeps the links of one phase from being
// loaded (and held in registers) during another
#define CPIC_PHASE() __builtin_amdgcn_sched_barrier(0)

// Q . F for the six colour fields at site c, time t_n (Sec. III.B
// interpolations), hat units:
//   out[0..2] = Q.E_x, Q.E_y, Q.E_eta ; out[3..5] = Q.B_x, Q.B_y, Q.B_eta
// Work split when several lanes share one particle (TPP lanes, role = lane
// index within the particle): each role evaluates a subset of the six field
// contractions and leaves the others zero; the lanes then add their results.
//   TPP = 1: everything.
//   TPP = 2: role 0 E_x, E_y, B_x, B_y; role 1 E_eta and the clover.
//   TPP = 4: role 0 E_x and B_y; role 1 E_y and B_x; role 2 E_eta and clover
//            leaves 0, 1; role 3 clover leaves 2, 3.
template <int TPP> __device__ __forceinline__ bool does_E(int role, int i)
{
    return TPP == 1 || (TPP == 2 ? role == 0 : role == i);
}
template <int TPP> __device__ __forceinline__ bool does_Eeta(int role) { return TPP == 1 || (TPP == 2 ? role == 1 : role == 2); }
template <int TPP> __device__ __forceinline__ bool does_Bt(int role, int i)   // i = 0: B_y (phi along x), 1: B_x
{
    return TPP == 1 || (TPP == 2 ? role == 0 : role == i);
}
template <int TPP> __device__ __forceinline__ int leaf_begin(int role) { return TPP == 1 ? 0 : (TPP == 2 ? (role == 1 ? 0 : 4) : (role == 2 ? 0 : (role == 3 ? 2 : 4))); }
template <int TPP> __device__ __forceinline__ int leaf_end(int role) { return TPP == 1 ? 4 : (TPP == 2 ? 4 : (role == 2 ? 2 : 4)); }

template <typename T, int TPP>
__device__ __forceinline__ void forces_dot(const View<T>& A, const View<T>& B, int N, int cx, int cy, int n, T t,
                                           bool electric_only, const a8<T>& Q, T* out, int role)
{
    constexpr uint32_t b = sizeof(T);
    const int xm = wrap(cx - 1, N), xp = wrap(cx + 1, N), ym = wrap(cy - 1, N), yp = wrap(cy + 1, N);
    const uint32_t s = (uint32_t)(cy * N + cx) * b;
    const uint32_t s_xm = (uint32_t)(cy * N + xm) * b, s_xp = (uint32_t)(cy * N + xp) * b;
    const uint32_t s_ym = (uint32_t)(ym * N + cx) * b, s_yp = (uint32_t)(yp * N + cx) * b;
    out[0] = out[1] = out[2] = out[3] = out[4] = out[5] = T(0);
    if (n > 0) {
        const T q = T(1) / (T(4) * t);
#pragma unroll
        for (int i = 0; i < 2; i++) {
            if (!does_E<TPP>(role, i)) continue;
            const uint32_t sb = i == 0 ? s_xm : s_ym;
            const uint32_t ce = kCompE + 8 * i;
            a8<T> here, back;
#pragma unroll
            for (int a = 0; a < 8; a++) {
                here.v[a] = bld(A, s, ce + a) + bld(B, s, ce + a);
                back.v[a] = bld(A, sb, ce + a) + bld(B, sb, ce + a);
            }
            // Q.(U^+ X U) = (U Q U^+).X
            const a8<T> qb = transport(vU(A, sb, i), Q);
            out[i] = q * (dot(Q, here) + dot(qb, back));
            CPIC_PHASE();
        }
        if (does_Eeta<TPP>(role)) {
            T e = 0;
#pragma unroll
            for (int a = 0; a < 8; a++) e += Q.v[a] * (bld(A, s, kCompPi + a) + bld(B, s, kCompPi + a));
            out[2] = T(0.5) * e;
        }
    } else if (does_Eeta<TPP>(role)) {
        T e = 0;
#pragma unroll
        for (int a = 0; a < 8; a++) e += Q.v[a] * bld(B, s, kCompPi + a);
        out[2] = e;
    }
    if (electric_only) return;
    CPIC_PHASE();
    if (n > 0) {
        // B_x = -(phi->_y - phi<-_y)/(2t), B_y = +(phi->_x - phi<-_x)/(2t);
        // Q.(U X U^+) = (U^+ Q U).X and Q.(U^+ X U) = (U Q U^+).X
        const T q = T(1) / (T(2) * t);
        if (does_Bt<TPP>(role, 1)) {
            T fy, by;
            { const a8<T> w = transport_adj(vU(A, s, 1), Q);    fy = dot(w, vA(A, s_yp, kCompPhi)); }
            CPIC_PHASE();
            { const a8<T> w = transport(vU(A, s_ym, 1), Q);     by = dot(w, vA(A, s_ym, kCompPhi)); }
            out[3] = -q * (fy - by);
            CPIC_PHASE();
        }
        if (does_Bt<TPP>(role, 0)) {
            T fx, bx;
            { const a8<T> w = transport_adj(vU(A, s, 0), Q);    fx = dot(w, vA(A, s_xp, kCompPhi)); }
            CPIC_PHASE();
            { const a8<T> w = transport(vU(A, s_xm, 0), Q);     bx = dot(w, vA(A, s_xm, kCompPhi)); }
            out[4] = q * (fx - bx);
            CPIC_PHASE();
        }
    }
    // B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}] (clover, all
    // counter-clockwise).  Each leaf is a product of four links; leaf k,
    // factor f is link `dir` at (x + dx, y + dy), daggered if `dg`, packed as
    // dx+1 | (dy+1) << 2 | dir << 4 | dg << 5.  The loop is kept rolled so
    // only one leaf's links are live at a time.
    //   U_12      = U_1(x) U_2(x+1) U_1(x+2)^+ U_2(x)^+
    //   U_{2,-1}  = U_2(x) U_1(x-1+2)^+ U_2(x-1)^+ U_1(x-1)
    //   U_{-1,-2} = U_1(x-1)^+ U_2(x-1-2)^+ U_1(x-1-2) U_2(x-2)
    //   U_{-2,1}  = U_2(x-2)^+ U_1(x-2) U_2(x+1-2) U_1(x)^+
    constexpr uint64_t L0 = (1 | 1 << 2 | 0 << 4 | 0 << 5) | (2 | 1 << 2 | 1 << 4 | 0 << 5) << 6 |
                            (1 | 2 << 2 | 0 << 4 | 1 << 5) << 12 | (1 | 1 << 2 | 1 << 4 | 1 << 5) << 18;
    constexpr uint64_t L1 = (1 | 1 << 2 | 1 << 4 | 0 << 5) | (0 | 2 << 2 | 0 << 4 | 1 << 5) << 6 |
                            (0 | 1 << 2 | 1 << 4 | 1 << 5) << 12 | (0 | 1 << 2 | 0 << 4 | 0 << 5) << 18;
    constexpr uint64_t L2 = (0 | 1 << 2 | 0 << 4 | 1 << 5) | (0 | 0 << 2 | 1 << 4 | 1 << 5) << 6 |
                            (0 | 0 << 2 | 0 << 4 | 0 << 5) << 12 | (1 | 0 << 2 | 1 << 4 | 0 << 5) << 18;
    constexpr uint64_t L3 = (1 | 0 << 2 | 1 << 4 | 1 << 5) | (1 | 0 << 2 | 0 << 4 | 0 << 5) << 6 |
                            (2 | 0 << 2 | 1 << 4 | 0 << 5) << 12 | (1 | 1 << 2 | 0 << 4 | 1 << 5) << 18;
    constexpr uint64_t kLeaf01 = L0 | L1 << 32, kLeaf23 = L2 | L3 << 32;
    T be = 0;
#pragma unroll 1
    for (int k = leaf_begin<TPP>(role); k < leaf_end<TPP>(role); k++) {
        const uint32_t code = (uint32_t)(((k < 2 ? kLeaf01 : kLeaf23) >> (32 * (k & 1))) & 0xFFFFFFu);
        m3<T> W;
#pragma unroll
        for (int fct = 0; fct < 4; fct++) {
            const uint32_t c = (code >> (6 * fct)) & 63u;
            const int dx = (int)(c & 3u) - 1, dy = (int)((c >> 2) & 3u) - 1, dir = (c >> 4) & 1u;
            const uint32_t so = (uint32_t)(wrap(cy + dy, N) * N + wrap(cx + dx, N)) * b;
            m3<T> L = vU(A, so, dir);
            if (c & 32u) L = adj(L);
            W = fct == 0 ? L : mul(W, L);
        }
        be += dot(Q, proj(W));
    }
    out[5] = T(-0.25) * be;
}

// particle block b of the grid -> logical block: consecutive logical blocks
// (neighbouring cells once the particles are sorted) share one XCD's L2
__device__ __forceinline__ int xcd_block(int nblocks)
{
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// TPP wavefronts per group of 64 particles: a block of 256 threads (4 waves)
// handles 256 / TPP particles; wave w works on particle group w / TPP in role
// w % TPP, so every wave follows one uniform path.  The role-0 wave owns the
// particle state: it rotates Q and publishes it in LDS; every role adds its
// field contractions into LDS; the role-0 wave then takes the Euler step.
template <typename T, int TPP>
__device__ __forceinline__ void push_body(const Fields<T>& Af, const Fields<T>& Bf, const Parts<T>& P,
                                          const PushArgs& a, const int* __restrict__ d_step, double* partials,
                                          int* err, int blk)
{
    const int n = *d_step;
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform over the event
    constexpr int PPB = 256 / TPP;                   // particles per block
    constexpr int NG = 4 / TPP;                      // particle groups (of 64) per block
    const int nblocks = (a.np + PPB - 1) / PPB;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int role = wave % TPP, grp = wave / TPP;
    const int p = blk * PPB + grp * 64 + lane;
    __shared__ T shQ[NG][8][64];
    __shared__ T shF[4][6][64];
    const int N = a.N, np = a.np;
    const uint32_t V = (uint32_t)N * N;
    const View<T> A = make_view<T>(Af.U, kRealsPerSite, V), B = make_view<T>(Bf.U, kRealsPerSite, V);
    const View<T> R = make_view<T>(P.r, kPartReals, (uint32_t)np);
    const View<int> C = make_view<int>(P.cell, 2, (uint32_t)np);
    const T dt = T(a.sc.dt), t = T(n * a.sc.dt);
    const int record_slot = is_record_step(a.sc, n) ? record_slot_of(a.sc, n) : -1;
    const bool renorm = is_reunit_step(a.sc, n);
    const bool live = p < np;
    const uint32_t po = (uint32_t)(live ? p : 0) * sizeof(T), pi = (uint32_t)(live ? p : 0) * sizeof(int);
    a8<T> Q;
    int nx = 0, ny = 0;
    T x = 0, y = 0;
    if (a.is_static) {
        nx = bld_i(C, pi, 0);
        ny = bld_i(C, pi, 1);
    } else {
        x = bld(R, po, PX_);
        y = bld(R, po, PY_);
        nx = (int)floor(x + T(0.5));
        ny = (int)floor(y + T(0.5));
        nx = nx >= N ? nx - N : nx;
        ny = ny >= N ? ny - N : ny;
    }
    if (role == 0) {
#pragma unroll
        for (int q = 0; q < 8; q++) Q.v[q] = bld(R, po, PQ0 + q);
        if (!a.is_static && live && n > a.sc.n_form) {
            int cx = bld_i(C, pi, 0), cy = bld_i(C, pi, 1);
            int d[2] = {nx - cx, ny - cy};
#pragma unroll
            for (int ax = 0; ax < 2; ax++) {
                int dd = d[ax];
                if (dd > N / 2) dd -= N;
                if (dd < -N / 2) dd += N;
                if (dd == 1) {
                    Q = rotate(vU(A, (uint32_t)(cy * N + cx) * (uint32_t)sizeof(T), ax), Q);
                } else if (dd == -1) {
                    const int cb = ax == 0 ? cy * N + wrap(cx - 1, N) : wrap(cy - 1, N) * N + cx;
                    Q = transport(vU(A, (uint32_t)cb * (uint32_t)sizeof(T), ax), Q);   // U Q U^+
                } else if (dd != 0) {
                    atomicAdd(err, 1);
                }
                if (ax == 0) cx = nx; else cy = ny;
            }
            const T deta = bld(R, po, PDETA);
            if (deta != T(0)) Q = rotate(expi(vA(A, (uint32_t)(ny * N + nx) * (uint32_t)sizeof(T), kCompPhi), deta), Q);
        }
        if (!a.is_static && renorm && live) Q = renorm_charge(Q, a.q0eig);
        if (TPP > 1) {
#pragma unroll
            for (int q = 0; q < 8; q++) shQ[grp][q][lane] = Q.v[q];
        }
    }
    if (TPP > 1) {
        __syncthreads();
        if (role != 0) {
#pragma unroll
            for (int q = 0; q < 8; q++) Q.v[q] = shQ[grp][q][lane];
        }
    }
    CPIC_PHASE();
    T f[6];
    if (live) forces_dot<T, TPP>(A, B, N, nx, ny, n, t, a.is_static != 0, Q, f, role);
    else f[0] = f[1] = f[2] = f[3] = f[4] = f[5] = T(0);
    if (TPP > 1) {
#pragma unroll
        for (int k = 0; k < 6; k++) shF[wave][k][lane] = f[k];
        __syncthreads();
        if (role == 0) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                T acc = shF[wave][k][lane];
#pragma unroll
                for (int r = 1; r < TPP; r++) acc += shF[wave + r][k][lane];
                f[k] = acc;
            }
        }
    }
    double obs[4] = {0, 0, 0, 0};
    if (role == 0 && live) {
        T px = bld(R, po, PPX), py = bld(R, po, PPY), pe = bld(R, po, PPETA);
        T eta = bld(R, po, PETA_);
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
            T xn = x + dt * v1, yn = y + dt * v2;
            if (xn >= T(N)) xn -= T(N); else if (xn < T(0)) xn += T(N);
            if (yn >= T(N)) yn -= T(N); else if (yn < T(0)) yn += T(N);
            const T deta = dt * pe / ptau;
            eta += deta;
            px = npx; py = npy; pe = npe;
            bst(R, po, PX_, xn); bst(R, po, PY_, yn); bst(R, po, PETA_, eta);
            bst(R, po, PPX, px); bst(R, po, PPY, py); bst(R, po, PPETA, pe); bst(R, po, PDETA, deta);
            bst_i(C, pi, 0, nx);
            bst_i(C, pi, 1, ny);
            if (n > a.sc.n_form || renorm) {
#pragma unroll
                for (int q = 0; q < 8; q++) bst(R, po, PQ0 + q, Q.v[q]);
            }
        }
        if (record_slot >= 0) {
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
            obs[0] = dpx * dpx + dpy * dpy - p02;
            obs[1] = pz * pz;
            obs[2] = par * par - p02;
            obs[3] = perp * perp;
        }
    }
    if (record_slot >= 0)
        block_reduce_store<4>(obs, 0u, partials + ((size_t)record_slot * nblocks + blk) * 4);
}

template <typename T, int TPP>
__global__ __launch_bounds__(256) void push_kernel(Fields<T> Af, Fields<T> Bf, Parts<T> P, PushArgs a,
                                                   const int* __restrict__ d_step, double* partials, int* err)
{
    const int nblocks = (a.np + 256 / TPP - 1) / (256 / TPP);
    const int blk = xcd_block(nblocks);
    if (blk < nblocks) push_body<T, TPP>(Af, Bf, P, a, d_step, partials, err, blk);
}

// batched events: logical block g -> (active event k, block g - blk_start[k])
__device__ __forceinline__ int find_event_p(const int* __restrict__ start, int nact, int g)
{
    int lo = 0, hi = nact;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}
template <typename T, int TPP>
__global__ __launch_bounds__(256) void batch_push_kernel(const EventDesc* __restrict__ ev, const int* __restrict__ act,
                                                         const int* __restrict__ blk_start, int nact)
{
    const int total = blk_start[nact];
    const int g = xcd_block(total);
    if (g >= total) return;
    const int k = find_event_p(blk_start, nact, g);
    const EventDesc& d = ev[act[k]];
    const int V = d.N * d.N, parity = (*d.d_step & 1) ^ d.flip;
    push_body<T, TPP>(fields_at<T>(d.f[parity], V), fields_at<T>(d.f[parity ^ 1], V),
                      Parts<T>{static_cast<T*>(d.pr), d.cell}, d.pa, d.d_step, d.partials, d.d_err, g - blk_start[k]);
}

// end of a step: on recording steps the block partials of the step's slot are
// summed (fixed order) into obs[slot]; then the step counter advances
__device__ __forceinline__ void step_end_body(const Schedule& sc, int nblocks, const double* __restrict__ partials,
                                              double* obs, int* d_step)
{
    const int n = *d_step;
    if (nblocks > 0 && is_record_step(sc, n)) {
        const int slot = record_slot_of(sc, n);
        const double* src = partials + (size_t)slot * nblocks * 4;
        double v[4] = {0, 0, 0, 0};
        for (int r = threadIdx.x; r < nblocks; r += blockDim.x)
            for (int c = 0; c < 4; c++) v[c] += src[(size_t)r * 4 + c];
        block_reduce_store<4>(v, 0u, obs + (size_t)slot * 4);
    }
    __syncthreads();
    if (threadIdx.x == 0) *d_step = n + 1;
}

// one block per active event: the step end of each event
__global__ __launch_bounds__(256) void batch_step_end_kernel(const EventDesc* __restrict__ ev, const int* __restrict__ act)
{
    const EventDesc& d = ev[act[blockIdx.x]];
    step_end_body(d.pa.sc, d.pa.np > 0 ? push_blocks_d(d.pa.np, d.pa.tpp) : 0, d.partials, d.obs, d.d_step);
}

template <typename T>
hipError_t launch_batch_push(const EventDesc* ev, const int* act, const int* blk_start, int nact, int total_blocks,
                             int tpp, hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    const dim3 g(8 * ((total_blocks + 7) / 8)), b(256);
    switch (tpp) {
    case 2: hipLaunchKernelGGL((batch_push_kernel<T, 2>), g, b, 0, st, ev, act, blk_start, nact); break;
    case 4: hipLaunchKernelGGL((batch_push_kernel<T, 4>), g, b, 0, st, ev, act, blk_start, nact); break;
    default: hipLaunchKernelGGL((batch_push_kernel<T, 1>), g, b, 0, st, ev, act, blk_start, nact);
    }
    return hipGetLastError();
}
hipError_t launch_batch_step_end(const EventDesc* ev, const int* act, int nact, hipStream_t st)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_step_end_kernel, dim3(nact), dim3(256), 0, st, ev, act);
    return hipGetLastError();
}
template hipError_t launch_batch_push<double>(const EventDesc*, const int*, const int*, int, int, int, hipStream_t);
template hipError_t launch_batch_push<float>(const EventDesc*, const int*, const int*, int, int, int, hipStream_t);

int push_blocks(int np, int tpp) { return push_blocks_d(np, tpp); }

template <typename T>
hipError_t launch_push(const Fields<T>& A, const Fields<T>& B, const Parts<T>& P, const PushArgs& a,
                       const int* d_step, double* partials, int* err, hipStream_t st)
{
    if (a.np <= 0) return hipSuccess;
    const int nb = push_blocks(a.np, a.tpp);
    const dim3 g(8 * ((nb + 7) / 8)), b(256);
    switch (a.tpp) {
    case 2: hipLaunchKernelGGL((push_kernel<T, 2>), g, b, 0, st, A, B, P, a, d_step, partials, err); break;
    case 4: hipLaunchKernelGGL((push_kernel<T, 4>), g, b, 0, st, A, B, P, a, d_step, partials, err); break;
    default: hipLaunchKernelGGL((push_kernel<T, 1>), g, b, 0, st, A, B, P, a, d_step, partials, err);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void step_end_kernel(Schedule sc, int nblocks, const double* __restrict__ partials,
                                                       double* obs, int* d_step)
{
    step_end_body(sc, nblocks, partials, obs, d_step);
}

hipError_t launch_step_end(const Schedule& sc, int nblocks, const double* partials, double* obs, int* d_step,
                           hipStream_t st)
{
    hipLaunchKernelGGL(step_end_kernel, dim3(1), dim3(256), 0, st, sc, nblocks, partials, obs, d_step);
    return hipGetLastError();
}

// out[c] = sum (or max, bit c of mask) over rows of partials[row][c]; one block,
// rows dealt to threads in a fixed pattern, then a fixed-order block reduction
template <int NC>
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double* __restrict__ partials, int nrows,
                                                          unsigned mask, double* out)
{
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = 0;
    for (int r = threadIdx.x; r < nrows; r += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; c++) {
            const double x = partials[(size_t)r * NC + c];
            v[c] = ((mask >> c) & 1) ? fmax(v[c], x) : v[c] + x;
        }
    block_reduce_store<NC>(v, mask, out);
}

hipError_t launch_reduce_rows(const double* partials, int nrows, int ncols, double* out, hipStream_t st)
{
    if (ncols == 4) {
        hipLaunchKernelGGL(reduce_rows_kernel<4>, dim3(1), dim3(256), 0, st, partials, nrows, 0u, out);
    } else if (ncols == 8) {
        // diagnostics layout: columns 1 and 6 are maxima
        hipLaunchKernelGGL(reduce_rows_kernel<8>, dim3(1), dim3(256), 0, st, partials, nrows, (1u << 1) | (1u << 6),
                           out);
    } else if (ncols == 2) {
        hipLaunchKernelGGL(reduce_rows_kernel<2>, dim3(1), dim3(256), 0, st, partials, nrows, 3u, out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// per block: max |q2 - q2_0|, max |q3 - q3_0| over the particles
template <typename T>
__global__ __launch_bounds__(256) void part_diag_kernel(Parts<T> P, int np, double q2r, double q3r, double* partials)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double v[2] = {0, 0};
    if (p < np) {
        a8<double> Q;
        for (int q = 0; q < 8; q++) Q.v[q] = P.r[(size_t)(PQ0 + q) * np + p];
        const m3<double> H = herm(Q);
        const m3<double> H2 = mul(H, H);
        double tr3 = 0;
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) tr3 += H.e[3 * i + k].re * H2.e[3 * k + i].re - H.e[3 * i + k].im * H2.e[3 * k + i].im;
        v[0] = fabs(dot(Q, Q) - q2r);
        v[1] = fabs(4.0 * tr3 - q3r);
    }
    block_reduce_store<2>(v, 3u, partials + (size_t)blockIdx.x * 2);
}
template <typename T>
hipError_t launch_part_diag(const Parts<T>& P, int np, double q2, double q3, double* partials, hipStream_t st)
{
    hipLaunchKernelGGL(part_diag_kernel<T>, dim3(push_blocks(np, 1)), dim3(256), 0, st, P, np, q2, q3, partials);
    return hipGetLastError();
}

template hipError_t launch_push<double>(const Fields<double>&, const Fields<double>&, const Parts<double>&,
                                        const PushArgs&, const int*, double*, int*, hipStream_t);
template hipError_t launch_push<float>(const Fields<float>&, const Fields<float>&, const Parts<float>&,
                                       const PushArgs&, const int*, double*, int*, hipStream_t);
template hipError_t launch_part_diag<double>(const Parts<double>&, int, double, double, double*, hipStream_t);
template hipError_t launch_part_diag<float>(const Parts<float>&, int, double, double, double*, hipStream_t);

}  // namespace cpic
