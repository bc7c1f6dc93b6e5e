// su2.hip -- the SU(2) variant of the hot path: the leapfrog of Sec. II.A,
// the Wong / CPIC push of Sec. III.B and the diagnostics, for N_c = 2.
//
// Links are unit quaternions and algebra elements 3-vectors (su2.h), so a
// site holds 20 reals instead of 68 and every product is a few dozen flops.
// The kernels read the stencil straight from global memory (one thread per
// site or particle); the structure, schedule and step-counter protocol are
// those of the SU(3) kernels.
#include "internal.h"
#include "reduce.h"
#include "su2.h"

namespace cpic {

namespace {

// consecutive logical blocks on one XCD (its L2 holds the neighbouring rows)
__device__ __forceinline__ int remap_block(int nblocks)
{
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}
__device__ __forceinline__ int wrapi(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

template <typename T> struct L2 {
    const T* U;
    int V;
    __device__ __forceinline__ q4<T> link(int i, int s) const
    {
        const T* p = U + (size_t)i * 4 * V;
        return {p[s], p[(size_t)V + s], p[2 * (size_t)V + s], p[3 * (size_t)V + s]};
    }
};
template <typename T> __device__ __forceinline__ v3<T> ld3(const T* p, int s, int V)
{
    return {{p[s], p[(size_t)V + s], p[2 * (size_t)V + s]}};
}
template <typename T> __device__ __forceinline__ void st3(T* p, int s, int V, const v3<T>& v)
{
    p[s] = v.v[0];
    p[(size_t)V + s] = v.v[1];
    p[2 * (size_t)V + s] = v.v[2];
}
template <typename T> __device__ __forceinline__ void stq(T* p, int i, int s, int V, const q4<T>& q)
{
    T* b = p + (size_t)i * 4 * V;
    b[s] = q.w;
    b[(size_t)V + s] = q.x;
    b[2 * (size_t)V + s] = q.y;
    b[3 * (size_t)V + s] = q.z;
}

struct Nb2 {
    int s, xp, xm, yp, ym, xpym, xmyp, xmym;
};
__device__ __forceinline__ Nb2 nbrs(int x, int y, int N)
{
    const int xp = wrapi(x + 1, N), xm = wrapi(x - 1, N), yp = wrapi(y + 1, N), ym = wrapi(y - 1, N);
    return {y * N + x, y * N + xp, y * N + xm, yp * N + x, ym * N + x, ym * N + xp, yp * N + xm, ym * N + xm};
}

// Kick forces at a site (the SU(3) kick_forces for N_c = 2):
//   F_E[i] = -t (Proj U_ij + Proj U_{i,-j}) + (1/t) i[phi->_i, phi]
//   F_pi   = (1/t) sum_i (phi->_i + phi<-_i - 2 phi)
// retr = Re Tr U_12 / 1 (w of the quaternion times 2) and grad2 =
// sum_i Tr(phi->_i - phi)^2 for the energy diagnostics.
template <typename T>
__device__ void kick2(const L2<T>& L, const T* phi, int V, const Nb2& c, T t, T inv_t, const v3<T>& PHI, v3<T>& F1,
                      v3<T>& F2, v3<T>& Fpi, T* retr = nullptr, T* grad2 = nullptr)
{
    const q4<T> u1 = L.link(0, c.s), u2 = L.link(1, c.s);
    // U_12(x) = U_1(x) U_2(x+1) U_1(x+2)^+ U_2(x)^+, U_21 its adjoint
    const q4<T> p12 = qmul(qmul(u1, L.link(1, c.xp)), qmul(qadj(L.link(0, c.yp)), qadj(u2)));
    // U_{1,-2}(x) = U_1(x) U_2(x+1-2)^+ U_1(x-2)^+ U_2(x-2)
    const q4<T> p1m2 = qmul(qmul(u1, qadj(L.link(1, c.xpym))), qmul(qadj(L.link(0, c.ym)), L.link(1, c.ym)));
    // U_21(x) = U_2(x) U_1(x+2) U_2(x+1)^+ U_1(x)^+
    const q4<T> p21 = qmul(qmul(u2, L.link(0, c.yp)), qmul(qadj(L.link(1, c.xp)), qadj(u1)));
    // U_{2,-1}(x) = U_2(x) U_1(x+2-1)^+ U_2(x-1)^+ U_1(x-1)
    const q4<T> p2m1 = qmul(qmul(u2, qadj(L.link(0, c.xmyp))), qmul(qadj(L.link(1, c.xm)), L.link(0, c.xm)));
    const v3<T> fw1 = qtransport(u1, ld3(phi, c.xp, V)), fw2 = qtransport(u2, ld3(phi, c.yp, V));
    const v3<T> bw1 = qtransport(L.link(0, c.xm), ld3(phi, c.xm, V), true);
    const v3<T> bw2 = qtransport(L.link(1, c.ym), ld3(phi, c.ym, V), true);
    const v3<T> P12 = qproj(p12), P1m2 = qproj(p1m2), P21 = qproj(p21), P2m1 = qproj(p2m1);
    const v3<T> c1 = vicomm(fw1, PHI), c2 = vicomm(fw2, PHI);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        F1.v[a] = -t * (P12.v[a] + P1m2.v[a]) + inv_t * c1.v[a];
        F2.v[a] = -t * (P21.v[a] + P2m1.v[a]) + inv_t * c2.v[a];
        Fpi.v[a] = inv_t * (fw1.v[a] + bw1.v[a] + fw2.v[a] + bw2.v[a] - T(4) * PHI.v[a]);
    }
    if (retr) *retr = T(2) * p12.w;
    if (grad2) {
        T g = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const T d1 = fw1.v[a] - PHI.v[a], d2 = fw2.v[a] - PHI.v[a];
            g += d1 * d1 + d2 * d2;
        }
        *grad2 = T(0.5) * g;  // Tr (X.sigma/2)^2 = |X|^2 / 2
    }
}

}  // namespace

// ------------------------------------------------------------------ field update
// one thread per site: kick at t_n (skipped at n = 0), drift at t_{n+1/2};
// FP32 runs renormalise the link quaternions on reunitarisation steps
template <typename T>
__global__ __launch_bounds__(256) void su2_field_kernel(Fields2<T> in, Fields2<T> out, int N, Schedule sc, int* d_step)
{
    const int V = N * N, nb = (V + 255) / 256;
    const int blk = remap_block(nb);
    if (blk >= nb) return;
    const int n = d_step[0];
    if (blk == 0 && threadIdx.x == 0) d_step[1] = n;
    const int s = blk * 256 + (int)threadIdx.x;
    if (s >= V) return;
    const Nb2 c = nbrs(s % N, s / N, N);
    const L2<T> L{in.U, V};
    const T dt = T(sc.dt), t = T(n * sc.dt), th = T((n + 0.5) * sc.dt);
    const v3<T> PHI = ld3(in.phi, s, V);
    v3<T> E1 = ld3(in.E, s, V), E2 = ld3(in.E + 3 * (size_t)V, s, V), PI = ld3(in.pi, s, V);
    if (n > 0) {
        v3<T> F1, F2, Fpi;
        kick2(L, in.phi, V, c, t, T(1) / t, PHI, F1, F2, Fpi);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            E1.v[a] += dt * F1.v[a];
            E2.v[a] += dt * F2.v[a];
            PI.v[a] += dt * Fpi.v[a];
        }
    }
    const T e = dt / th;
    q4<T> u1 = qmul(qexpi(E1, e), L.link(0, s)), u2 = qmul(qexpi(E2, e), L.link(1, s));
    if constexpr (sizeof(T) == 4)
        if (is_reunit_step(sc, n)) {
            u1 = qnormalize(u1);
            u2 = qnormalize(u2);
        }
    v3<T> ph;
#pragma unroll
    for (int a = 0; a < 3; a++) ph.v[a] = PHI.v[a] + dt * th * PI.v[a];
    stq(out.U, 0, s, V, u1);
    stq(out.U, 1, s, V, u2);
    st3(out.phi, s, V, ph);
    st3(out.E, s, V, E1);
    st3(out.E + 3 * (size_t)V, s, V, E2);
    st3(out.pi, s, V, PI);
}

template <typename T>
hipError_t launch_su2_field(const Fields2<T>& in, const Fields2<T>& out, int N, const Schedule& sc, int* d_step,
                            hipStream_t st, const KTimer& tm)
{
    const int nb = (N * N + 255) / 256;
    klaunch(tm, su2_field_kernel<T>, dim3(8 * ((nb + 7) / 8)), dim3(256), st, in, out, N, sc, d_step);
    return hipGetLastError();
}

// ------------------------------------------------------------------ particle push
// The SU(3) push for N_c = 2: colour rotation for the move n-1 -> n with the
// crossed links and the rapidity Wilson line, the fields of Sec. III.B at the
// nearest grid point, one Euler step; on recording steps each group of 64
// writes its four double-precision sums.  Four wavefronts share a group of 64
// particles: the owner (wave 0) rotates Q while three helpers evaluate the six
// field vectors, two each, into LDS (wave 1: E_x and B_y, both through the x
// links; wave 2: E_y and B_x; wave 3: E_eta and B_eta); after one barrier the
// owner contracts them with Q and takes the step.  One thread per particle
// would leave about one and a half wavefronts per SIMD at 1e5 particles, too
// few to cover the chains of dependent gathers.
template <typename T>
__global__ __launch_bounds__(256) void su2_push_kernel(Fields2<T> Af, Fields2<T> Bf, Parts<T> P, PushArgs a,
                                                       int* d_step, double* partials, int* err)
{
    const int np = a.np, N = a.N, V = N * N;
    const int nb = (np + 63) / 64;
    const int blk = remap_block(nb);
    if (blk >= nb) return;
    const int n = d_step[1];
    if (blk == 0 && threadIdx.x == 0) d_step[0] = n + 1;
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform over the grid
    __shared__ T shF[3][6][64];
    const int lane = (int)threadIdx.x & 63, role = (int)threadIdx.x >> 6;
    const int p = blk * 64 + lane;
    const bool live = p < np;
    const int q = live ? p : 0;
    auto R = [&](int col) -> T& { return P.r[(size_t)col * np + q]; };
    const L2<T> L{Af.U, V};
    const T dt = T(a.sc.dt), t = T(n * a.sc.dt);
    const int record_slot = is_record_step(a.sc, n) ? record_slot_of(a.sc, n) : -1;
    // the nearest grid point (every wave)
    int nx, ny;
    T x = 0, y = 0;
    if (a.is_static) {
        nx = P.cell[q];
        ny = P.cell[np + q];
    } else {
        x = R(PX_);
        y = R(PY_);
        nx = (int)floor(x + T(0.5));
        ny = (int)floor(y + T(0.5));
        nx = nx >= N ? nx - N : nx;
        ny = ny >= N ? ny - N : ny;
    }
    const Nb2 c = nbrs(nx, ny, N);
    v3<T> Q = {{0, 0, 0}};
    if (role == 0) {
        if (live) {
            Q = {{R(PQ0), R(PQ0 + 1), R(PQ0 + 2)}};
            if (!a.is_static && n > a.sc.n_form) {
                int cx = P.cell[q], cy = P.cell[np + q];
                const int d[2] = {nx - cx, ny - cy};
#pragma unroll
                for (int ax = 0; ax < 2; ax++) {
                    int dd = d[ax];
                    if (dd > N / 2) dd -= N;
                    if (dd < -N / 2) dd += N;
                    if (dd == 1) {
                        Q = qtransport(L.link(ax, cy * N + cx), Q, true);                 // U^+ Q U
                    } else if (dd == -1) {
                        const int cb = ax == 0 ? cy * N + wrapi(cx - 1, N) : wrapi(cy - 1, N) * N + cx;
                        Q = qtransport(L.link(ax, cb), Q);                                // U Q U^+
                    } else if (dd != 0) {
                        atomicAdd(err, 1);
                    }
                    if (ax == 0) cx = nx; else cy = ny;
                }
                const T deta = R(PDETA);
                if (deta != T(0)) Q = qtransport(qexpi(ld3(Af.phi, ny * N + nx, V), deta), Q, true);
            }
        }
    } else {
        // helper: field vectors fa (electric) and fb (magnetic) of its direction
        v3<T> fa = {{0, 0, 0}}, fb = {{0, 0, 0}};
        if (live) {
            const bool mag = !a.is_static;
            if (role < 3) {
                const int i = role - 1;
                if (n > 0) {
                    // E_i = (1/4t) [S_i(c) + U_i(c-i)^+ S_i(c-i) U_i(c-i)], S_i = E_i(n-1/2) + E_i(n+1/2)
                    const T q4t = T(1) / (T(4) * t);
                    const int back = i == 0 ? c.xm : c.ym;
                    const size_t o = (size_t)i * 3 * V;
                    v3<T> here = ld3(Af.E + o, c.s, V), bk = ld3(Af.E + o, back, V);
                    const v3<T> hn = ld3(Bf.E + o, c.s, V), bn = ld3(Bf.E + o, back, V);
#pragma unroll
                    for (int a2 = 0; a2 < 3; a2++) {
                        here.v[a2] += hn.v[a2];
                        bk.v[a2] += bn.v[a2];
                    }
                    const v3<T> tb = qtransport(L.link(i, back), bk, true);
#pragma unroll
                    for (int a2 = 0; a2 < 3; a2++) fa.v[a2] = q4t * (here.v[a2] + tb.v[a2]);
                    if (mag) {
                        // B_y = +(1/2t) D_x (wave 1), B_x = -(1/2t) D_y (wave 2), D_i = phi->_i - phi<-_i
                        const T h = (i == 0 ? T(1) : T(-1)) / (T(2) * t);
                        const v3<T> fw = qtransport(L.link(i, c.s), ld3(Af.phi, i == 0 ? c.xp : c.yp, V));
                        const v3<T> bw = qtransport(L.link(i, back), ld3(Af.phi, back, V), true);
#pragma unroll
                        for (int a2 = 0; a2 < 3; a2++) fb.v[a2] = h * (fw.v[a2] - bw.v[a2]);
                    }
                }
            } else {
                if (n > 0) {
                    const v3<T> po = ld3(Af.pi, c.s, V), pn = ld3(Bf.pi, c.s, V);
#pragma unroll
                    for (int a2 = 0; a2 < 3; a2++) fa.v[a2] = T(0.5) * (po.v[a2] + pn.v[a2]);
                } else {
                    fa = ld3(Bf.pi, c.s, V);
                }
                if (mag) {
                    // B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}] at c
                    const q4<T> u1 = L.link(0, c.s), u2 = L.link(1, c.s);
                    const q4<T> c12 = qmul(qmul(u1, L.link(1, c.xp)), qmul(qadj(L.link(0, c.yp)), qadj(u2)));
                    const q4<T> c2m1 =
                        qmul(qmul(u2, qadj(L.link(0, c.xmyp))), qmul(qadj(L.link(1, c.xm)), L.link(0, c.xm)));
                    const q4<T> cm1m2 = qmul(qmul(qadj(L.link(0, c.xm)), qadj(L.link(1, c.xmym))),
                                             qmul(L.link(0, c.xmym), L.link(1, c.ym)));
                    const q4<T> cm21 =
                        qmul(qmul(qadj(L.link(1, c.ym)), L.link(0, c.ym)), qmul(L.link(1, c.xpym), qadj(u1)));
                    const v3<T> pb = qproj(qadd(qadd(c12, c2m1), qadd(cm1m2, cm21)));
#pragma unroll
                    for (int a2 = 0; a2 < 3; a2++) fb.v[a2] = T(-0.25) * pb.v[a2];
                }
            }
        }
#pragma unroll
        for (int a2 = 0; a2 < 3; a2++) {
            shF[role - 1][a2][lane] = fa.v[a2];
            shF[role - 1][3 + a2][lane] = fb.v[a2];
        }
    }
    __syncthreads();
    if (role != 0) return;
    double obs[4] = {0, 0, 0, 0};
    if (live) {
        // f: E_x, E_y, E_eta, B_x, B_y, B_eta
        v3<T> f[6];
#pragma unroll
        for (int a2 = 0; a2 < 3; a2++) {
            f[0].v[a2] = shF[0][a2][lane];
            f[4].v[a2] = shF[0][3 + a2][lane];
            f[1].v[a2] = shF[1][a2][lane];
            f[3].v[a2] = shF[1][3 + a2][lane];
            f[2].v[a2] = shF[2][a2][lane];
            f[5].v[a2] = shF[2][3 + a2][lane];
        }
        T px = R(PPX), py = R(PPY), pe = R(PPETA), eta = R(PETA_);
        const T e1 = vdot(Q, f[0]), e2 = vdot(Q, f[1]), ee = vdot(Q, f[2]);
        if (a.is_static) {
            px += dt * e1;
            py += dt * e2;
            pe += dt * ee;
            R(PPX) = px; R(PPY) = py; R(PPETA) = pe;
        } else {
            const T b1 = vdot(Q, f[3]), b2 = vdot(Q, f[4]), be = vdot(Q, f[5]);
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
            R(PX_) = xn; R(PY_) = yn; R(PETA_) = eta;
            R(PPX) = px; R(PPY) = py; R(PPETA) = pe; R(PDETA) = deta;
            P.cell[q] = nx;
            P.cell[np + q] = ny;
            R(PQ0) = Q.v[0]; R(PQ0 + 1) = Q.v[1]; R(PQ0 + 2) = Q.v[2];
        }
        if (record_slot >= 0) {
            const double dpx = px, dpy = py, tn = (double)(n + 1) * a.sc.dt;
            double pz;
            if (a.is_static) {
                pz = pe;
            } else {
                const double dpe = pe, et = eta;
                const double ptn = sqrt(dpx * dpx + dpy * dpy + (tn * dpe) * (tn * dpe) + a.mhat * a.mhat);
                pz = ptn * sinh(et) + tn * dpe * cosh(et);
            }
            const double ux0 = R(PUX0), uy0 = R(PUY0), pt0 = R(PPT0);
            const double par = dpx * ux0 + dpy * uy0, perp = -dpx * uy0 + dpy * ux0;
            obs[0] = dpx * dpx + dpy * dpy - pt0 * pt0;
            obs[1] = pz * pz;
            obs[2] = par * par - pt0 * pt0;
            obs[3] = perp * perp;
        }
    }
    if (record_slot >= 0) {
        const int ngroups = (np + 63) / 64;
        double* dst = partials + ((size_t)record_slot * ngroups + blk) * 4;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double v = wave_sum(obs[k]);
            if (lane == 0) dst[k] = v;
        }
    }
}

template <typename T>
hipError_t launch_su2_push(const Fields2<T>& A, const Fields2<T>& B, const Parts<T>& P, const PushArgs& a,
                           int* d_step, double* partials, int* err, hipStream_t st, const KTimer& tm)
{
    if (a.np <= 0) return hipSuccess;
    const int nb = (a.np + 63) / 64;
    klaunch(tm, su2_push_kernel<T>, dim3(8 * ((nb + 7) / 8)), dim3(256), st, A, B, P, a, d_step, partials, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ diagnostics
// per block: sum |G|^2, max |G|, the four energy terms (momenta averaged to
// integer time with half kicks), max and sum of squares of |U|^2 - 1 per link
template <typename T>
__global__ __launch_bounds__(256) void su2_diag_kernel(Fields2<T> f, int N, T t, T inv_t, T half_dt, int n,
                                                       double* partials)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (s < V) {
        const Nb2 c = nbrs(s % N, s / N, N);
        const L2<T> L{f.U, V};
        const v3<T> PHI = ld3(f.phi, s, V), PI = ld3(f.pi, s, V);
        const v3<T> E1 = ld3(f.E, s, V), E2 = ld3(f.E + 3 * (size_t)V, s, V);
        const v3<T> g1 = qtransport(L.link(0, c.xm), ld3(f.E, c.xm, V), true);
        const v3<T> g2 = qtransport(L.link(1, c.ym), ld3(f.E + 3 * (size_t)V, c.ym, V), true);
        const v3<T> gc = vicomm(PHI, PI);
        double G2 = 0;
        for (int a = 0; a < 3; a++) {
            const double g = (double)E1.v[a] - g1.v[a] + E2.v[a] - g2.v[a] + gc.v[a];
            G2 += g * g;
        }
        v[0] = G2;
        v[1] = sqrt(G2);
        v3<T> F1, F2, Fpi;
        T retr = 0, grad2 = 0;
        kick2(L, f.phi, V, c, t, inv_t, PHI, F1, F2, Fpi, &retr, &grad2);
        const T h = n > 0 ? half_dt : T(0);
        double e2 = 0, p2 = 0;
        for (int a = 0; a < 3; a++) {
            const double ea = E1.v[a] + h * F1.v[a], eb = E2.v[a] + h * F2.v[a], pa = PI.v[a] + h * Fpi.v[a];
            e2 += 0.5 * (ea * ea + eb * eb);
            p2 += 0.5 * pa * pa;
        }
        v[2] = (double)inv_t * e2;
        v[3] = (double)t * p2;
        v[4] = 2.0 * (double)t * (2.0 - (double)retr);
        v[5] = (double)inv_t * (double)grad2;
        double umax = 0, usq = 0;
        for (int i = 0; i < 2; i++) {
            const q4<T> u = L.link(i, s);
            const double d = fabs((double)u.w * u.w + (double)u.x * u.x + (double)u.y * u.y + (double)u.z * u.z - 1.0);
            umax = fmax(umax, d);
            usq += d * d;
        }
        v[6] = umax;
        v[7] = usq;
    }
    block_reduce_store<8>(v, (1u << 1) | (1u << 6), partials + (size_t)blockIdx.x * 8);
}

template <typename T>
hipError_t launch_su2_diag(const Fields2<T>& f, int N, double dt, int n, double* partials, int nblk_cap,
                           int* nblk_out, hipStream_t st)
{
    const int V = N * N, nblk = (V + 255) / 256;
    if (nblk > nblk_cap) return hipErrorInvalidValue;
    *nblk_out = nblk;
    const double t = n * dt;
    hipLaunchKernelGGL(su2_diag_kernel<T>, dim3(nblk), dim3(256), 0, st, f, N, T(t), T(n > 0 ? 1.0 / t : 0.0),
                       T(0.5 * dt), n, partials);
    return hipGetLastError();
}

#define CPIC_SU2_INST(T)                                                                                             \
    template hipError_t launch_su2_field<T>(const Fields2<T>&, const Fields2<T>&, int, const Schedule&, int*,      \
                                            hipStream_t, const KTimer&);                                           \
    template hipError_t launch_su2_push<T>(const Fields2<T>&, const Fields2<T>&, const Parts<T>&, const PushArgs&, \
                                           int*, double*, int*, hipStream_t, const KTimer&);                        \
    template hipError_t launch_su2_diag<T>(const Fields2<T>&, int, double, int, double*, int, int*, hipStream_t);
CPIC_SU2_INST(double)
CPIC_SU2_INST(float)
#undef CPIC_SU2_INST

}  // namespace cpic
