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

namespace cpic {

template <typename T> __device__ __forceinline__ m3<T> gU(const T* __restrict__ U, int i, int s, int V)
{
    const T* p = U + (size_t)i * 18 * V + s;
    m3<T> m;
#pragma unroll
    for (int c = 0; c < 9; c++) m.e[c] = {p[(size_t)(2 * c) * V], p[(size_t)(2 * c + 1) * V]};
    return m;
}
template <typename T> __device__ __forceinline__ a8<T> gA(const T* __restrict__ p, int s, int V)
{
    a8<T> r;
#pragma unroll
    for (int a = 0; a < 8; a++) r.v[a] = p[(size_t)a * V + s];
    return r;
}
__device__ __forceinline__ int wrap(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

// components of A^+ Q A
template <typename T> __device__ __forceinline__ a8<T> rotate(const m3<T>& A, const a8<T>& Q) { return transport_adj(A, Q); }

// Replace the spectrum of Q by the sorted spectrum of Q0 (keeps the
// eigenvectors): restores both classical Casimirs exactly.
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
    T lam[3];
    for (int k = 0; k < 3; k++) lam[k] = T(2) * r * cos(th - T(2.0943951023931954923) * k);
    // sort ascending (lam[0] is the largest root, lam[1] the smallest)
    int ord[3] = {1, 2, 0};
    if (lam[ord[1]] < lam[ord[0]]) { int q = ord[0]; ord[0] = ord[1]; ord[1] = q; }
    cx<T> v[3][3];
    for (int k = 0; k < 2; k++) {
        const T l = lam[ord[k]];
        cx<T> m[9];
        for (int q = 0; q < 9; q++) m[q] = H.e[q];
        m[0].re -= l; m[4].re -= l; m[8].re -= l;
        // null vector: the largest cross product of two rows
        T best = -1;
        for (int pr = 0; pr < 3; pr++) {
            const int ra = pr == 2 ? 1 : 0, rb = pr == 0 ? 1 : 2;
            cx<T> c[3];
            for (int j = 0; j < 3; j++) {
                const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                const cx<T> u = cmul(m[3 * ra + j1], m[3 * rb + j2]), w = cmul(m[3 * ra + j2], m[3 * rb + j1]);
                c[j] = {u.re - w.re, u.im - w.im};
            }
            const T nn = c[0].re * c[0].re + c[0].im * c[0].im + c[1].re * c[1].re + c[1].im * c[1].im +
                         c[2].re * c[2].re + c[2].im * c[2].im;
            if (nn > best) {
                best = nn;
                for (int j = 0; j < 3; j++) v[k][j] = c[j];
            }
        }
        if (k == 1) {  // orthogonalise against the first vector
            cx<T> ip = {0, 0};
            for (int j = 0; j < 3; j++) { cx<T> q = ccmul(v[0][j], v[1][j]); ip.re += q.re; ip.im += q.im; }
            for (int j = 0; j < 3; j++) { cx<T> q = cmul(ip, v[0][j]); v[1][j].re -= q.re; v[1][j].im -= q.im; }
        }
        T nn = 0;
        for (int j = 0; j < 3; j++) nn += v[k][j].re * v[k][j].re + v[k][j].im * v[k][j].im;
        const T inv = T(1) / sqrt(nn);
        for (int j = 0; j < 3; j++) { v[k][j].re *= inv; v[k][j].im *= inv; }
    }
    for (int j = 0; j < 3; j++) {  // v2 = conj(v0 x v1)
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const cx<T> u = cmul(v[0][j1], v[1][j2]), w = cmul(v[0][j2], v[1][j1]);
        v[2][j] = {u.re - w.re, -(u.im - w.im)};
    }
    // Q' = sum_k eig0_k v_k v_k^+
    cx<T> M[9];
    for (int q = 0; q < 9; q++) M[q] = {0, 0};
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                const cx<T> q = cmulc(v[k][i], v[k][j]);
                M[3 * i + j].re += T(eig0[k]) * q.re;
                M[3 * i + j].im += T(eig0[k]) * q.im;
            }
    return herm_comp(M[0], M[4], M[8], M[1], M[2], M[5]);
}

// colour fields at site c, time t_n (Sec. III.B interpolations), hat units:
// F[0..2] = E_x, E_y, E_eta; F[3..5] = B_x, B_y, B_eta
template <typename T>
__device__ __forceinline__ void fields_at(const Fields<T>& A, const T* __restrict__ En, const T* __restrict__ pin,
                                          int N, int cx, int cy, int n, T t, bool electric_only, a8<T>* F)
{
    const int V = N * N;
    const int xm = wrap(cx - 1, N), xp = wrap(cx + 1, N), ym = wrap(cy - 1, N), yp = wrap(cy + 1, N);
    const int s = cy * N + cx;
    const int s_xm = cy * N + xm, s_xp = cy * N + xp, s_ym = ym * N + cx, s_yp = yp * N + cx;
    if (n > 0) {
        const T q = T(1) / (T(4) * t);
        for (int i = 0; i < 2; i++) {
            const int sb = i == 0 ? s_xm : s_ym;
            const T* Eo = A.E + (size_t)i * 8 * V;
            const T* Enw = En + (size_t)i * 8 * V;
            a8<T> here, back;
#pragma unroll
            for (int a = 0; a < 8; a++) {
                here.v[a] = Eo[(size_t)a * V + s] + Enw[(size_t)a * V + s];
                back.v[a] = Eo[(size_t)a * V + sb] + Enw[(size_t)a * V + sb];
            }
            const a8<T> tb = transport_adj(gU(A.U, i, sb, V), back);
#pragma unroll
            for (int a = 0; a < 8; a++) F[i].v[a] = q * (here.v[a] + tb.v[a]);
        }
#pragma unroll
        for (int a = 0; a < 8; a++) F[2].v[a] = T(0.5) * (A.pi[(size_t)a * V + s] + pin[(size_t)a * V + s]);
    } else {
        F[0] = azero<T>();
        F[1] = azero<T>();
#pragma unroll
        for (int a = 0; a < 8; a++) F[2].v[a] = pin[(size_t)a * V + s];
    }
    if (electric_only) return;
    if (n > 0) {
        const T q = T(1) / (T(2) * t);
        const m3<T> U1 = gU(A.U, 0, s, V), U2 = gU(A.U, 1, s, V);
        const a8<T> f2 = transport(U2, gA(A.phi, s_yp, V));
        const a8<T> b2 = transport_adj(gU(A.U, 1, s_ym, V), gA(A.phi, s_ym, V));
        const a8<T> f1 = transport(U1, gA(A.phi, s_xp, V));
        const a8<T> b1 = transport_adj(gU(A.U, 0, s_xm, V), gA(A.phi, s_xm, V));
#pragma unroll
        for (int a = 0; a < 8; a++) {
            F[3].v[a] = -q * (f2.v[a] - b2.v[a]);
            F[4].v[a] = q * (f1.v[a] - b1.v[a]);
        }
    } else {
        F[3] = azero<T>();
        F[4] = azero<T>();
    }
    // B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}] (clover, all counter-clockwise)
    const int s_xmym = ym * N + xm, s_xmyp = yp * N + xm, s_xpym = ym * N + xp;
    a8<T> acc;
    {
        const m3<T> P = mul_adj(mul(gU(A.U, 0, s, V), gU(A.U, 1, s_xp, V)), mul(gU(A.U, 1, s, V), gU(A.U, 0, s_yp, V)));
        acc = proj(P);
    }
    {   // U_2(x) U_1(x-1+2)^+ U_2(x-1)^+ U_1(x-1)
        const m3<T> P = mul(mul_adj(gU(A.U, 1, s, V), gU(A.U, 0, s_xmyp, V)),
                            adj_mul(gU(A.U, 1, s_xm, V), gU(A.U, 0, s_xm, V)));
        axpy(acc, T(1), proj(P));
    }
    {   // U_1(x-1)^+ U_2(x-1-2)^+ U_1(x-1-2) U_2(x-2)
        const m3<T> P = mul(adj_mul(gU(A.U, 0, s_xm, V), adj(gU(A.U, 1, s_xmym, V))),
                            mul(gU(A.U, 0, s_xmym, V), gU(A.U, 1, s_ym, V)));
        axpy(acc, T(1), proj(P));
    }
    {   // U_2(x-2)^+ U_1(x-2) U_2(x+1-2) U_1(x)^+
        const m3<T> P = mul_adj(mul(adj_mul(gU(A.U, 1, s_ym, V), gU(A.U, 0, s_ym, V)), gU(A.U, 1, s_xpym, V)),
                                gU(A.U, 0, s, V));
        axpy(acc, T(1), proj(P));
    }
#pragma unroll
    for (int a = 0; a < 8; a++) F[5].v[a] = T(-0.25) * acc.v[a];
}

template <typename T>
__global__ __launch_bounds__(256) void push_kernel(Fields<T> A, const T* __restrict__ En, const T* __restrict__ pin,
                                                   Parts<T> P, PushArgs a, const int* __restrict__ d_step,
                                                   double* partials, int* err)
{
    const int n = *d_step;
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform over the grid
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N, np = a.np;
    const T dt = T(a.sc.dt), t = T(n * a.sc.dt);
    const int record_slot = is_record_step(a.sc, n) ? record_slot_of(a.sc, n) : -1;
    const bool renorm = is_reunit_step(a.sc, n);
    double obs[4] = {0, 0, 0, 0};
    if (p < np) {
        T* r = P.r;
        auto col = [&](int c) -> T& { return r[(size_t)c * np + p]; };
        a8<T> Q;
#pragma unroll
        for (int q = 0; q < 8; q++) Q.v[q] = col(PQ0 + q);
        const T ux0 = col(PUX0), uy0 = col(PUY0), pt0 = col(PPT0);
        T px = col(PPX), py = col(PPY), pe = col(PPETA);
        T eta = col(PETA_);
        a8<T> F[6];
        if (a.is_static) {
            const int cx = P.cell[p], cy = P.cell[np + p];
            fields_at(A, En, pin, N, cx, cy, n, t, true, F);
            px += dt * dot(Q, F[0]);
            py += dt * dot(Q, F[1]);
            pe += dt * dot(Q, F[2]);  // p^z of the static branch
            col(PPX) = px; col(PPY) = py; col(PPETA) = pe;
        } else {
            const T x = col(PX_), y = col(PY_);
            int nx = (int)floor(x + T(0.5)), ny = (int)floor(y + T(0.5));
            nx = nx >= N ? nx - N : nx;
            ny = ny >= N ? ny - N : ny;
            if (n > a.sc.n_form) {
                int cx = P.cell[p], cy = P.cell[np + p];
                const int V = N * N;
                int d[2] = {nx - cx, ny - cy};
                for (int ax = 0; ax < 2; ax++) {
                    int dd = d[ax];
                    if (dd > N / 2) dd -= N;
                    if (dd < -N / 2) dd += N;
                    const int c = cy * N + cx;
                    if (dd == 1) {
                        Q = rotate(gU(A.U, ax, c, V), Q);
                    } else if (dd == -1) {
                        const int cb = ax == 0 ? cy * N + wrap(cx - 1, N) : wrap(cy - 1, N) * N + cx;
                        Q = rotate(adj(gU(A.U, ax, cb, V)), Q);
                    } else if (dd != 0) {
                        atomicAdd(err, 1);
                    }
                    if (ax == 0) cx = nx; else cy = ny;
                }
                const T deta = col(PDETA);
                if (deta != T(0)) Q = rotate(expi(gA(A.phi, ny * N + nx, V), deta), Q);
            }
            if (renorm) Q = renorm_charge(Q, a.q0eig);
            fields_at(A, En, pin, N, nx, ny, n, t, false, F);
            const T e1 = dot(Q, F[0]), e2 = dot(Q, F[1]), ee = dot(Q, F[2]);
            const T b1 = dot(Q, F[3]), b2 = dot(Q, F[4]), be = dot(Q, F[5]);
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
            col(PX_) = xn; col(PY_) = yn; col(PETA_) = eta;
            col(PPX) = px; col(PPY) = py; col(PPETA) = pe; col(PDETA) = deta;
            P.cell[p] = nx;
            P.cell[np + p] = ny;
        }
        if (n > a.sc.n_form || renorm) {
#pragma unroll
            for (int q = 0; q < 8; q++) col(PQ0 + q) = Q.v[q];
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
        block_reduce_store<4>(obs, 0u, partials + ((size_t)record_slot * gridDim.x + blockIdx.x) * 4);
}

int push_blocks(int np) { return (np + 255) / 256; }

template <typename T>
hipError_t launch_push(const Fields<T>& A, const T* E_new, const T* pi_new, const Parts<T>& P, const PushArgs& a,
                       const int* d_step, double* partials, int* err, hipStream_t st)
{
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(push_kernel<T>, dim3(push_blocks(a.np)), dim3(256), 0, st, A, E_new, pi_new, P, a, d_step,
                       partials, err);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void step_end_kernel(Schedule sc, int nblocks, const double* __restrict__ partials,
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
    hipLaunchKernelGGL(part_diag_kernel<T>, dim3(push_blocks(np)), dim3(256), 0, st, P, np, q2, q3, partials);
    return hipGetLastError();
}

template hipError_t launch_push<double>(const Fields<double>&, const double*, const double*, const Parts<double>&,
                                        const PushArgs&, const int*, double*, int*, hipStream_t);
template hipError_t launch_push<float>(const Fields<float>&, const float*, const float*, const Parts<float>&,
                                       const PushArgs&, const int*, double*, int*, hipStream_t);
template hipError_t launch_part_diag<double>(const Parts<double>&, int, double, double, double*, hipStream_t);
template hipError_t launch_part_diag<float>(const Parts<float>&, int, double, double, double*, hipStream_t);

}  // namespace cpic
