// ic.hip -- MV-model initial condition on the GPU (Sec. II, II.A) and the
// test-particle initial conditions (Sec. III.B, IV.B).  Always double
// precision; a float run converts the finished state.
//
//   charges   Gaussian colour charges per sheet from Philox4x64-10
//   Poisson   2-D FFT (rows in LDS, mixed radix 2/3/4 Stockham) -> multiply by
//             1/(khat^2 + m^2) with the zero mode and the modes above the UV
//             cut removed -> inverse FFT
//   Wilson    V^+(x) <- V^+(x) exp(-i alpha_n(x)), sheets in order
//   links     U^X_i(x) = V(x) V(x+i)^+, then the tau = 0 Glasma links from the
//             lattice initial condition, solved per link by Newton's method
//   pi(0)     from U, U^A, U^B
#include <vector>

#include "internal.h"
#include "philox.h"
#include "su2.h"
#include "su3.h"

namespace cpic {

using d2 = double2;

// ------------------------------------------------------------------ charges
// out[(sheet*pairs + pair)*V + s] = (rho^{2 pair}, rho^{2 pair + 1}) for the
// sheet index sheet0 + sheet of nucleus `nucleus`; stream key (seed,
// 1 + nucleus), counter (s, sheet, block, 0), block b holding colours
// 4b .. 4b+3.  pairs = 4 for SU(3) (colours 0..7), 2 for SU(2) (colours 0..2
// and an unused fourth).
__global__ void charges_kernel(d2* out, int V, uint64_t seed, int nucleus, int sheet0, double sigma, int pairs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int sh = blockIdx.y;
    if (s >= V) return;
    double z[8];
    for (int b = 0; b < 2; b++) {
        if (2 * b >= pairs) break;
        const u64x4 r = philox4x64((uint64_t)s, (uint64_t)(sheet0 + sh), (uint64_t)b, 0, seed, 1 + (uint64_t)nucleus);
        box_muller(r.v[0], r.v[1], z[4 * b], z[4 * b + 1]);
        box_muller(r.v[2], r.v[3], z[4 * b + 2], z[4 * b + 3]);
    }
    for (int p = 0; p < pairs; p++)
        out[((size_t)sh * pairs + p) * V + s] = make_double2(sigma * z[2 * p], sigma * z[2 * p + 1]);
}

// ------------------------------------------------------------------ FFT
struct Radices {
    int n;
    int r[20];
};
static Radices radices_of(int N)
{
    Radices R{};
    while (N % 4 == 0) { R.r[R.n++] = 4; N /= 4; }
    while (N % 2 == 0) { R.r[R.n++] = 2; N /= 2; }
    while (N % 3 == 0) { R.r[R.n++] = 3; N /= 3; }
    if (N != 1) R.n = -1;
    return R;
}
constexpr int kMaxFFT = 1024;

__device__ __forceinline__ d2 cm(d2 a, d2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ d2 ad(d2 a, d2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ d2 sb(d2 a, d2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ d2 mul_i(d2 a, double sg) { return make_double2(-sg * a.y, sg * a.x); }  // (sg i) a

// The radices of the stages packed two bits each (R - 2), first stage lowest:
// the kernels read them from one register instead of indexing an array.
static unsigned radix_code(const Radices& R)
{
    unsigned c = 0;
    for (int s = R.n - 1; s >= 0; s--) c = (c << 2) | (unsigned)(R.r[s] - 2);
    return c;
}
__device__ __forceinline__ int stage_radix(unsigned code, int stg) { return (int)((code >> (2 * stg)) & 3u) + 2; }

// The twiddle factors of every stage (R, Ns) of the Stockham FFT below,
// tw[(Ns - 1) + k (R - 1) + q - 1] = exp(sign 2 pi i k q / (Ns R)) for k < Ns
// and 1 <= q < R.  The stages' entries follow one another without gaps, since
// the Ns of a stage is the product of the radices before it: N - 1 in all.
// Made once per initial condition (one block), so that the butterflies read
// their factors instead of evaluating a sine and a cosine each.
__global__ void twiddle_kernel(d2* tw, int nstages, unsigned rcode, int sign)
{
    int Ns = 1;
    for (int stg = 0; stg < nstages; stg++) {
        const int R = stage_radix(rcode, stg);
        for (int t = threadIdx.x; t < Ns * (R - 1); t += blockDim.x) {
            const int k = t / (R - 1), q = t % (R - 1) + 1;
            double sn, cs;
            sincospi((double)sign * 2.0 * (double)(k * q) / (double)(Ns * R), &sn, &cs);
            tw[Ns - 1 + t] = make_double2(cs, sn);
        }
        Ns *= R;
    }
}

// One radix-R stage of the Stockham FFT: butterfly j < N / R takes the inputs
// j + q N / R, multiplies them by the twiddles of its k = j mod Ns, and writes
// the R outputs to (j - k) R + k + q Ns.
template <int R>
__device__ __forceinline__ void fft_stage(const d2* __restrict__ in, d2* __restrict__ out, int N, int Ns, double sg,
                                          const d2* __restrict__ tw)
{
    const int NR = N / R;
    for (int j = threadIdx.x; j < NR; j += blockDim.x) {
        const int k = (int)((unsigned)j % (unsigned)Ns);
        d2 v[R];
#pragma unroll
        for (int q = 0; q < R; q++) v[q] = in[j + q * NR];
        if (Ns > 1) {
            const d2* w = tw + (Ns - 1) + k * (R - 1) - 1;
#pragma unroll
            for (int q = 1; q < R; q++) v[q] = cm(v[q], w[q]);
        }
        d2 o[R];
        if constexpr (R == 2) {
            o[0] = ad(v[0], v[1]);
            o[1] = sb(v[0], v[1]);
        } else if constexpr (R == 4) {
            const d2 a = ad(v[0], v[2]), b = sb(v[0], v[2]), c = ad(v[1], v[3]), d = mul_i(sb(v[1], v[3]), sg);
            o[0] = ad(a, c); o[2] = sb(a, c); o[1] = ad(b, d); o[3] = sb(b, d);
        } else {
            static_assert(R == 3, "radix 2, 3 or 4");
            const d2 t = ad(v[1], v[2]);
            const d2 m = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
            const d2 dd = sb(v[1], v[2]);
            const d2 d = mul_i(make_double2(0.86602540378443864676 * dd.x, 0.86602540378443864676 * dd.y), sg);
            o[0] = ad(v[0], t); o[1] = ad(m, d); o[2] = sb(m, d);
        }
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; q++) out[base + q * Ns] = o[q];
    }
}

// One complex DFT of length N per block (X[k] = sum_n x[n] exp(sign 2 pi i n k / N)),
// Stockham autosort stages in LDS (2 N complex values, dynamic), twiddles from
// the table of twiddle_kernel for this sign.
__global__ __launch_bounds__(256) void fft_rows_kernel(d2* data, int N, int sign, int nstages, unsigned rcode,
                                                       const d2* __restrict__ tw)
{
    extern __shared__ d2 lds[];
    d2 *a = lds, *b = lds + N;
    d2* row = data + (size_t)blockIdx.x * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = row[i];
    __syncthreads();
    int Ns = 1;
    const double sg = sign;
    for (int stg = 0; stg < nstages; stg++) {
        const int R = stage_radix(rcode, stg);
        if (R == 4) fft_stage<4>(a, b, N, Ns, sg, tw);
        else if (R == 2) fft_stage<2>(a, b, N, Ns, sg, tw);
        else fft_stage<3>(a, b, N, Ns, sg, tw);
        __syncthreads();
        d2* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) row[i] = a[i];
}

// out[f][c][r] = in[f][r][c]
__global__ void transpose_kernel(const d2* __restrict__ in, d2* __restrict__ out, int N)
{
    __shared__ d2 tile[32][33];
    const size_t f = blockIdx.z, off = f * (size_t)N * N;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int r = r0 + k, c = c0 + threadIdx.x;
        if (r < N && c < N) tile[k][threadIdx.x] = in[off + (size_t)r * N + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int r = c0 + k, c = r0 + threadIdx.x;
        if (r < N && c < N) out[off + (size_t)r * N + c] = tile[threadIdx.x][k];
    }
}

// multiply by K(k1,k2) = 1/(khat^2 + m^2), khat^2 = 4 sum_i sin^2(pi k_i/N); K = 0 at
// k = 0 and where the continuum |k| = (2 pi/N) |k~| exceeds the UV cut (k~ signed)
__global__ void poisson_kernel(d2* data, int N, int nfields, double mhat, double uvhat, double scale)
{
    const size_t V = (size_t)N * N;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * nfields) return;
    const int e = (int)(i % V);
    const int k1 = e / N, k2 = e % N;
    const double s1 = sinpi((double)k1 / N), s2 = sinpi((double)k2 / N);
    double K = 1.0 / (4.0 * (s1 * s1 + s2 * s2) + mhat * mhat);
    if (k1 == 0 && k2 == 0) K = 0.0;
    if (uvhat > 0) {
        const double q1 = k1 > N / 2 ? k1 - N : k1, q2 = k2 > N / 2 ? k2 - N : k2;
        if ((2.0 * M_PI / N) * sqrt(q1 * q1 + q2 * q2) > uvhat) K = 0.0;
    }
    d2 v = data[i];
    data[i] = make_double2(v.x * K * scale, v.y * K * scale);
}

// ------------------------------------------------------------------ Wilson lines
__device__ __forceinline__ m3<double> ldM(const double* p, int s, int V)
{
    m3<double> m;
    for (int c = 0; c < 9; c++) m.e[c] = {p[(size_t)(2 * c) * V + s], p[(size_t)(2 * c + 1) * V + s]};
    return m;
}
__device__ __forceinline__ void stM(double* p, int s, int V, const m3<double>& m)
{
    for (int c = 0; c < 9; c++) {
        p[(size_t)(2 * c) * V + s] = m.e[c].re;
        p[(size_t)(2 * c + 1) * V + s] = m.e[c].im;
    }
}

__global__ void identity_kernel(double* M, int V)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < V) stM(M, s, V, identity<double>());
}

// Vdag(x) <- Vdag(x) exp(-i alpha_n(x)) for the sheets of one chunk, in order
__global__ void wilson_kernel(const d2* __restrict__ alpha, int nsh, int V, double* Vdag)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    m3<double> v = ldM(Vdag, s, V);
    for (int sh = 0; sh < nsh; sh++) {
        a8<double> a;
        for (int p = 0; p < 4; p++) {
            const d2 w = alpha[((size_t)sh * 4 + p) * V + s];
            a.v[2 * p] = w.x;
            a.v[2 * p + 1] = w.y;
        }
        v = mul(v, expi(a, -1.0));
    }
    stM(Vdag, s, V, v);
}

// SU(2): V^+ as quaternions [4][V]; colours (0, 1) from pair 0, colour 2 from pair 1
__global__ void identity2_kernel(double* Q, int V)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    Q[s] = 1.0;
    Q[(size_t)V + s] = Q[2 * (size_t)V + s] = Q[3 * (size_t)V + s] = 0.0;
}
__device__ __forceinline__ q4<double> ldQ(const double* p, int s, int V)
{
    return {p[s], p[(size_t)V + s], p[2 * (size_t)V + s], p[3 * (size_t)V + s]};
}
__device__ __forceinline__ void stQ(double* p, int s, int V, const q4<double>& q)
{
    p[s] = q.w;
    p[(size_t)V + s] = q.x;
    p[2 * (size_t)V + s] = q.y;
    p[3 * (size_t)V + s] = q.z;
}
__global__ void wilson2_kernel(const d2* __restrict__ alpha, int nsh, int V, double* Vdag)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    q4<double> v = ldQ(Vdag, s, V);
    for (int sh = 0; sh < nsh; sh++) {
        const d2 w0 = alpha[((size_t)sh * 2) * V + s], w1 = alpha[((size_t)sh * 2 + 1) * V + s];
        v = qmul(v, qexpi(v3<double>{{w0.x, w0.y, w1.x}}, -1.0));
    }
    stQ(Vdag, s, V, v);
}

// U^X_i(x) = V(x) V(x+i)^+ = (V^+(x))^+ V^+(x+i)
__global__ void pure_gauge_kernel(const double* __restrict__ Vdag, int N, double* UX)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int x = s % N, y = s / N;
    const int sx = y * N + (x + 1 == N ? 0 : x + 1), sy = (y + 1 == N ? 0 : y + 1) * N + x;
    const m3<double> here = ldM(Vdag, s, V);
    stM(UX, s, V, adj_mul(here, ldM(Vdag, sx, V)));
    stM(UX + 18 * (size_t)V, s, V, adj_mul(here, ldM(Vdag, sy, V)));
}

// rows 1, 2 by Gram-Schmidt, row 3 = conj(r1 x r2)
// Gaussian elimination with partial pivoting, unrolled so that J stays in
// registers: the pivot (the first largest |J[r][c]|, r >= c) is brought up by
// conditional swaps instead of an indexed row exchange.
__device__ __forceinline__ int solve8(double (&J)[8][8], double (&b)[8], double (&x)[8])
{
#pragma unroll
    for (int c = 0; c < 8; c++) {
#pragma unroll
        for (int r = c + 1; r < 8; r++) {
            const bool sw = fabs(J[r][c]) > fabs(J[c][c]);
#pragma unroll
            for (int k = c; k < 8; k++) {
                const double t = J[c][k];
                J[c][k] = sw ? J[r][k] : t;
                J[r][k] = sw ? t : J[r][k];
            }
            const double t = b[c];
            b[c] = sw ? b[r] : t;
            b[r] = sw ? t : b[r];
        }
        if (J[c][c] == 0.0) return -1;
#pragma unroll
        for (int r = c + 1; r < 8; r++) {
            const double f = J[r][c] / J[c][c];
#pragma unroll
            for (int k = c; k < 8; k++) J[r][k] -= f * J[c][k];
            b[r] -= f * b[c];
        }
    }
#pragma unroll
    for (int r = 7; r >= 0; r--) {
        double acc = b[r];
#pragma unroll
        for (int k = r + 1; k < 8; k++) acc -= J[r][k] * x[k];
        x[r] = acc / J[r][r];
    }
    return 0;
}

// tau = 0 links: Newton on Proj[(U^A + U^B)(1 + U^+)] = 0 in the coordinates of
// U = exp(iX) U_0, Jacobian columns Proj[-i W U^+ T^b] (W = U^A + U^B), start at
// the row-projected W; stop at |F|_inf < tol or when the step is at rounding level
__global__ __launch_bounds__(128) void links_kernel(const double* __restrict__ UA, const double* __restrict__ UB, int V, double tol,
                             int maxit, double* U, int* fails)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 2 * V) return;
    const int i = id / V, s = id % V;
    const m3<double> A = ldM(UA + (size_t)i * 18 * V, s, V), B = ldM(UB + (size_t)i * 18 * V, s, V);
    m3<double> W;
    for (int c = 0; c < 9; c++) W.e[c] = {A.e[c].re + B.e[c].re, A.e[c].im + B.e[c].im};
    m3<double> u = reunitarize(W);
    bool ok = false;
    for (int it = 0; it < maxit; it++) {
        const m3<double> WUd = mul_adj(W, u);
        m3<double> M = WUd;
        for (int c = 0; c < 9; c++) { M.e[c].re += W.e[c].re; M.e[c].im += W.e[c].im; }
        const a8<double> F = proj(M);
        double fmax = 0;
        for (int a = 0; a < 8; a++) fmax = fmax > fabs(F.v[a]) ? fmax : fabs(F.v[a]);
        if (fmax < tol) { ok = true; break; }
        double J[8][8], rhs[8], X[8];
        for (int b = 0; b < 8; b++) {
            a8<double> e = azero<double>();
            e.v[b] = 1.0;
            m3<double> Z = mul(WUd, herm(e));
            for (int c = 0; c < 9; c++) Z.e[c] = {Z.e[c].im, -Z.e[c].re};  // -i Z
            const a8<double> col = proj(Z);
            for (int a = 0; a < 8; a++) J[a][b] = col.v[a];
        }
        for (int a = 0; a < 8; a++) rhs[a] = -F.v[a];
        if (solve8(J, rhs, X)) break;
        a8<double> xa;
        double xmax = 0;
        for (int a = 0; a < 8; a++) { xa.v[a] = X[a]; xmax = xmax > fabs(X[a]) ? xmax : fabs(X[a]); }
        u = mul(expi(xa, 1.0), u);
        if (xmax < 1e-15) { ok = true; break; }
    }
    if (!ok) atomicAdd(fails, 1);
    stM(U + (size_t)i * 18 * V, s, V, u);
}

// pi(x) = (1/2) sum_i Proj[(U_i(x)-1)(U^B_i(x)^+ - U^A_i(x)^+) + (U_i(x-i)^+ - 1)(U^B_i(x-i) - U^A_i(x-i))]
__global__ void pi0_kernel(const double* __restrict__ UA, const double* __restrict__ UB, const double* __restrict__ U,
                           int N, double* pi)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int x = s % N, y = s / N;
    m3<double> acc;
    for (int c = 0; c < 9; c++) acc.e[c] = {0, 0};
    for (int i = 0; i < 2; i++) {
        const int sm = i == 0 ? y * N + (x == 0 ? N - 1 : x - 1) : (y == 0 ? N - 1 : y - 1) * N + x;
        const size_t o = (size_t)i * 18 * V;
        m3<double> u = ldM(U + o, s, V), a = ldM(UA + o, s, V), b = ldM(UB + o, s, V);
        m3<double> L = u, R;
        L.e[0].re -= 1; L.e[4].re -= 1; L.e[8].re -= 1;
        for (int c = 0; c < 9; c++) {  // U^B^+ - U^A^+
            const int tr = 3 * (c % 3) + c / 3;
            R.e[c] = {b.e[tr].re - a.e[tr].re, -(b.e[tr].im - a.e[tr].im)};
        }
        m3<double> P1 = mul(L, R);
        u = ldM(U + o, sm, V); a = ldM(UA + o, sm, V); b = ldM(UB + o, sm, V);
        L = adj(u);
        L.e[0].re -= 1; L.e[4].re -= 1; L.e[8].re -= 1;
        for (int c = 0; c < 9; c++) R.e[c] = {b.e[c].re - a.e[c].re, b.e[c].im - a.e[c].im};
        m3<double> P2 = mul(L, R);
        for (int c = 0; c < 9; c++) {
            acc.e[c].re += P1.e[c].re + P2.e[c].re;
            acc.e[c].im += P1.e[c].im + P2.e[c].im;
        }
    }
    const a8<double> p = proj(acc);
    for (int a = 0; a < 8; a++) pi[(size_t)a * V + s] = 0.5 * p.v[a];
}

__global__ void zero_kernel(double* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ------------------------------------------------------------------ particles
// key (seed, 3), counter (p, block, 0, 0).  Block 0: x, y, azimuth, p_T.
// Blocks 1..5: normals; the 3x3 complex Ginibre matrix Z takes entry (r,c)
// from normals 2(3r+c), 2(3r+c)+1; its columns orthonormalised by modified
// Gram-Schmidt give a Haar unitary (positive R diagonal), Q = U Q0 U^+.
__global__ void particles_kernel(PartICArgs a, double* r, int* cell)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int np = a.np, N = a.N;
    if (p >= np) return;
    const uint64_t seed = a.seed;
    const u64x4 w = philox4x64((uint64_t)p, 0, 0, 0, seed, 3);
    const double x = N * u01_co(w.v[0]), y = N * u01_co(w.v[1]);
    const double phi0 = a.azimuth_uniform ? 2.0 * M_PI * u01_co(w.v[2]) : 0.0;
    const double pt = a.pt_min + (a.pt_max - a.pt_min) * u01_co(w.v[3]);
    double z[20];
    for (int b = 1; b <= 5; b++) {
        const u64x4 q = philox4x64((uint64_t)p, (uint64_t)b, 0, 0, seed, 3);
        box_muller(q.v[0], q.v[1], z[4 * (b - 1)], z[4 * (b - 1) + 1]);
        box_muller(q.v[2], q.v[3], z[4 * (b - 1) + 2], z[4 * (b - 1) + 3]);
    }
    m3<double> G;
    for (int rr = 0; rr < 3; rr++)
        for (int cc = 0; cc < 3; cc++) G.e[3 * rr + cc] = {z[2 * (3 * rr + cc)], z[2 * (3 * rr + cc) + 1]};
    for (int k = 0; k < 3; k++) {
        cx<double> v[3] = {G.e[k], G.e[3 + k], G.e[6 + k]};
        for (int j = 0; j < k; j++) {
            cx<double> ip = {0, 0};
            for (int rr = 0; rr < 3; rr++) {
                const cx<double> q = ccmul(G.e[3 * rr + j], v[rr]);
                ip.re += q.re; ip.im += q.im;
            }
            for (int rr = 0; rr < 3; rr++) {
                const cx<double> q = cmul(ip, G.e[3 * rr + j]);
                v[rr].re -= q.re; v[rr].im -= q.im;
            }
        }
        double nn = 0;
        for (int rr = 0; rr < 3; rr++) nn += v[rr].re * v[rr].re + v[rr].im * v[rr].im;
        nn = sqrt(nn);
        for (int rr = 0; rr < 3; rr++) G.e[3 * rr + k] = {v[rr].re / nn, v[rr].im / nn};
    }
    a8<double> q0;
    for (int c = 0; c < 8; c++) q0.v[c] = a.q0[c];
    const a8<double> Q = transport(G, q0);
    const double cph = cos(phi0), sph = sin(phi0);
    auto col = [&](int c) -> double& { return r[(size_t)c * np + p]; };
    col(PX_) = x; col(PY_) = y; col(PETA_) = 0;
    col(PPX) = pt * cph; col(PPY) = pt * sph; col(PPETA) = 0; col(PDETA) = 0;
    col(PUX0) = cph; col(PUY0) = sph; col(PPT0) = pt;
    col(PPTAU) = 0.0;  // set by the push at the formation step
    for (int c = 0; c < 8; c++) col(PQ0 + c) = Q.v[c];
    int nx = (int)floor(x + 0.5), ny = (int)floor(y + 0.5);
    cell[p] = nx >= N ? nx - N : nx;
    cell[np + p] = ny >= N ? ny - N : ny;
}

__global__ void convert_kernel(const double* __restrict__ s, float* __restrict__ d, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

// ------------------------------------------------------------------ drivers
#define CK(x)                                \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// the forward and inverse twiddle tables (2 N entries, freed by the caller)
static hipError_t make_twiddles(d2** tw, int N, const Radices& R, hipStream_t st)
{
    CK(hipMalloc(tw, sizeof(d2) * 2 * N));
    hipLaunchKernelGGL(twiddle_kernel, dim3(1), dim3(256), 0, st, *tw, R.n, radix_code(R), -1);
    hipLaunchKernelGGL(twiddle_kernel, dim3(1), dim3(256), 0, st, *tw + N, R.n, radix_code(R), +1);
    return hipGetLastError();
}

// one nucleus: Wilson line V^+ of its sheets (SU(3): [18][V] matrices; SU(2):
// [4][V] quaternions)
// tw: the twiddle tables of the forward (first N entries) and inverse transforms
static hipError_t nucleus_wilson(const ICArgs& a, int nucleus, d2* buf, d2* tmp, int chunk, double* Vdag,
                                 const Radices& R, const d2* tw, hipStream_t st, int nc = 3)
{
    const int N = a.N, V = N * N;
    const int pairs = nc == 2 ? 2 : 4;
    const size_t lds = (size_t)2 * N * sizeof(d2);
    const unsigned rc = radix_code(R);
    const double sigma = a.g2mua / sqrt((double)a.n_sheets);
    if (nc == 2) hipLaunchKernelGGL(identity2_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, V);
    else hipLaunchKernelGGL(identity_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, V);
    for (int s0 = 0; s0 < a.n_sheets; s0 += chunk) {
        const int nsh = a.n_sheets - s0 < chunk ? a.n_sheets - s0 : chunk;
        const int nf = pairs * nsh;
        hipLaunchKernelGGL(charges_kernel, dim3((V + 255) / 256, nsh), dim3(256), 0, st, buf, V, a.seed, nucleus, s0,
                           sigma, pairs);
        hipLaunchKernelGGL(fft_rows_kernel, dim3(nf * N), dim3(256), lds, st, buf, N, -1, R.n, rc, tw);
        hipLaunchKernelGGL(transpose_kernel, dim3((N + 31) / 32, (N + 31) / 32, nf), dim3(32, 8), 0, st, buf, tmp, N);
        hipLaunchKernelGGL(fft_rows_kernel, dim3(nf * N), dim3(256), lds, st, tmp, N, -1, R.n, rc, tw);
        const size_t tot = (size_t)V * nf;
        hipLaunchKernelGGL(poisson_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tmp, N, nf, a.mhat,
                           a.uvhat, 1.0 / ((double)N * N));
        hipLaunchKernelGGL(fft_rows_kernel, dim3(nf * N), dim3(256), lds, st, tmp, N, +1, R.n, rc, tw + N);
        hipLaunchKernelGGL(transpose_kernel, dim3((N + 31) / 32, (N + 31) / 32, nf), dim3(32, 8), 0, st, tmp, buf, N);
        hipLaunchKernelGGL(fft_rows_kernel, dim3(nf * N), dim3(256), lds, st, buf, N, +1, R.n, rc, tw + N);
        if (nc == 2) hipLaunchKernelGGL(wilson2_kernel, dim3((V + 255) / 256), dim3(256), 0, st, buf, nsh, V, Vdag);
        else hipLaunchKernelGGL(wilson_kernel, dim3((V + 255) / 256), dim3(256), 0, st, buf, nsh, V, Vdag);
        CK(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t ic_glasma(const ICArgs& a, Fields<double> out, int* d_fails, hipStream_t st)
{
    const int N = a.N, V = N * N;
    const Radices R = radices_of(N);
    if (R.n < 0 || N > kMaxFFT || N < 4) return hipErrorInvalidValue;
    const size_t per_sheet = (size_t)4 * V * sizeof(d2);
    int chunk = (int)((size_t)256 << 20) / (int)(per_sheet > 0 ? per_sheet : 1);
    chunk = chunk < 1 ? 1 : (chunk > a.n_sheets ? a.n_sheets : chunk);
    d2 *buf = nullptr, *tmp = nullptr;
    d2* tw = nullptr;
    double *Vdag = nullptr, *UA = nullptr, *UB = nullptr;
    hipError_t e = make_twiddles(&tw, N, R, st);
    if (e == hipSuccess) e = hipMalloc(&buf, per_sheet * chunk);
    if (e == hipSuccess) e = hipMalloc(&tmp, per_sheet * chunk);
    if (e == hipSuccess) e = hipMalloc(&Vdag, sizeof(double) * 18 * V);
    if (e == hipSuccess) e = hipMalloc(&UA, sizeof(double) * 36 * V);
    if (e == hipSuccess) e = hipMalloc(&UB, sizeof(double) * 36 * V);
    if (e == hipSuccess) e = nucleus_wilson(a, 0, buf, tmp, chunk, Vdag, R, tw, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pure_gauge_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, N, UA);
        e = nucleus_wilson(a, 1, buf, tmp, chunk, Vdag, R, tw, st);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pure_gauge_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, N, UB);
        hipLaunchKernelGGL(links_kernel, dim3((2 * V + 127) / 128), dim3(128), 0, st, UA, UB, V, a.tol, a.maxit,
                           out.U, d_fails);
        hipLaunchKernelGGL(pi0_kernel, dim3((V + 255) / 256), dim3(256), 0, st, UA, UB, out.U, N, out.pi);
        const size_t nz = (size_t)24 * V;  // phi (8V) and E (16V) are adjacent
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, out.phi, nz);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    (void)hipFree(buf); (void)hipFree(tmp); (void)hipFree(Vdag); (void)hipFree(UA); (void)hipFree(UB);
    (void)hipFree(tw);
    return e;
}

// ------------------------------------------------------------------ SU(2)
// U^X_i(x) = V(x) V(x+i)^+ on quaternions [2][4][V]
__global__ void pure_gauge2_kernel(const double* __restrict__ Vdag, int N, double* UX)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int x = s % N, y = s / N;
    const int sx = y * N + (x + 1 == N ? 0 : x + 1), sy = (y + 1 == N ? 0 : y + 1) * N + x;
    const q4<double> here = qadj(ldQ(Vdag, s, V));
    stQ(UX, s, V, qmul(here, ldQ(Vdag, sx, V)));
    stQ(UX + 4 * (size_t)V, s, V, qmul(here, ldQ(Vdag, sy, V)));
}
// tau = 0 links: W = U^A + U^B is a real multiple of an SU(2) element S, and
// U = S^2 = W W / |W|^2 solves Proj[W (1 + U^+)] = 0 (W (1 + U^+) = W + W^+ |W|^0
// is then a multiple of 1)
__global__ void links2_kernel(const double* __restrict__ UA, const double* __restrict__ UB, int V, double* U)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * V) return;
    const int i = k / V, s = k - i * V;
    const size_t o = (size_t)i * 4 * V;
    const q4<double> W = qadd(ldQ(UA + o, s, V), ldQ(UB + o, s, V));
    const double n2 = W.w * W.w + W.x * W.x + W.y * W.y + W.z * W.z;
    const q4<double> S2 = qmul(W, W);
    stQ(U + o, s, V, {S2.w / n2, S2.x / n2, S2.y / n2, S2.z / n2});
}
// pi(0) of the SU(3) kernel on quaternions
__global__ void pi02_kernel(const double* __restrict__ UA, const double* __restrict__ UB, const double* __restrict__ U,
                            int N, double* pi)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int x = s % N, y = s / N;
    q4<double> acc = {0, 0, 0, 0};
    for (int i = 0; i < 2; i++) {
        const int sm = i == 0 ? y * N + (x == 0 ? N - 1 : x - 1) : (y == 0 ? N - 1 : y - 1) * N + x;
        const size_t o = (size_t)i * 4 * V;
        const q4<double> P1 = qmul(qsub(ldQ(U + o, s, V), qone<double>()),
                                   qsub(qadj(ldQ(UB + o, s, V)), qadj(ldQ(UA + o, s, V))));
        const q4<double> P2 = qmul(qsub(qadj(ldQ(U + o, sm, V)), qone<double>()),
                                   qsub(ldQ(UB + o, sm, V), ldQ(UA + o, sm, V)));
        acc = qadd(acc, qadd(P1, P2));
    }
    const v3<double> p = qproj(acc);
    for (int a = 0; a < 3; a++) pi[(size_t)a * V + s] = 0.5 * p.v[a];
}

hipError_t ic_glasma2(const ICArgs& a, Fields2<double> out, hipStream_t st)
{
    const int N = a.N, V = N * N;
    const Radices R = radices_of(N);
    if (R.n < 0 || N > kMaxFFT || N < 4) return hipErrorInvalidValue;
    const size_t per_sheet = (size_t)2 * V * sizeof(d2);
    int chunk = (int)((size_t)256 << 20) / (int)(per_sheet > 0 ? per_sheet : 1);
    chunk = chunk < 1 ? 1 : (chunk > a.n_sheets ? a.n_sheets : chunk);
    d2 *buf = nullptr, *tmp = nullptr;
    d2* tw = nullptr;
    double *Vdag = nullptr, *UA = nullptr, *UB = nullptr;
    hipError_t e = make_twiddles(&tw, N, R, st);
    if (e == hipSuccess) e = hipMalloc(&buf, per_sheet * chunk);
    if (e == hipSuccess) e = hipMalloc(&tmp, per_sheet * chunk);
    if (e == hipSuccess) e = hipMalloc(&Vdag, sizeof(double) * 4 * V);
    if (e == hipSuccess) e = hipMalloc(&UA, sizeof(double) * 8 * V);
    if (e == hipSuccess) e = hipMalloc(&UB, sizeof(double) * 8 * V);
    if (e == hipSuccess) e = nucleus_wilson(a, 0, buf, tmp, chunk, Vdag, R, tw, st, 2);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pure_gauge2_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, N, UA);
        e = nucleus_wilson(a, 1, buf, tmp, chunk, Vdag, R, tw, st, 2);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pure_gauge2_kernel, dim3((V + 255) / 256), dim3(256), 0, st, Vdag, N, UB);
        hipLaunchKernelGGL(links2_kernel, dim3((2 * V + 255) / 256), dim3(256), 0, st, UA, UB, V, out.U);
        hipLaunchKernelGGL(pi02_kernel, dim3((V + 255) / 256), dim3(256), 0, st, UA, UB, out.U, N, out.pi);
        const size_t nz = (size_t)9 * V;  // phi (3V) and E (6V) are adjacent
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, out.phi, nz);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    (void)hipFree(buf); (void)hipFree(tmp); (void)hipFree(Vdag); (void)hipFree(UA); (void)hipFree(UB);
    (void)hipFree(tw);
    return e;
}

// SU(2) particles: block 0 as for SU(3); the charge from the Darboux
// parametrisation (Sec. IV.A) with J^2 = q2: words 0, 1 of block 1 give
// phi = 2 pi u and xi = J (2 u' - 1), Q = (cos phi rho, sin phi rho, xi),
// rho = sqrt(J^2 - xi^2).  Records keep the SU(3) layout (Q^4..Q^8 = 0).
__global__ void particles2_kernel(PartICArgs a, double J, double* r, int* cell)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int np = a.np, N = a.N;
    if (p >= np) return;
    const u64x4 w = philox4x64((uint64_t)p, 0, 0, 0, a.seed, 3);
    const u64x4 v = philox4x64((uint64_t)p, 1, 0, 0, a.seed, 3);
    const double x = N * u01_co(w.v[0]), y = N * u01_co(w.v[1]);
    const double phi0 = a.azimuth_uniform ? 2.0 * M_PI * u01_co(w.v[2]) : 0.0;
    const double pt = a.pt_min + (a.pt_max - a.pt_min) * u01_co(w.v[3]);
    const double ph = 2.0 * M_PI * u01_co(v.v[0]), xi = J * (2.0 * u01_co(v.v[1]) - 1.0);
    const double rho = sqrt(J * J - xi * xi);
    const double cph = cos(phi0), sph = sin(phi0);
    auto col = [&](int c) -> double& { return r[(size_t)c * np + p]; };
    col(PX_) = x; col(PY_) = y; col(PETA_) = 0;
    col(PPX) = pt * cph; col(PPY) = pt * sph; col(PPETA) = 0; col(PDETA) = 0;
    col(PUX0) = cph; col(PUY0) = sph; col(PPT0) = pt;
    col(PPTAU) = 0.0;  // set by the push at the formation step
    col(PQ0) = cos(ph) * rho; col(PQ0 + 1) = sin(ph) * rho; col(PQ0 + 2) = xi;
    for (int c = 3; c < 8; c++) col(PQ0 + c) = 0.0;
    int nx = (int)floor(x + 0.5), ny = (int)floor(y + 0.5);
    cell[p] = nx >= N ? nx - N : nx;
    cell[np + p] = ny >= N ? ny - N : ny;
}

hipError_t ic_particles2(const PartICArgs& a, double q2, double* r, int* cell, hipStream_t st)
{
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(particles2_kernel, dim3((a.np + 127) / 128), dim3(128), 0, st, a, sqrt(q2), r, cell);
    return hipGetLastError();
}

hipError_t ic_particles(const PartICArgs& a, double* r, int* cell, hipStream_t st)
{
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(particles_kernel, dim3((a.np + 127) / 128), dim3(128), 0, st, a, r, cell);
    return hipGetLastError();
}

hipError_t convert_to_float(const double* src, float* dst, size_t n, hipStream_t st)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace cpic
