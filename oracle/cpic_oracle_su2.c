/*
 * cpic_oracle_su2.c -- the SU(2) variant of the plain FP64 CPU oracle
 * (arXiv:2303.05599 treats the colour charges and Casimirs for SU(2) and
 * SU(3) side by side, Sec. IV; the field and particle equations of Sec. II.A
 * and III.B hold for any SU(N_c)).
 *
 * TEST INFRASTRUCTURE ONLY, like cpic_oracle.c (same library, same
 * conventions and readings, written for 2x2 matrices):
 *   links U[i][s] are 2x2 complex, row-major;
 *   algebra fields hold the 3 real components X^a of X = X^a T^a with
 *   T^a = sigma^a / 2;
 *   particle records have the 20 columns of the SU(3) oracle, with Q^1..Q^3
 *   in columns 6..8 and columns 9..13 zero.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx e[2][2]; } M2;

void orc_philox(const uint64_t *ctr_in, const uint64_t *key_in, uint64_t *out);

/* generators T^a = sigma^a / 2 (Pauli matrices) */
static M2 gen2(int a)
{
    M2 t;
    memset(&t, 0, sizeof t);
    if (a == 0) { t.e[0][1] = 0.5; t.e[1][0] = 0.5; }
    if (a == 1) { t.e[0][1] = -0.5 * I; t.e[1][0] = 0.5 * I; }
    if (a == 2) { t.e[0][0] = 0.5; t.e[1][1] = -0.5; }
    return t;
}

/* ------------------------- 2x2 complex algebra ------------------------- */
static M2 z2(void) { M2 z; memset(&z, 0, sizeof z); return z; }
static M2 id2(void) { M2 z = z2(); z.e[0][0] = z.e[1][1] = 1; return z; }
static M2 mul2(M2 a, M2 b)
{
    M2 c = z2();
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            for (int k = 0; k < 2; k++) c.e[i][j] += a.e[i][k] * b.e[k][j];
    return c;
}
static M2 adj2(M2 a)
{
    M2 c;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) c.e[i][j] = conj(a.e[j][i]);
    return c;
}
static M2 add2(M2 a, M2 b)
{
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) a.e[i][j] += b.e[i][j];
    return a;
}
static M2 sub2(M2 a, M2 b)
{
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) a.e[i][j] -= b.e[i][j];
    return a;
}
static M2 scale2(M2 a, cplx s)
{
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) a.e[i][j] *= s;
    return a;
}
static cplx tr2(M2 a) { return a.e[0][0] + a.e[1][1]; }
static M2 mul2_3(M2 a, M2 b, M2 c) { return mul2(mul2(a, b), c); }
static M2 mul2_4(M2 a, M2 b, M2 c, M2 d) { return mul2(mul2(mul2(a, b), c), d); }

static M2 alg2(const double *x)
{
    M2 m = z2();
    for (int a = 0; a < 3; a++) m = add2(m, scale2(gen2(a), x[a]));
    return m;
}
/* x^a = 2 Re Tr(T^a X) for Hermitian X */
static void comps2(M2 X, double *x)
{
    for (int a = 0; a < 3; a++) x[a] = 2.0 * creal(tr2(mul2(gen2(a), X)));
}
/* Proj[M]: traceless Hermitian part of -i (M - M^+)/2, as for SU(3) */
static void proj2(M2 M, double *x)
{
    M2 A = scale2(sub2(M, adj2(M)), 0.5);
    cplx tr = tr2(A) / 2.0;
    A.e[0][0] -= tr;
    A.e[1][1] -= tr;
    comps2(scale2(A, -I), x);
}
/* exp(A) by scaling and squaring of the Taylor series */
static M2 exp2m(M2 A)
{
    double nrm = 0;
    for (int i = 0; i < 2; i++) {
        double r = cabs(A.e[i][0]) + cabs(A.e[i][1]);
        if (r > nrm) nrm = r;
    }
    int s = 0;
    while (nrm > 0.5) { nrm *= 0.5; s++; }
    M2 B = scale2(A, ldexp(1.0, -s));
    M2 sum = id2(), term = id2();
    for (int k = 1; k <= 24; k++) {
        term = scale2(mul2(term, B), 1.0 / k);
        sum = add2(sum, term);
    }
    for (int k = 0; k < s; k++) sum = mul2(sum, sum);
    return sum;
}
static M2 expi2(const double *x, double scale)
{
    double y[3];
    for (int a = 0; a < 3; a++) y[a] = scale * x[a];
    return exp2m(scale2(alg2(y), I));
}

/* --------------------------- lattice helpers --------------------------- */
static inline int nb2(int s, int dx, int dy, int N)
{
    int x = s % N, y = s / N;
    x = ((x + dx) % N + N) % N;
    y = ((y + dy) % N + N) % N;
    return y * N + x;
}
static inline int dir2(int s, int i, int sign, int N) { return i == 0 ? nb2(s, sign, 0, N) : nb2(s, 0, sign, N); }
static inline M2 lnk(const cplx *U, int N, int i, int s)
{
    M2 m;
    memcpy(&m, U + ((size_t)i * N * N + s) * 4, sizeof m);
    return m;
}
static inline void set_lnk(cplx *U, int N, int i, int s, M2 m) { memcpy(U + ((size_t)i * N * N + s) * 4, &m, sizeof m); }
/* U_ij(x) = U_i(x) U_j(x+i) U_i(x+j)^+ U_j(x)^+ */
static M2 plaq2(const cplx *U, int N, int i, int j, int s)
{
    return mul2_4(lnk(U, N, i, s), lnk(U, N, j, dir2(s, i, +1, N)), adj2(lnk(U, N, i, dir2(s, j, +1, N))),
                  adj2(lnk(U, N, j, s)));
}
/* U_{i,-j}(x) = U_i(x) U_j(x+i-j)^+ U_i(x-j)^+ U_j(x-j) */
static M2 plaq2_ineg(const cplx *U, int N, int i, int j, int s)
{
    int xmj = dir2(s, j, -1, N), xpimj = dir2(xmj, i, +1, N);
    return mul2_4(lnk(U, N, i, s), adj2(lnk(U, N, j, xpimj)), adj2(lnk(U, N, i, xmj)), lnk(U, N, j, xmj));
}
static M2 fwd2(const cplx *U, const double *phi, int N, int i, int s)
{
    M2 u = lnk(U, N, i, s);
    return mul2_3(u, alg2(phi + 3 * (size_t)dir2(s, i, +1, N)), adj2(u));
}
static M2 bwd2(const cplx *U, const double *phi, int N, int i, int s)
{
    int xm = dir2(s, i, -1, N);
    M2 u = lnk(U, N, i, xm);
    return mul2_3(adj2(u), alg2(phi + 3 * (size_t)xm), u);
}

/* ============================ field equations ============================
 * The SU(3) oracle's kick, drift and leapfrog (Sec. II.A) for 2x2 links. */
void orc2_forces(int N, double t, const cplx *U, const double *phi, double *FE, double *Fpi)
{
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        M2 ph = alg2(phi + 3 * (size_t)s);
        M2 lap = z2();
        for (int i = 0; i < 2; i++) {
            int j = 1 - i;
            double p1[3], p2[3], cm[3];
            proj2(plaq2(U, N, i, j, s), p1);
            proj2(plaq2_ineg(U, N, i, j, s), p2);
            M2 fw = fwd2(U, phi, N, i, s), bw = bwd2(U, phi, N, i, s);
            comps2(scale2(sub2(mul2(fw, ph), mul2(ph, fw)), I), cm);
            for (int a = 0; a < 3; a++) FE[((size_t)i * V + s) * 3 + a] = -t * (p1[a] + p2[a]) + cm[a] / t;
            lap = add2(lap, sub2(add2(fw, bw), scale2(ph, 2.0)));
        }
        double l[3];
        comps2(lap, l);
        for (int a = 0; a < 3; a++) Fpi[(size_t)s * 3 + a] = l[a] / t;
    }
}

static void kick2(int N, double t, double dt, const cplx *U, const double *phi, double *E, double *pi)
{
    const size_t V = (size_t)N * N;
    double *FE = malloc(sizeof(double) * 6 * V), *Fp = malloc(sizeof(double) * 3 * V);
    orc2_forces(N, t, U, phi, FE, Fp);
    for (size_t k = 0; k < 6 * V; k++) E[k] += dt * FE[k];
    for (size_t k = 0; k < 3 * V; k++) pi[k] += dt * Fp[k];
    free(FE);
    free(Fp);
}

static void drift2(int N, double th, double dt, cplx *U, double *phi, const double *E, const double *pi)
{
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        for (int i = 0; i < 2; i++)
            set_lnk(U, N, i, s, mul2(expi2(E + ((size_t)i * V + s) * 3, dt / th), lnk(U, N, i, s)));
        for (int a = 0; a < 3; a++) phi[(size_t)s * 3 + a] += dt * th * pi[(size_t)s * 3 + a];
    }
}

/* one leapfrog step n -> n+1; kick skipped at n = 0; t_fixed > 0 freezes time */
void orc2_field_step(int N, int n, double dt, double t_fixed, cplx *U, double *phi, double *E, double *pi)
{
    double t = t_fixed > 0 ? t_fixed : n * dt;
    double th = t_fixed > 0 ? t_fixed : (n + 0.5) * dt;
    if (n > 0 || t_fixed > 0) kick2(N, t, dt, U, phi, E, pi);
    drift2(N, th, dt, U, phi, E, pi);
}

/* the lattice Hamiltonian terms of orc_energy, 2 Re Tr(1 - U_12) with Tr 1 = 2 */
void orc2_energy(int N, double t, const cplx *U, const double *phi, const double *E, const double *pi, double *out)
{
    const int V = N * N;
    double kt = 0, kl = 0, vb = 0, vp = 0;
    for (int s = 0; s < V; s++) {
        for (int k = 0; k < 3; k++) {
            kt += 0.5 * (E[(size_t)s * 3 + k] * E[(size_t)s * 3 + k] +
                         E[((size_t)V + s) * 3 + k] * E[((size_t)V + s) * 3 + k]);
            kl += 0.5 * pi[(size_t)s * 3 + k] * pi[(size_t)s * 3 + k];
        }
        vb += 2.0 * creal(2.0 - tr2(plaq2(U, N, 0, 1, s)));
        M2 ph = alg2(phi + 3 * (size_t)s);
        for (int i = 0; i < 2; i++) {
            M2 d = sub2(fwd2(U, phi, N, i, s), ph);
            vp += creal(tr2(mul2(d, d)));
        }
    }
    out[0] = kt / t;
    out[1] = kl * t;
    out[2] = vb * t;
    out[3] = vp / t;
}

/* Gauss residual sum_i [E_i(x) - U_i(x-i)^+ E_i(x-i) U_i(x-i)] + i[phi, pi] */
void orc2_gauss(int N, const cplx *U, const double *phi, const double *E, const double *pi, double *G)
{
    const int V = N * N;
    for (int s = 0; s < V; s++) {
        M2 g = z2();
        for (int i = 0; i < 2; i++) {
            int xm = dir2(s, i, -1, N);
            M2 u = lnk(U, N, i, xm);
            g = add2(g, sub2(alg2(E + ((size_t)i * V + s) * 3), mul2_3(adj2(u), alg2(E + ((size_t)i * V + xm) * 3), u)));
        }
        M2 ph = alg2(phi + 3 * (size_t)s), pp = alg2(pi + 3 * (size_t)s);
        g = add2(g, scale2(sub2(mul2(ph, pp), mul2(pp, ph)), I));
        comps2(g, G + 3 * (size_t)s);
    }
}

/* ======================== MV initial condition ======================== */
static double u01c(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
static double u01o(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }

/* colours 1..3 of a sheet: the first three of the four normals of Philox
 * block 0 of the SU(3) stream (key (seed, 1 + nucleus), counter (site,
 * sheet, 0, 0)), Box-Muller on word pairs (0,1) and (2,3) */
void orc2_mv_charges(int N, uint64_t seed, int nucleus, int sheet, double sigma, double *rho)
{
    const int V = N * N;
    uint64_t key[2] = {seed, (uint64_t)(1 + nucleus)};
    for (int s = 0; s < V; s++) {
        uint64_t ctr[4] = {(uint64_t)s, (uint64_t)sheet, 0, 0}, r[4];
        orc_philox(ctr, key, r);
        double z[4];
        for (int k = 0; k < 2; k++) {
            double rad = sqrt(-2.0 * log(u01o(r[2 * k]))), ang = 2.0 * M_PI * u01c(r[2 * k + 1]);
            z[2 * k] = rad * cos(ang);
            z[2 * k + 1] = rad * sin(ang);
        }
        for (int a = 0; a < 3; a++) rho[(size_t)s * 3 + a] = sigma * z[a];
    }
}

void orc2_wilson_mult(int N, const double *alpha, cplx *Vdag)
{
    const int V = N * N;
    for (int s = 0; s < V; s++) {
        M2 v;
        memcpy(&v, Vdag + (size_t)s * 4, sizeof v);
        v = mul2(v, expi2(alpha + (size_t)s * 3, -1.0));
        memcpy(Vdag + (size_t)s * 4, &v, sizeof v);
    }
}

void orc2_pure_gauge(int N, const cplx *Vdag, cplx *UX)
{
    const int V = N * N;
    for (int i = 0; i < 2; i++)
        for (int s = 0; s < V; s++) {
            M2 a, b;
            memcpy(&a, Vdag + (size_t)s * 4, sizeof a);
            memcpy(&b, Vdag + (size_t)dir2(s, i, +1, N) * 4, sizeof b);
            set_lnk(UX, N, i, s, mul2(adj2(a), b));
        }
}

/*
 * Glasma links at tau = 0: the condition Proj[(U^A + U^B)(1 + U^+)] = 0 of
 * the SU(3) oracle.  For SU(2), W = U^A + U^B is a real multiple of an
 * SU(2) matrix S, and U = W (W^+)^-1 = S^2 solves it exactly:
 * W (1 + U^+) = c (S + S^+) is a multiple of the identity.
 */
void orc2_links(int N, const cplx *UA, const cplx *UB, cplx *U)
{
    const int V = N * N;
    for (int i = 0; i < 2; i++)
        for (int s = 0; s < V; s++) {
            M2 W = add2(lnk(UA, N, i, s), lnk(UB, N, i, s));
            M2 Wd = adj2(W);
            cplx det = Wd.e[0][0] * Wd.e[1][1] - Wd.e[0][1] * Wd.e[1][0];
            M2 inv;
            inv.e[0][0] = Wd.e[1][1] / det;
            inv.e[1][1] = Wd.e[0][0] / det;
            inv.e[0][1] = -Wd.e[0][1] / det;
            inv.e[1][0] = -Wd.e[1][0] / det;
            set_lnk(U, N, i, s, mul2(W, inv));
        }
}

/* pi(0) of the SU(3) oracle (same reading, same 1/2) */
void orc2_pi0(int N, const cplx *UA, const cplx *UB, const cplx *U, double *pi)
{
    const int V = N * N;
    for (int s = 0; s < V; s++) {
        M2 acc = z2();
        for (int i = 0; i < 2; i++) {
            int xm = dir2(s, i, -1, N);
            M2 t1 = mul2(sub2(lnk(U, N, i, s), id2()), sub2(adj2(lnk(UB, N, i, s)), adj2(lnk(UA, N, i, s))));
            M2 t2 = mul2(sub2(adj2(lnk(U, N, i, xm)), id2()), sub2(lnk(UB, N, i, xm), lnk(UA, N, i, xm)));
            acc = add2(acc, add2(t1, t2));
        }
        double p[3];
        proj2(acc, p);
        for (int a = 0; a < 3; a++) pi[(size_t)s * 3 + a] = 0.5 * p[a];
    }
}

/* ============================ test particles ============================ */
enum { Q_X = 0, Q_Y, Q_ETA, Q_PX, Q_PY, Q_PETA, Q_Q, Q_CX = 14, Q_CY, Q_DETA, Q_UX0, Q_UY0, Q_PT0, Q_NCOL };

/* classical quadratic Casimir q2 = D_R C_2(R) [eq:q23c23]: 3/2 (F), 6 (A) */
double orc2_q2(int rep) { return rep == 1 ? 6.0 : 1.5; }

/*
 * Particle initial conditions: positions, azimuth and p_T from Philox block
 * 0 as in the SU(3) oracle (key (seed, 3), counter (p, 0, 0, 0)); the
 * charge from the Darboux parametrisation of Sec. IV.A with J^2 = q2:
 * Q = (cos(phi) sqrt(J^2 - xi^2), sin(phi) sqrt(J^2 - xi^2), xi), phi = 2 pi u1,
 * xi = J (2 u2 - 1), u1, u2 from words 0 and 1 of block 1.
 */
void orc2_particles_init(int N, int np, uint64_t seed, double pt_min, double pt_max, int azimuth_uniform, int rep,
                         double *P)
{
    const double J = sqrt(orc2_q2(rep));
    uint64_t key[2] = {seed, 3};
    for (int p = 0; p < np; p++) {
        double *r = P + (size_t)p * Q_NCOL;
        memset(r, 0, sizeof(double) * Q_NCOL);
        uint64_t c0[4] = {(uint64_t)p, 0, 0, 0}, w[4], c1[4] = {(uint64_t)p, 1, 0, 0}, v[4];
        orc_philox(c0, key, w);
        orc_philox(c1, key, v);
        r[Q_X] = N * u01c(w[0]);
        r[Q_Y] = N * u01c(w[1]);
        double phi0 = azimuth_uniform ? 2.0 * M_PI * u01c(w[2]) : 0.0;
        double pt = pt_min + (pt_max - pt_min) * u01c(w[3]);
        double ph = 2.0 * M_PI * u01c(v[0]), xi = J * (2.0 * u01c(v[1]) - 1.0);
        double rho = sqrt(J * J - xi * xi);
        r[Q_Q] = cos(ph) * rho;
        r[Q_Q + 1] = sin(ph) * rho;
        r[Q_Q + 2] = xi;
        r[Q_PX] = pt * cos(phi0);
        r[Q_PY] = pt * sin(phi0);
        r[Q_CX] = fmod(floor(r[Q_X] + 0.5), N);
        r[Q_CY] = fmod(floor(r[Q_Y] + 0.5), N);
        r[Q_UX0] = cos(phi0);
        r[Q_UY0] = sin(phi0);
        r[Q_PT0] = pt;
    }
}

/* colour fields at site c at t_n, the interpolations of orc_particle_fields:
 * out[3k + a], k = E_1, E_2, E_eta, B_1, B_2, B_eta */
void orc2_particle_fields(int N, int n, double dt, int s, const cplx *U, const double *phi, const double *E_old,
                          const double *E_new, const double *pi_old, const double *pi_new, double *out)
{
    const int V = N * N;
    const double t = n * dt;
    memset(out, 0, sizeof(double) * 18);
    for (int i = 0; n > 0 && i < 2; i++) {
        int xm = dir2(s, i, -1, N);
        M2 u = lnk(U, N, i, xm);
        double here[3], back[3], e[3];
        for (int a = 0; a < 3; a++) {
            here[a] = E_new[((size_t)i * V + s) * 3 + a] + E_old[((size_t)i * V + s) * 3 + a];
            back[a] = E_new[((size_t)i * V + xm) * 3 + a] + E_old[((size_t)i * V + xm) * 3 + a];
        }
        comps2(add2(alg2(here), mul2_3(adj2(u), alg2(back), u)), e);
        for (int a = 0; a < 3; a++) out[3 * i + a] = e[a] / (4.0 * t);
    }
    for (int a = 0; a < 3; a++)
        out[6 + a] = n == 0 ? pi_new[(size_t)s * 3 + a] : 0.5 * (pi_new[(size_t)s * 3 + a] + pi_old[(size_t)s * 3 + a]);
    if (n > 0) {
        double b[3];
        comps2(sub2(fwd2(U, phi, N, 1, s), bwd2(U, phi, N, 1, s)), b);
        for (int a = 0; a < 3; a++) out[9 + a] = -b[a] / (2.0 * t);
        comps2(sub2(fwd2(U, phi, N, 0, s), bwd2(U, phi, N, 0, s)), b);
        for (int a = 0; a < 3; a++) out[12 + a] = b[a] / (2.0 * t);
    }
    int xm1 = nb2(s, -1, 0, N), xm2 = nb2(s, 0, -1, N), xm1m2 = nb2(s, -1, -1, N);
    int xp1 = nb2(s, 1, 0, N), xp2 = nb2(s, 0, 1, N), xm1p2 = nb2(s, -1, 1, N), xp1m2 = nb2(s, 1, -1, N);
    M2 c12 = mul2_4(lnk(U, N, 0, s), lnk(U, N, 1, xp1), adj2(lnk(U, N, 0, xp2)), adj2(lnk(U, N, 1, s)));
    M2 c2m1 = mul2_4(lnk(U, N, 1, s), adj2(lnk(U, N, 0, xm1p2)), adj2(lnk(U, N, 1, xm1)), lnk(U, N, 0, xm1));
    M2 cm1m2 = mul2_4(adj2(lnk(U, N, 0, xm1)), adj2(lnk(U, N, 1, xm1m2)), lnk(U, N, 0, xm1m2), lnk(U, N, 1, xm2));
    M2 cm21 = mul2_4(adj2(lnk(U, N, 1, xm2)), lnk(U, N, 0, xm2), lnk(U, N, 1, xp1m2), adj2(lnk(U, N, 0, s)));
    double bz[3];
    proj2(add2(add2(c12, c2m1), add2(cm1m2, cm21)), bz);
    for (int a = 0; a < 3; a++) out[15 + a] = -0.25 * bz[a];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void rot2(double *Q, M2 A)
{
    double q[3];
    comps2(mul2_3(adj2(A), alg2(Q), A), q);
    memcpy(Q, q, sizeof q);
}

/* one particle step at t_n (the SU(3) oracle's orc_particles_step, CPIC rotation) */
int orc2_particles_step(int N, int n, int n_form, double dt, double mhat, int is_static, const cplx *U,
                        const double *phi, const double *E_old, const double *E_new, const double *pi_old,
                        const double *pi_new, int np, double *P)
{
    int errors = 0;
    const double t = n * dt;
#pragma omp parallel for schedule(static) reduction(+ : errors)
    for (int p = 0; p < np; p++) {
        double *r = P + (size_t)p * Q_NCOL;
        double f[18];
        if (is_static) {
            int s = (int)r[Q_CY] * N + (int)r[Q_CX];
            orc2_particle_fields(N, n, dt, s, U, phi, E_old, E_new, pi_old, pi_new, f);
            r[Q_PX] += dt * dot3(r + Q_Q, f);
            r[Q_PY] += dt * dot3(r + Q_Q, f + 3);
            r[Q_PETA] += dt * dot3(r + Q_Q, f + 6);
            continue;
        }
        int cx = (int)r[Q_CX], cy = (int)r[Q_CY];
        int nx = ((int)floor(r[Q_X] + 0.5)) % N, ny = ((int)floor(r[Q_Y] + 0.5)) % N;
        if (n > n_form) {
            int d[2] = {nx - cx, ny - cy};
            for (int ax = 0; ax < 2; ax++) {
                if (d[ax] > N / 2) d[ax] -= N;
                if (d[ax] < -N / 2) d[ax] += N;
                int c = cy * N + cx;
                if (d[ax] == 1) rot2(r + Q_Q, lnk(U, N, ax, c));
                else if (d[ax] == -1) rot2(r + Q_Q, adj2(lnk(U, N, ax, dir2(c, ax, -1, N))));
                else if (d[ax] != 0) errors++;
                if (ax == 0) cx = nx; else cy = ny;
            }
            rot2(r + Q_Q, expi2(phi + 3 * (size_t)(ny * N + nx), r[Q_DETA]));
        }
        orc2_particle_fields(N, n, dt, ny * N + nx, U, phi, E_old, E_new, pi_old, pi_new, f);
        const double *Q = r + Q_Q;
        double e1 = dot3(Q, f), e2 = dot3(Q, f + 3), ee = dot3(Q, f + 6);
        double b1 = dot3(Q, f + 9), b2 = dot3(Q, f + 12), be = dot3(Q, f + 15);
        double px = r[Q_PX], py = r[Q_PY], pe = r[Q_PETA];
        double ptau = sqrt(px * px + py * py + (t * pe) * (t * pe) + mhat * mhat);
        double v1 = px / ptau, v2 = py / ptau, vl = t * pe / ptau;
        r[Q_PX] = px + dt * (e1 + be * v2 - b2 * vl);
        r[Q_PY] = py + dt * (e2 - be * v1 + b1 * vl);
        if (n > 0) r[Q_PETA] = pe + dt * (ee - b1 * v2 + b2 * v1 - 2.0 * pe) / t;
        double x = r[Q_X] + dt * v1, y = r[Q_Y] + dt * v2;
        if (x >= N) x -= N; else if (x < 0) x += N;
        if (y >= N) y -= N; else if (y < 0) y += N;
        r[Q_X] = x;
        r[Q_Y] = y;
        r[Q_DETA] = dt * pe / ptau;
        r[Q_ETA] += r[Q_DETA];
        r[Q_CX] = nx;
        r[Q_CY] = ny;
    }
    return errors;
}

/* ----------------------------- pin exports ----------------------------- */
void orc2_generator(int a, cplx *out)
{
    M2 t = gen2(a);
    memcpy(out, &t, sizeof t);
}
void orc2_expi(const double *x, double scale, cplx *out)
{
    M2 m = expi2(x, scale);
    memcpy(out, &m, sizeof m);
}
void orc2_proj(const cplx *M, double *out)
{
    M2 m;
    memcpy(&m, M, sizeof m);
    proj2(m, out);
}
