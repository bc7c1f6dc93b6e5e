/*
 * cpic_oracle.c -- plain FP64 CPU oracle for the colored particle-in-cell
 * (CPIC) method of arXiv:2303.05599 ("Simulating jets and heavy quarks in
 * the Glasma using the colored particle-in-cell method").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP
 * path: it has its own SU(3) algebra, exponential, random numbers and
 * lattice stencils, written as slowly and plainly as possible so that each
 * step can be checked against the paper by eye.
 *
 * Conventions (hat units, everything dimensionless):
 *   sites s = y*N + x, x along e1, periodic in both directions;
 *   links U[i][s] (i = 0: e1, i = 1: e2) are 3x3 complex, row-major;
 *   algebra fields E[i][s][a], phi[s][a], pi[s][a] hold the 8 real
 *   components X^a of X = X^a T^a with T^a = lambda^a / 2;
 *   phi = g A_eta, E_i = g a P^i, pi = g a^2 P^eta, t = tau / a.
 *
 * Where the paper is ambiguous the reading taken here is listed in the
 * design notes; the main ones are marked "reading:" below.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx e[3][3]; } M3;

/* ------------------------------------------------------------------ */
/* SU(3) generators T^a = lambda^a / 2 (Appendix B.1, Gell-Mann basis) */
/* ------------------------------------------------------------------ */
static M3 GEN[8];
static int gen_ready = 0;

static void build_generators(void)
{
    if (gen_ready) return;
    memset(GEN, 0, sizeof(GEN));
    const double s3 = sqrt(3.0);
    /* lambda_1 */ GEN[0].e[0][1] = 1;      GEN[0].e[1][0] = 1;
    /* lambda_2 */ GEN[1].e[0][1] = -I;     GEN[1].e[1][0] = I;
    /* lambda_3 */ GEN[2].e[0][0] = 1;      GEN[2].e[1][1] = -1;
    /* lambda_4 */ GEN[3].e[0][2] = 1;      GEN[3].e[2][0] = 1;
    /* lambda_5 */ GEN[4].e[0][2] = -I;     GEN[4].e[2][0] = I;
    /* lambda_6 */ GEN[5].e[1][2] = 1;      GEN[5].e[2][1] = 1;
    /* lambda_7 */ GEN[6].e[1][2] = -I;     GEN[6].e[2][1] = I;
    /* lambda_8 */ GEN[7].e[0][0] = 1 / s3; GEN[7].e[1][1] = 1 / s3; GEN[7].e[2][2] = -2 / s3;
    for (int a = 0; a < 8; a++)
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) GEN[a].e[r][c] *= 0.5;
    gen_ready = 1;
}

__attribute__((constructor)) static void oracle_init(void) { build_generators(); }

/* ------------------------- 3x3 complex algebra ------------------------- */
static M3 m_zero(void) { M3 z; memset(&z, 0, sizeof z); return z; }
static M3 m_id(void) { M3 z = m_zero(); z.e[0][0] = z.e[1][1] = z.e[2][2] = 1; return z; }

static M3 m_mul(M3 a, M3 b)
{
    M3 c = m_zero();
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) c.e[i][j] += a.e[i][k] * b.e[k][j];
    return c;
}
static M3 m_adj(M3 a)
{
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c.e[i][j] = conj(a.e[j][i]);
    return c;
}
static M3 m_add(M3 a, M3 b)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) a.e[i][j] += b.e[i][j];
    return a;
}
static M3 m_sub(M3 a, M3 b)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) a.e[i][j] -= b.e[i][j];
    return a;
}
static M3 m_scale(M3 a, cplx s)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) a.e[i][j] *= s;
    return a;
}
static cplx m_tr(M3 a) { return a.e[0][0] + a.e[1][1] + a.e[2][2]; }
static M3 m_mul3(M3 a, M3 b, M3 c) { return m_mul(m_mul(a, b), c); }
static M3 m_mul4(M3 a, M3 b, M3 c, M3 d) { return m_mul(m_mul(m_mul(a, b), c), d); }

/* X = sum_a x^a T^a */
static M3 alg_to_mat(const double *x)
{
    M3 m = m_zero();
    for (int a = 0; a < 8; a++) m = m_add(m, m_scale(GEN[a], x[a]));
    return m;
}
/* x^a = 2 Re Tr(T^a X) for Hermitian X (Tr T^a T^b = delta^ab / 2) */
static void mat_to_alg(M3 X, double *x)
{
    for (int a = 0; a < 8; a++) x[a] = 2.0 * creal(m_tr(m_mul(GEN[a], X)));
}

/*
 * Proj[M]: the traceless Hermitian generator part of M, i.e. the paper's
 * "[M]_ah" of Sec. II.A and Sec. III.B read as a Hermitian algebra
 * element (reading: the printed anti-Hermitian part multiplied by -i, so
 * that Proj[exp(i eps X)] = eps X + O(eps^3)).
 */
static void proj(M3 M, double *x)
{
    M3 A = m_scale(m_sub(M, m_adj(M)), 0.5);          /* (M - M^+)/2 */
    cplx tr = m_tr(A) / 3.0;
    for (int i = 0; i < 3; i++) A.e[i][i] -= tr;       /* traceless  */
    M3 P = m_scale(A, -I);                              /* Hermitian  */
    mat_to_alg(P, x);
}

/* exp(A) by scaling and squaring of the Taylor series (definition of exp) */
static M3 m_exp(M3 A)
{
    double nrm = 0;
    for (int i = 0; i < 3; i++) {
        double r = 0;
        for (int j = 0; j < 3; j++) r += cabs(A.e[i][j]);
        if (r > nrm) nrm = r;
    }
    int s = 0;
    while (nrm > 0.5) { nrm *= 0.5; s++; }
    M3 B = m_scale(A, ldexp(1.0, -s));
    M3 sum = m_id(), term = m_id();
    for (int k = 1; k <= 24; k++) {
        term = m_scale(m_mul(term, B), 1.0 / k);
        sum = m_add(sum, term);
    }
    for (int k = 0; k < s; k++) sum = m_mul(sum, sum);
    return sum;
}
/* exp(i X) for X = x^a T^a */
static M3 expi_alg(const double *x, double scale)
{
    double y[8];
    for (int a = 0; a < 8; a++) y[a] = scale * x[a];
    return m_exp(m_scale(alg_to_mat(y), I));
}

/* inverse of a 3x3 complex matrix: adjugate over determinant */
static M3 m_inv(M3 a)
{
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            c.e[i][j] = a.e[i1][j1] * a.e[i2][j2] - a.e[i1][j2] * a.e[i2][j1];
        }
    const cplx det = a.e[0][0] * c.e[0][0] + a.e[0][1] * c.e[1][0] + a.e[0][2] * c.e[2][0];
    return m_scale(c, 1.0 / det);
}
static double m_dist(M3 a, M3 b)
{
    double d = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) d += cabs(a.e[i][j] - b.e[i][j]);
    return d;
}
/* principal square root (no eigenvalue on the negative real axis) by the
 * Denman-Beavers iteration Y <- (Y + Z^-1)/2, Z <- (Z + Y^-1)/2 from Y = M,
 * Z = 1: Y -> M^(1/2), Z -> M^(-1/2) */
static M3 m_sqrt(M3 M)
{
    M3 Y = M, Z = m_id();
    for (int k = 0; k < 100; k++) {
        M3 Yn = m_scale(m_add(Y, m_inv(Z)), 0.5);
        M3 Zn = m_scale(m_add(Z, m_inv(Y)), 0.5);
        const double d = m_dist(Yn, Y);
        Y = Yn;
        Z = Zn;
        if (d < 1e-17) break;
    }
    return Y;
}
/* principal logarithm by inverse scaling and squaring: log M = 2^s log(M^(1/2^s))
 * with square roots until M^(1/2^s) is within 0.05 of 1, then the series
 * log(1 + E) = E - E^2/2 + E^3/3 - ... */
static M3 m_log(M3 M)
{
    int s = 0;
    while (m_dist(M, m_id()) > 0.05 && s < 60) {
        M = m_sqrt(M);
        s++;
    }
    const M3 E = m_sub(M, m_id());
    M3 sum = m_zero(), pw = m_id();
    for (int k = 1; k <= 40; k++) {
        pw = m_mul(pw, E);
        sum = m_add(sum, m_scale(pw, (k % 2 ? 1.0 : -1.0) / k));
    }
    return m_scale(sum, ldexp(1.0, s));
}
/* components a^a of the Hermitian generator of a link: U = exp(i a^a T^a),
 * a = -i log U (principal branch; the trace part, nonzero only beyond the
 * branch of traceless generators, is dropped by the projection onto T^a) */
static void link_generator(M3 U, double *a)
{
    mat_to_alg(m_scale(m_log(U), -I), a);
}

/* Gram-Schmidt on rows 1 and 2, row 3 = conj(r1 x r2): a unitary matrix
 * with unit determinant.  Used as the starting point of the initial-link
 * solve (reading of the lattice initial condition, Sec. II.A). */
static M3 su3_project_rows(M3 W)
{
    M3 R = m_zero();
    double n0 = 0;
    for (int j = 0; j < 3; j++) n0 += creal(W.e[0][j] * conj(W.e[0][j]));
    n0 = sqrt(n0);
    for (int j = 0; j < 3; j++) R.e[0][j] = W.e[0][j] / n0;
    cplx ip = 0;
    for (int j = 0; j < 3; j++) ip += conj(R.e[0][j]) * W.e[1][j];
    double n1 = 0;
    for (int j = 0; j < 3; j++) {
        R.e[1][j] = W.e[1][j] - ip * R.e[0][j];
        n1 += creal(R.e[1][j] * conj(R.e[1][j]));
    }
    n1 = sqrt(n1);
    for (int j = 0; j < 3; j++) R.e[1][j] /= n1;
    R.e[2][0] = conj(R.e[0][1] * R.e[1][2] - R.e[0][2] * R.e[1][1]);
    R.e[2][1] = conj(R.e[0][2] * R.e[1][0] - R.e[0][0] * R.e[1][2]);
    R.e[2][2] = conj(R.e[0][0] * R.e[1][1] - R.e[0][1] * R.e[1][0]);
    return R;
}

/* --------------------------- lattice helpers --------------------------- */
static inline int nb(int s, int dx, int dy, int N)
{
    int x = s % N, y = s / N;
    x = ((x + dx) % N + N) % N;
    y = ((y + dy) % N + N) % N;
    return y * N + x;
}
static inline int step_dir(int s, int i, int sign, int N)
{
    return i == 0 ? nb(s, sign, 0, N) : nb(s, 0, sign, N);
}
static inline M3 link(const cplx *U, int N, int i, int s)
{
    M3 m;
    memcpy(&m, U + ((size_t)i * N * N + s) * 9, sizeof m);
    return m;
}
static inline void set_link(cplx *U, int N, int i, int s, M3 m)
{
    memcpy(U + ((size_t)i * N * N + s) * 9, &m, sizeof m);
}

/* plaquette U_ij(x) = U_i(x) U_j(x+i) U_i(x+j)^+ U_j(x)^+   (Sec. II.A) */
static M3 plaq(const cplx *U, int N, int i, int j, int s)
{
    return m_mul4(link(U, N, i, s), link(U, N, j, step_dir(s, i, +1, N)),
                  m_adj(link(U, N, i, step_dir(s, j, +1, N))), m_adj(link(U, N, j, s)));
}
/* U_{i,-j}(x) = U_i(x) U_j(x+i-j)^+ U_i(x-j)^+ U_j(x-j)   (Sec. II.A) */
static M3 plaq_ineg(const cplx *U, int N, int i, int j, int s)
{
    int xmj = step_dir(s, j, -1, N);
    int xpimj = step_dir(xmj, i, +1, N);
    return m_mul4(link(U, N, i, s), m_adj(link(U, N, j, xpimj)), m_adj(link(U, N, i, xmj)),
                  link(U, N, j, xmj));
}
/* forward transported scalar  phi->_i(x) = U_i(x) phi(x+i) U_i(x)^+ */
static M3 phi_fwd(const cplx *U, const double *phi, int N, int i, int s)
{
    M3 u = link(U, N, i, s);
    return m_mul3(u, alg_to_mat(phi + 8 * (size_t)step_dir(s, i, +1, N)), m_adj(u));
}
/* backward transported scalar phi<-_i(x) = U_i(x-i)^+ phi(x-i) U_i(x-i) */
static M3 phi_bwd(const cplx *U, const double *phi, int N, int i, int s)
{
    int xm = step_dir(s, i, -1, N);
    M3 u = link(U, N, i, xm);
    return m_mul3(m_adj(u), alg_to_mat(phi + 8 * (size_t)xm), u);
}

/* =====================================================================
 * Field equations (Sec. II.A, lattice equations of motion + leapfrog)
 * ===================================================================== */

/*
 * Kick forces at time t (both use U and phi at that time):
 *   F_E[i](x) = -t (Proj U_ij(x) + Proj U_{i,-j}(x)) + (1/t) i[phi->_i(x), phi(x)]
 *   F_pi(x)   = (1/t) sum_i ( phi->_i(x) + phi<-_i(x) - 2 phi(x) )
 * These are the lattice equations of motion of Sec. II.A (the
 * "d_tau P^i" and "d_tau P^eta" lines) in hat units, with [.]_ah read as
 * Proj and the transported scalar as written there.
 */
void orc_forces(int N, double t, const cplx *U, const double *phi, double *FE, double *Fpi)
{
    build_generators();
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        M3 ph = alg_to_mat(phi + 8 * (size_t)s);
        M3 lap = m_zero();
        for (int i = 0; i < 2; i++) {
            int j = 1 - i;
            double p1[8], p2[8], cm[8];
            proj(plaq(U, N, i, j, s), p1);
            proj(plaq_ineg(U, N, i, j, s), p2);
            M3 fw = phi_fwd(U, phi, N, i, s);
            M3 bw = phi_bwd(U, phi, N, i, s);
            M3 comm = m_scale(m_sub(m_mul(fw, ph), m_mul(ph, fw)), I);   /* i[phi->, phi] */
            mat_to_alg(comm, cm);
            for (int a = 0; a < 8; a++)
                FE[((size_t)i * V + s) * 8 + a] = -t * (p1[a] + p2[a]) + cm[a] / t;
            lap = m_add(lap, m_sub(m_add(fw, bw), m_scale(ph, 2.0)));
        }
        double l[8];
        mat_to_alg(lap, l);
        for (int a = 0; a < 8; a++) Fpi[(size_t)s * 8 + a] = l[a] / t;
    }
}

/* kick: E += dt*F_E, pi += dt*F_pi, forces from U, phi at time t (in place) */
void orc_kick(int N, double t, double dt, const cplx *U, const double *phi, double *E, double *pi)
{
    const size_t V = (size_t)N * N;
    double *FE = malloc(sizeof(double) * 16 * V);
    double *Fp = malloc(sizeof(double) * 8 * V);
    orc_forces(N, t, U, phi, FE, Fp);
    for (size_t k = 0; k < 16 * V; k++) E[k] += dt * FE[k];
    for (size_t k = 0; k < 8 * V; k++) pi[k] += dt * Fp[k];
    free(FE);
    free(Fp);
}

/*
 * drift at t_half: U_i <- exp(i (dt/t_half) E_i) U_i,  phi <- phi + dt t_half pi.
 * The link update follows from the definition of P^i through the time
 * derivative of the link (Sec. II.A); the scalar update from P^eta.
 */
void orc_drift(int N, double t_half, double dt, cplx *U, double *phi, const double *E, const double *pi)
{
    build_generators();
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        for (int i = 0; i < 2; i++) {
            M3 ex = expi_alg(E + ((size_t)i * V + s) * 8, dt / t_half);
            set_link(U, N, i, s, m_mul(ex, link(U, N, i, s)));
        }
        for (int a = 0; a < 8; a++) phi[(size_t)s * 8 + a] += dt * t_half * pi[(size_t)s * 8 + a];
    }
}

/*
 * One leapfrog step n -> n+1 (Sec. II.A: momenta at half-integer, fields
 * at integer times).  t_n = n dt.  At n = 0 the kick is skipped
 * (reading: E(1/2) = E(0) = 0 and pi(1/2) = pi(0), since both forces are
 * singular at tau = 0 while A_eta vanishes there).  When t_fixed > 0 every
 * time argument is replaced by t_fixed (frozen-time test mode).
 */
void orc_field_step(int N, int n, double dt, double t_fixed, cplx *U, double *phi, double *E, double *pi)
{
    double t = t_fixed > 0 ? t_fixed : n * dt;
    double th = t_fixed > 0 ? t_fixed : (n + 0.5) * dt;
    if (n > 0 || t_fixed > 0) orc_kick(N, t, dt, U, phi, E, pi);
    orc_drift(N, th, dt, U, phi, E, pi);
}

/*
 * Lattice Hamiltonian at time t (the energy whose variations give the
 * kick forces above):
 *   out[0] = (1/t) sum_x sum_i Tr E_i^2      (transverse electric)
 *   out[1] = t sum_x Tr pi^2                 (longitudinal electric)
 *   out[2] = 2 t sum_x Re Tr(1 - U_12(x))    (longitudinal magnetic)
 *   out[3] = (1/t) sum_x sum_i Tr(phi->_i - phi)^2  (transverse magnetic)
 */
void orc_energy(int N, double t, const cplx *U, const double *phi, const double *E, const double *pi, double *out)
{
    build_generators();
    const int V = N * N;
    double kt = 0, kl = 0, vb = 0, vp = 0;
    for (int s = 0; s < V; s++) {
        for (int i = 0; i < 2; i++)
            for (int a = 0; a < 8; a++) {
                double e = E[((size_t)i * V + s) * 8 + a];
                kt += 0.5 * e * e;
            }
        for (int a = 0; a < 8; a++) kl += 0.5 * pi[(size_t)s * 8 + a] * pi[(size_t)s * 8 + a];
        vb += 2.0 * creal(3.0 - m_tr(plaq(U, N, 0, 1, s)));
        M3 ph = alg_to_mat(phi + 8 * (size_t)s);
        for (int i = 0; i < 2; i++) {
            M3 d = m_sub(phi_fwd(U, phi, N, i, s), ph);
            vp += creal(m_tr(m_mul(d, d)));
        }
    }
    out[0] = kt / t;
    out[1] = kl * t;
    out[2] = vb * t;
    out[3] = vp / t;
}

/*
 * Gauss constraint residual G(x) = sum_i [E_i(x) - U_i(x-i)^+ E_i(x-i) U_i(x-i)]
 *                                 + i [phi(x), pi(x)]
 * (the constraint stated with the Yang-Mills equations in Sec. II, in
 * lattice form with backward covariant differences).
 */
void orc_gauss(int N, const cplx *U, const double *phi, const double *E, const double *pi, double *G)
{
    build_generators();
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        M3 g = m_zero();
        for (int i = 0; i < 2; i++) {
            int xm = step_dir(s, i, -1, N);
            M3 u = link(U, N, i, xm);
            M3 e_here = alg_to_mat(E + ((size_t)i * V + s) * 8);
            M3 e_back = m_mul3(m_adj(u), alg_to_mat(E + ((size_t)i * V + xm) * 8), u);
            g = m_add(g, m_sub(e_here, e_back));
        }
        M3 ph = alg_to_mat(phi + 8 * (size_t)s), pp = alg_to_mat(pi + 8 * (size_t)s);
        g = m_add(g, m_scale(m_sub(m_mul(ph, pp), m_mul(pp, ph)), I));
        mat_to_alg(g, G + 8 * (size_t)s);
    }
}

/* max over links of ||U U^+ - 1||_max and |det U - 1| */
void orc_unitarity(int N, const cplx *U, double *out)
{
    double mu = 0, md = 0;
    for (int i = 0; i < 2; i++)
        for (int s = 0; s < N * N; s++) {
            M3 u = link(U, N, i, s);
            M3 d = m_sub(m_mul(u, m_adj(u)), m_id());
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++)
                    if (cabs(d.e[r][c]) > mu) mu = cabs(d.e[r][c]);
            cplx det = u.e[0][0] * (u.e[1][1] * u.e[2][2] - u.e[1][2] * u.e[2][1])
                     - u.e[0][1] * (u.e[1][0] * u.e[2][2] - u.e[1][2] * u.e[2][0])
                     + u.e[0][2] * (u.e[1][0] * u.e[2][1] - u.e[1][1] * u.e[2][0]);
            if (cabs(det - 1) > md) md = cabs(det - 1);
        }
    out[0] = mu;
    out[1] = md;
}

/* =====================================================================
 * Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror,
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * ===================================================================== */
void orc_philox(const uint64_t *ctr_in, const uint64_t *key_in, uint64_t *out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
/* uniform in [0,1) and in (0,1] from the top 53 bits */
static double u01_open1(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
static double u01_open0(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }
/* Box-Muller: two normals from two words */
static void box_muller(uint64_t ra, uint64_t rb, double *z0, double *z1)
{
    double rad = sqrt(-2.0 * log(u01_open0(ra)));
    double ang = 2.0 * M_PI * u01_open1(rb);
    *z0 = rad * cos(ang);
    *z1 = rad * sin(ang);
}
/* four normals from one Philox block */
static void normals4(const uint64_t *ctr, const uint64_t *key, double *z)
{
    uint64_t r[4];
    orc_philox(ctr, key, r);
    box_muller(r[0], r[1], &z[0], &z[1]);
    box_muller(r[2], r[3], &z[2], &z[3]);
}

/* =====================================================================
 * MV-model initial condition (Sec. II and II.A)
 * ===================================================================== */

/*
 * Colour charges of one sheet of one nucleus: Gaussian, zero mean, variance
 * sigma^2 = (g^2 mu a)^2 / N_s per site and colour (the sheet-regularised
 * MV correlator [eq:MVchargecorrnum], with the transverse delta read as a
 * Kronecker delta over lattice sites).  Stream layout: key = (seed,
 * 1 + nucleus), counter = (site, sheet, block, 0), block b gives colours
 * 4b..4b+3.
 */
void orc_mv_charges(int N, uint64_t seed, int nucleus, int sheet, double sigma, double *rho)
{
    const int V = N * N;
    uint64_t key[2] = {seed, (uint64_t)(1 + nucleus)};
    for (int s = 0; s < V; s++)
        for (int b = 0; b < 2; b++) {
            uint64_t ctr[4] = {(uint64_t)s, (uint64_t)sheet, (uint64_t)b, 0};
            double z[4];
            normals4(ctr, key, z);
            for (int j = 0; j < 4; j++) rho[(size_t)s * 8 + 4 * b + j] = sigma * z[j];
        }
}

/* Vdag(x) <- Vdag(x) exp(-i alpha_n(x)): the sheet product of Sec. II.A,
 * sheet 1 leftmost, applied one sheet at a time in order. */
void orc_wilson_mult(int N, const double *alpha, cplx *Vdag)
{
    build_generators();
    const int V = N * N;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < V; s++) {
        M3 v;
        memcpy(&v, Vdag + (size_t)s * 9, sizeof v);
        v = m_mul(v, expi_alg(alpha + (size_t)s * 8, -1.0));
        memcpy(Vdag + (size_t)s * 9, &v, sizeof v);
    }
}

/* pure-gauge links of one nucleus U^X_i(x) = V(x) V(x+i)^+  [eq:puregaugefields] */
void orc_pure_gauge(int N, const cplx *Vdag, cplx *UX)
{
    const int V = N * N;
    for (int i = 0; i < 2; i++)
        for (int s = 0; s < V; s++) {
            M3 vd_here, vd_next;
            memcpy(&vd_here, Vdag + (size_t)s * 9, sizeof(M3));
            memcpy(&vd_next, Vdag + (size_t)step_dir(s, i, +1, N) * 9, sizeof(M3));
            set_link(UX, N, i, s, m_mul(m_adj(vd_here), vd_next));
        }
}

/* solve J x = b (8x8) by Gaussian elimination with partial pivoting */
static int solve8(double J[8][8], double *b, double *x)
{
    for (int c = 0; c < 8; c++) {
        int p = c;
        for (int r = c + 1; r < 8; r++)
            if (fabs(J[r][c]) > fabs(J[p][c])) p = r;
        if (J[p][c] == 0) return -1;
        if (p != c) {
            for (int k = 0; k < 8; k++) { double t = J[c][k]; J[c][k] = J[p][k]; J[p][k] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < 8; r++) {
            double f = J[r][c] / J[c][c];
            for (int k = c; k < 8; k++) J[r][k] -= f * J[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 7; r >= 0; r--) {
        double acc = b[r];
        for (int k = r + 1; k < 8; k++) acc -= J[r][k] * x[k];
        x[r] = acc / J[r][r];
    }
    return 0;
}

/*
 * Glasma links at tau = 0.  Reading of the lattice form of the continuum
 * condition A^i = alpha^i_A + alpha^i_B [eq:Glasmainitcond]: for every link
 * solve Proj[(U^A + U^B)(1 + U^+)] = 0 for U in SU(3) by Newton's method in
 * the 8 coordinates of U = exp(i X) U_0, starting from the row-projected
 * U^A + U^B.  Jacobian J^ab = Proj^a[-i W U^+ T^b], W = U^A + U^B.
 * Returns the number of links that did not converge; *max_iter receives
 * the largest iteration count.
 */
int orc_kv_links(int N, const cplx *UA, const cplx *UB, cplx *U, double tol, int maxit, int *max_iter)
{
    build_generators();
    const int V = N * N;
    int fails = 0, worst = 0;
    for (int i = 0; i < 2; i++)
        for (int s = 0; s < V; s++) {
            M3 W = m_add(link(UA, N, i, s), link(UB, N, i, s));
            M3 u = su3_project_rows(W);
            int it, ok = 0;
            for (it = 0; it < maxit; it++) {
                double F[8];
                proj(m_mul(W, m_add(m_id(), m_adj(u))), F);
                double fmax = 0;
                for (int a = 0; a < 8; a++) if (fabs(F[a]) > fmax) fmax = fabs(F[a]);
                if (fmax < tol) { ok = 1; break; }
                double J[8][8];
                M3 WUd = m_mul(W, m_adj(u));
                for (int b = 0; b < 8; b++) {
                    double col[8];
                    proj(m_scale(m_mul(WUd, GEN[b]), -I), col);
                    for (int a = 0; a < 8; a++) J[a][b] = col[a];
                }
                double rhs[8], X[8];
                for (int a = 0; a < 8; a++) rhs[a] = -F[a];
                if (solve8(J, rhs, X)) break;
                u = m_mul(expi_alg(X, 1.0), u);
                double xmax = 0;
                for (int a = 0; a < 8; a++) if (fabs(X[a]) > xmax) xmax = fabs(X[a]);
                if (xmax < 1e-15) { ok = 1; it++; break; }   /* at the rounding floor */
            }
            if (!ok) fails++;
            if (it > worst) worst = it;
            set_link(U, N, i, s, u);
        }
    if (max_iter) *max_iter = worst;
    return fails;
}

/*
 * Longitudinal electric field at tau = 0 (reading of the lattice form of
 * A^eta(0) = (ig/2)[alpha^i_A, alpha^i_B] [eq:Glasmainitcond] together with
 * P^eta = (1/tau) d_tau A_eta and A_eta = -tau^2 A^eta):
 *   pi(x) = (1/2) sum_i Proj[ (U_i(x) - 1)(U^B_i(x)^+ - U^A_i(x)^+)
 *                            + (U_i(x-i)^+ - 1)(U^B_i(x-i) - U^A_i(x-i)) ]
 * whose weak-field limit is -i sum_i [alpha^i_A, alpha^i_B] (averaged over
 * the two links that meet at x).
 */
void orc_pi0(int N, const cplx *UA, const cplx *UB, const cplx *U, double *pi)
{
    build_generators();
    const int V = N * N;
    for (int s = 0; s < V; s++) {
        M3 acc = m_zero();
        for (int i = 0; i < 2; i++) {
            int xm = step_dir(s, i, -1, N);
            M3 t1 = m_mul(m_sub(link(U, N, i, s), m_id()),
                          m_sub(m_adj(link(UB, N, i, s)), m_adj(link(UA, N, i, s))));
            M3 t2 = m_mul(m_sub(m_adj(link(U, N, i, xm)), m_id()),
                          m_sub(link(UB, N, i, xm), link(UA, N, i, xm)));
            acc = m_add(acc, m_add(t1, t2));
        }
        double p[8];
        proj(acc, p);
        for (int a = 0; a < 8; a++) pi[(size_t)s * 8 + a] = 0.5 * p[a];
    }
}

/* =====================================================================
 * Test particles (Sec. III.B, Sec. IV.B)
 * ===================================================================== */

/* particle record columns */
enum { P_X = 0, P_Y, P_ETA, P_PX, P_PY, P_PETA, P_Q, P_CX = 14, P_CY, P_DETA, P_UX0, P_UY0, P_PT0, P_NCOL };

/*
 * Initial colour vector Q_0 with the classical Casimirs of Sec. IV
 * [eq:q23_main]: fundamental q2 = 4, q3 = 10/3 (only Q^5 and Q^8 nonzero,
 * as printed in [eq:initq0]; here Q^8 is the exact root of
 * Q8^3 - 12 Q8 - 20/sqrt(3) = 0 nearest the printed value and
 * Q^5 = -sqrt(4 - Q8^2)); adjoint Q^1 = sqrt(24), q3 = 0.
 */
void orc_q0(int rep, double *q0)
{
    for (int a = 0; a < 8; a++) q0[a] = 0;
    if (rep == 1) { q0[0] = sqrt(24.0); return; }
    /* depressed cubic t^3 + p t + q = 0, three real roots (trigonometric form) */
    double p = -12.0, q = -20.0 / sqrt(3.0);
    double best = 0, bestd = 1e300;
    for (int k = 0; k < 3; k++) {
        double r = 2.0 * sqrt(-p / 3.0) *
                   cos(acos(1.5 * q / p * sqrt(-3.0 / p)) / 3.0 - 2.0 * M_PI * k / 3.0);
        double d = fabs(r - (-1.06209));
        if (d < bestd) { bestd = d; best = r; }
    }
    q0[7] = best;
    q0[4] = -sqrt(4.0 - best * best);
}

/* q2 = Q^a Q^a and q3 = d_abc Q^a Q^b Q^c = 4 Tr(Q^3) (Appendix A.2) */
void orc_casimirs(const double *Q, double *q2, double *q3)
{
    build_generators();
    double s = 0;
    for (int a = 0; a < 8; a++) s += Q[a] * Q[a];
    M3 q = alg_to_mat(Q);
    *q2 = s;
    *q3 = 4.0 * creal(m_tr(m_mul3(q, q, q)));
}

/*
 * Particle initial conditions (toy model of Sec. III.B; colour charges by
 * the Haar measure, Sec. IV.B).  Stream: key = (seed, 3),
 * counter = (particle, block, 0, 0).  Block 0: x, y uniform in [0,N),
 * azimuth uniform in [0, 2 pi) (or 0 when !azimuth_uniform), p_T uniform
 * in [pt_min, pt_max).  Blocks 1..5: 18 normals, the real and imaginary
 * parts of a 3x3 complex Ginibre matrix Z (entry (r,c) uses normals
 * 2(3r+c) and 2(3r+c)+1).  The Haar-random unitary is the Gram-Schmidt
 * orthonormalisation of the columns of Z (R has positive diagonal, so no
 * phase fix is needed); Q = U Q_0 U^+ and Q^a = 2 Tr(T^a Q).
 */
void orc_particles_init(int N, int np, uint64_t seed, double pt_min, double pt_max, int azimuth_uniform,
                        int rep, double *P)
{
    build_generators();
    double q0[8];
    orc_q0(rep, q0);
    M3 Q0 = alg_to_mat(q0);
    uint64_t key[2] = {seed, 3};
    for (int p = 0; p < np; p++) {
        double *r = P + (size_t)p * P_NCOL;
        uint64_t c0[4] = {(uint64_t)p, 0, 0, 0}, w[4];
        orc_philox(c0, key, w);
        r[P_X] = N * u01_open1(w[0]);
        r[P_Y] = N * u01_open1(w[1]);
        double phi0 = azimuth_uniform ? 2.0 * M_PI * u01_open1(w[2]) : 0.0;
        double pt = pt_min + (pt_max - pt_min) * u01_open1(w[3]);
        double z[20];
        for (int b = 1; b <= 5; b++) {
            uint64_t cb[4] = {(uint64_t)p, (uint64_t)b, 0, 0};
            normals4(cb, key, z + 4 * (b - 1));
        }
        cplx Z[3][3];
        for (int rr = 0; rr < 3; rr++)
            for (int cc = 0; cc < 3; cc++) Z[rr][cc] = z[2 * (3 * rr + cc)] + I * z[2 * (3 * rr + cc) + 1];
        /* modified Gram-Schmidt on the columns */
        M3 Uh = m_zero();
        for (int k = 0; k < 3; k++) {
            cplx v[3] = {Z[0][k], Z[1][k], Z[2][k]};
            for (int j = 0; j < k; j++) {
                cplx ip = 0;
                for (int rr = 0; rr < 3; rr++) ip += conj(Uh.e[rr][j]) * v[rr];
                for (int rr = 0; rr < 3; rr++) v[rr] -= ip * Uh.e[rr][j];
            }
            double nrm = 0;
            for (int rr = 0; rr < 3; rr++) nrm += creal(v[rr] * conj(v[rr]));
            nrm = sqrt(nrm);
            for (int rr = 0; rr < 3; rr++) Uh.e[rr][k] = v[rr] / nrm;
        }
        double q[8];
        mat_to_alg(m_mul3(Uh, Q0, m_adj(Uh)), q);
        r[P_ETA] = 0;
        r[P_PX] = pt * cos(phi0);
        r[P_PY] = pt * sin(phi0);
        r[P_PETA] = 0;
        for (int a = 0; a < 8; a++) r[P_Q + a] = q[a];
        r[P_CX] = fmod(floor(r[P_X] + 0.5), N);
        r[P_CY] = fmod(floor(r[P_Y] + 0.5), N);
        r[P_DETA] = 0;
        r[P_UX0] = cos(phi0);
        r[P_UY0] = sin(phi0);
        r[P_PT0] = pt;
    }
}

/*
 * Colour fields at lattice site c at time t_n (Sec. III.B, the interpolations
 * that are second order in lattice and time spacing), hat units g a^2 F:
 *   out[0],out[1] = E_1, E_2:
 *     (1/(4t)) [E_i(c,n+1/2) + E_i(c,n-1/2) + U_i(c-i)^+ (E_i(c-i,n+1/2)+E_i(c-i,n-1/2)) U_i(c-i)]
 *   out[2] = E_eta = (pi(c,n+1/2) + pi(c,n-1/2)) / 2
 *   out[3] = B_1 = -(1/(2t)) [phi->_2(c) - phi<-_2(c)]
 *   out[4] = B_2 = +(1/(2t)) [phi->_1(c) - phi<-_1(c)]
 *     (reading: B_i = eps_ij F_{eta j}/tau as defined in [eq:glasmafields_main];
 *      the printed interpolation carries the same index on both sides)
 *   out[5] = B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}](c)
 * At n == 0 (t = 0): E_i = 0, E_eta = pi(c, 1/2), B_i = 0, B_eta as above
 * (reading for particles formed at tau = 0).
 */
void orc_particle_fields(int N, int n, double dt, int s, const cplx *U, const double *phi, const double *E_old,
                         const double *E_new, const double *pi_old, const double *pi_new, double *out)
{
    build_generators();
    const int V = N * N;
    double t = n * dt;
    memset(out, 0, sizeof(double) * 48);
    for (int i = 0; i < 2; i++) {
        if (n == 0) break;
        int xm = step_dir(s, i, -1, N);
        M3 u = link(U, N, i, xm);
        double here[8], back[8];
        for (int a = 0; a < 8; a++) {
            here[a] = E_new[((size_t)i * V + s) * 8 + a] + E_old[((size_t)i * V + s) * 8 + a];
            back[a] = E_new[((size_t)i * V + xm) * 8 + a] + E_old[((size_t)i * V + xm) * 8 + a];
        }
        M3 tot = m_add(alg_to_mat(here), m_mul3(m_adj(u), alg_to_mat(back), u));
        double e[8];
        mat_to_alg(tot, e);
        for (int a = 0; a < 8; a++) out[8 * i + a] = e[a] / (4.0 * t);
    }
    for (int a = 0; a < 8; a++)
        out[16 + a] = n == 0 ? pi_new[(size_t)s * 8 + a]
                             : 0.5 * (pi_new[(size_t)s * 8 + a] + pi_old[(size_t)s * 8 + a]);
    if (n > 0) {
        double b[8];
        mat_to_alg(m_sub(phi_fwd(U, phi, N, 1, s), phi_bwd(U, phi, N, 1, s)), b);
        for (int a = 0; a < 8; a++) out[24 + a] = -b[a] / (2.0 * t);
        mat_to_alg(m_sub(phi_fwd(U, phi, N, 0, s), phi_bwd(U, phi, N, 0, s)), b);
        for (int a = 0; a < 8; a++) out[32 + a] = b[a] / (2.0 * t);
    }
    /* clover of four counter-clockwise plaquettes around c */
    int xm1 = nb(s, -1, 0, N), xm2 = nb(s, 0, -1, N), xm1m2 = nb(s, -1, -1, N);
    int xp1 = nb(s, 1, 0, N), xp2 = nb(s, 0, 1, N), xm1p2 = nb(s, -1, 1, N), xp1m2 = nb(s, 1, -1, N);
    M3 c12 = m_mul4(link(U, N, 0, s), link(U, N, 1, xp1), m_adj(link(U, N, 0, xp2)), m_adj(link(U, N, 1, s)));
    M3 c2m1 = m_mul4(link(U, N, 1, s), m_adj(link(U, N, 0, xm1p2)), m_adj(link(U, N, 1, xm1)), link(U, N, 0, xm1));
    M3 cm1m2 = m_mul4(m_adj(link(U, N, 0, xm1)), m_adj(link(U, N, 1, xm1m2)), link(U, N, 0, xm1m2), link(U, N, 1, xm2));
    M3 cm21 = m_mul4(m_adj(link(U, N, 1, xm2)), link(U, N, 0, xm2), link(U, N, 1, xp1m2), m_adj(link(U, N, 0, s)));
    double bz[8];
    proj(m_add(m_add(c12, c2m1), m_add(cm1m2, cm21)), bz);
    for (int a = 0; a < 8; a++) out[40 + a] = -0.25 * bz[a];
}

static double dot8(const double *a, const double *b)
{
    double s = 0;
    for (int k = 0; k < 8; k++) s += a[k] * b[k];
    return s;
}
/* Q <- A^+ Q A  on the component vector */
static void rotate_q(double *Q, M3 A)
{
    double q[8];
    mat_to_alg(m_mul3(m_adj(A), alg_to_mat(Q), A), q);
    memcpy(Q, q, sizeof q);
}

/*
 * One particle step at time t_n, n >= n_form (Sec. III.B).
 *  1. CPIC colour rotation for the move n-1 -> n (only for n > n_form), with
 *     links and A_eta at t_n [eq:colorrotnum]: for each transverse axis in
 *     turn (x first, then y) a +1 change of the nearest grid point gives
 *     Q <- U_i(c)^+ Q U_i(c), a -1 change Q <- U_i(c-i) Q U_i(c-i)^+; then
 *     Q <- W^+ Q W with W = exp(i deta phi(c')).
 *  2. Fields at the new nearest grid point c' at t_n.
 *  3. Explicit Euler step of [eq:wongpos] and [eq:wonginmilne], with
 *     p^tau from its constraint, Q.X = Q^a X^a (g/T_R Tr(Q X) with T_R of
 *     the 3x3 matrices, i.e. 2 Tr(Q X)):
 *       p^x   += dt (e_x + b_eta v_y - b_y v_L)
 *       p^y   += dt (e_y - b_eta v_x + b_x v_L)
 *       p^eta += dt (1/t) (e_eta - b_x v_y + b_y v_x - 2 p^eta)   (skipped at t = 0)
 *       x += dt v_x, y += dt v_y, eta += dt p^eta/p^tau, periodic wrap.
 * Static branch (infinite mass, the limit of Sec. V.A): no motion and no
 * rotation; p^x, p^y, p^z += dt (e_x, e_y, e_eta), p^z kept in the p^eta column.
 *
 * color_mode 1 replaces the colour rotation of step 1 by the alternative of
 * Sec. III.B: the charge follows dQ/dt = i[Q, A_x v_x + A_y v_y + phi v_eta]
 * with the gauge fields taken from the links by the matrix logarithm,
 * a A_i(x + i/2) = -i log U_i(x) (hat units), stepped by explicit Euler with
 * the rest of the particle's variables (reading): Q_{n+1} = Q_n + dt i[Q_n, M_n].
 * A_x is taken on the x link whose midpoint is nearest to the particle,
 * (floor(x), NGP row), A_y on the y link at (NGP column, floor(y)), phi at
 * the nearest grid point, all at t_n; v_eta = p^eta / p^tau.
 *
 * ptau_ode (may be NULL; moving particles only): p^tau integrated from its own
 * equation of motion [eq:ptaueq] instead of the constraint [eq:ptau], the
 * temporal-constraint check of Appendix D.  In hat units
 *   dp^tau/dt = -t (p^eta)^2 / p^tau
 *               + (e_eta t p^eta + e_x p^x + e_y p^y) / p^tau,
 * Euler-stepped with the rest of the particle (the same charges, fields and
 * momenta at n; p^tau on the right-hand side is the integrated value).  At
 * the formation step it starts from the constraint.
 *
 * Returns the number of particles whose grid point moved by more than one
 * cell along an axis (an error).
 */
int orc_particles_step(int N, int n, int n_form, double dt, double mhat, int is_static, int color_mode,
                       const cplx *U, const double *phi, const double *E_old, const double *E_new,
                       const double *pi_old, const double *pi_new, int np, double *P, double *ptau_ode)
{
    build_generators();
    int errors = 0;
    double t = n * dt;
#pragma omp parallel for schedule(static) reduction(+ : errors)
    for (int p = 0; p < np; p++) {
        double *r = P + (size_t)p * P_NCOL;
        double f[48];
        if (is_static) {
            int s = (int)r[P_CY] * N + (int)r[P_CX];
            orc_particle_fields(N, n, dt, s, U, phi, E_old, E_new, pi_old, pi_new, f);
            r[P_PX] += dt * dot8(r + P_Q, f + 0);
            r[P_PY] += dt * dot8(r + P_Q, f + 8);
            r[P_PETA] += dt * dot8(r + P_Q, f + 16);
            continue;
        }
        int cx = (int)r[P_CX], cy = (int)r[P_CY];
        int nx = ((int)floor(r[P_X] + 0.5)) % N, ny = ((int)floor(r[P_Y] + 0.5)) % N;
        if (n > n_form) {
            const int rotate = color_mode == 0;
            int d[2] = {nx - cx, ny - cy};
            for (int ax = 0; ax < 2; ax++) {
                if (d[ax] > N / 2) d[ax] -= N;
                if (d[ax] < -N / 2) d[ax] += N;
                int c = cy * N + cx;
                if (d[ax] == 1) {
                    if (rotate) rotate_q(r + P_Q, link(U, N, ax, c));
                } else if (d[ax] == -1) {
                    if (rotate) rotate_q(r + P_Q, m_adj(link(U, N, ax, step_dir(c, ax, -1, N))));
                } else if (d[ax] != 0) {
                    errors++;
                }
                if (ax == 0) cx = nx; else cy = ny;
            }
            if (rotate) rotate_q(r + P_Q, expi_alg(phi + 8 * (size_t)(ny * N + nx), r[P_DETA]));
        }
        int s = ny * N + nx;
        orc_particle_fields(N, n, dt, s, U, phi, E_old, E_new, pi_old, pi_new, f);
        const double *Q = r + P_Q;
        double e1 = dot8(Q, f), e2 = dot8(Q, f + 8), ee = dot8(Q, f + 16);
        double b1 = dot8(Q, f + 24), b2 = dot8(Q, f + 32), be = dot8(Q, f + 40);
        double px = r[P_PX], py = r[P_PY], pe = r[P_PETA];
        double ptau = sqrt(px * px + py * py + (t * pe) * (t * pe) + mhat * mhat);
        double v1 = px / ptau, v2 = py / ptau, vl = t * pe / ptau;
        if (ptau_ode) {
            if (n == n_form) ptau_ode[p] = ptau;
            const double pt = ptau_ode[p];
            ptau_ode[p] = pt + dt * (-t * pe * pe + ee * t * pe + e1 * px + e2 * py) / pt;
        }
        if (color_mode == 1) {
            /* Q_{n+1} = Q_n + dt i[Q_n, M_n], from the state at n */
            const int lx = ((int)floor(r[P_X])) % N, ly = ((int)floor(r[P_Y])) % N;
            double gx[8], gy[8], M[8], dq[8];
            link_generator(link(U, N, 0, ny * N + lx), gx);
            link_generator(link(U, N, 1, ly * N + nx), gy);
            const double veta = pe / ptau;
            for (int a = 0; a < 8; a++) M[a] = v1 * gx[a] + v2 * gy[a] + veta * phi[(size_t)(ny * N + nx) * 8 + a];
            const M3 Qm = alg_to_mat(Q), Mm = alg_to_mat(M);
            mat_to_alg(m_scale(m_sub(m_mul(Qm, Mm), m_mul(Mm, Qm)), I), dq);
            for (int a = 0; a < 8; a++) r[P_Q + a] += dt * dq[a];
        }
        r[P_PX] = px + dt * (e1 + be * v2 - b2 * vl);
        r[P_PY] = py + dt * (e2 - be * v1 + b1 * vl);
        if (n > 0) r[P_PETA] = pe + dt * (ee - b1 * v2 + b2 * v1 - 2.0 * pe) / t;
        double x = r[P_X] + dt * v1, y = r[P_Y] + dt * v2;
        if (x >= N) x -= N; else if (x < 0) x += N;
        if (y >= N) y -= N; else if (y < 0) y += N;
        r[P_X] = x;
        r[P_Y] = y;
        r[P_DETA] = dt * pe / ptau;
        r[P_ETA] += r[P_DETA];
        r[P_CX] = nx;
        r[P_CY] = ny;
    }
    return errors;
}

/*
 * Momentum broadening sums at time t [eq:mombroad], summed over particles
 * in index order:
 *   out[0] = sum dp_T^2 = sum (p_x^2 + p_y^2 - p_T(form)^2)
 *   out[1] = sum dp_L^2 = sum p_z^2, p^z = p^tau sinh(eta) + t p^eta cosh(eta)
 *            (lab-frame longitudinal momentum; zero at formation)
 *   out[2] = sum (p_par^2 - p_T(form)^2) along the initial direction
 *   out[3] = sum p_perp^2 across it
 * For the static branch p_z is the tracked value.
 */
void orc_particles_observe(double t, double mhat, int is_static, int np, const double *P, double *out)
{
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int p = 0; p < np; p++) {
        const double *r = P + (size_t)p * P_NCOL;
        double px = r[P_PX], py = r[P_PY], pz;
        if (is_static) {
            pz = r[P_PETA];
        } else {
            double pe = r[P_PETA];
            double ptau = sqrt(px * px + py * py + (t * pe) * (t * pe) + mhat * mhat);
            pz = ptau * sinh(r[P_ETA]) + t * pe * cosh(r[P_ETA]);
        }
        double par = px * r[P_UX0] + py * r[P_UY0];
        double perp = -px * r[P_UY0] + py * r[P_UX0];
        double pt02 = r[P_PT0] * r[P_PT0];
        s0 += px * px + py * py - pt02;
        s1 += pz * pz;
        s2 += par * par - pt02;
        s3 += perp * perp;
    }
    out[0] = s0; out[1] = s1; out[2] = s2; out[3] = s3;
}

/*
 * Light-like jet limit (Sec. V.B, [eq:mombroadjets]): one step of the
 * integral of the transported Lorentz force along straight paths in +x at the
 * speed of light, one path per lattice site, formed at step n_form.
 *
 * Path p = y*N + i starts at x = i + x_off in row y.  After m = n - n_form
 * steps it is at x = i + x_off + m dt, so its nearest grid point is
 * i + k(m) with k(m) = floor(x_off + m dt + 1/2) (mod N).
 *   - m = 0: W = 1, F = 0.
 *   - Wilson line (reading): when the nearest grid point moves from c to
 *     c + x, W <- W U_x(c), with the link at t_n.  W is then the ordered
 *     product of the x links crossed so far, and Tr(Q_0 W f W^+) is the
 *     force that a charge carried along by the colour rotation of Sec. III.B
 *     feels (f~ = W f W^+).
 *   - Force components for velocity +x, at the nearest grid point c, from
 *     the fields of orc_particle_fields:
 *       f_x = E_x,  f_y = E_y - B_eta,  f_z = E_eta + B_y.
 *   - The time integral is a sum over the steps with m % stride == 0, each
 *     weighted by stride * dt (stride = 1: every step, like the Euler push;
 *     stride = 1/dt: steps of one lattice spacing).
 * W: [V][3][3] complex, F: [V][3][8] (f_x, f_y, f_z components).
 * Requires dt <= 1 (at most one cell per step).
 */
void orc_jet_step(int N, int n, int n_form, double dt, double x_off, int stride, const cplx *U, const double *phi,
                  const double *E_old, const double *E_new, const double *pi_old, const double *pi_new, cplx *W,
                  double *F)
{
    build_generators();
    const int V = N * N;
    const int m = n - n_form;
    if (m < 0) return;
    const long k = (long)floor(x_off + m * dt + 0.5);
    const long kp = m > 0 ? (long)floor(x_off + (m - 1) * dt + 0.5) : k;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < V; p++) {
        const int i = p % N, y = p / N;
        M3 *w = (M3 *)(W + (size_t)p * 9);
        double *Fp = F + (size_t)p * 24;
        if (m == 0) {
            *w = m_id();
            memset(Fp, 0, sizeof(double) * 24);
        } else if (k != kp) {
            const int c_old = y * N + (int)(((i + kp) % N + N) % N);
            *w = m_mul(*w, link(U, N, 0, c_old));
        }
        if (m % stride != 0) continue;
        const int c = y * N + (int)(((i + k) % N + N) % N);
        double f[48];
        orc_particle_fields(N, n, dt, c, U, phi, E_old, E_new, pi_old, pi_new, f);
        double comp[3][8];
        for (int a = 0; a < 8; a++) {
            comp[0][a] = f[a];
            comp[1][a] = f[8 + a] - f[40 + a];
            comp[2][a] = f[16 + a] + f[32 + a];
        }
        for (int j = 0; j < 3; j++) {
            double ft[8];
            mat_to_alg(m_mul3(*w, alg_to_mat(comp[j]), m_adj(*w)), ft);
            for (int a = 0; a < 8; a++) Fp[8 * j + a] += stride * dt * ft[a];
        }
    }
}

/* number of OpenMP threads of the oracle's parallel loops (CPU baseline timing) */
#include <omp.h>
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------- exports used only by the oracle's own pins ------------------- */
/* T^a as 3x3 complex, row-major (a = 0..7) */
void orc_generator(int a, cplx *out)
{
    build_generators();
    memcpy(out, &GEN[a], sizeof(M3));
}
/* Proj[M] components */
void orc_proj(const cplx *M, double *out)
{
    build_generators();
    M3 m;
    memcpy(&m, M, sizeof m);
    proj(m, out);
}
/* components of -i log U (principal logarithm) */
void orc_link_generator(const cplx *U, double *out)
{
    build_generators();
    M3 m;
    memcpy(&m, U, sizeof m);
    link_generator(m, out);
}
/* exp(i scale x^a T^a) */
void orc_expi(const double *x, double scale, cplx *out)
{
    build_generators();
    M3 m = expi_alg(x, scale);
    memcpy(out, &m, sizeof m);
}
