/*
 * Plain FP64 CPU oracle of one D2Q9 pseudopotential MRT lattice Boltzmann
 * timestep, after Shan, Zhu, Yao, Yin and Jiang, "Pseudopotential MRT lattice
 * Boltzmann model for cavitation bubble collapse with high density ratio"
 * (arXiv:1605.01800).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Precision: IEEE binary64, built with -ffp-contract=off, fixed loop order.
 *
 * Layout (this file's own): f[(y*nx + x)*9 + a], fields g[y*nx + x].
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - D2Q9 velocity order: rest, 4 axis directions, 4 diagonals, so that the
 *     force weights of Eq. 7 are w_1..4 = 1/3 and w_5..8 = 1/12.
 *   - M is not printed; the paper calls it orthogonal and Eq. 4 fixes the
 *     moment order (rho, e, zeta, jx, qx, jy, qy, pxx, pxy).  The rows used are
 *     the usual orthogonal D2Q9 set with that order.  M^-1 is obtained by
 *     Gauss-Jordan elimination, not from a hand-derived closed form.
 *   - Eq. 15 is used with eta = b*rho/4 as printed; the caller passes b = 4,
 *     which is the value that reproduces the densities printed in Section 3.2.
 *   - Solid nodes of the halfway bounce-back walls take the pseudopotential of
 *     the adjacent fluid row (mirror), for the neighbour sum of Eq. 7.
 *   - Initial populations are w_a * rho (equilibrium at rest).
 *   - psi^2 < 0 or any non-finite value is never clamped: it is propagated and
 *     reported by the step's return code.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny;
    int32_t walls;      /* 0: periodic in y; 1: halfway bounce-back walls at y=-1/2 and y=ny-1/2 */
    int32_t pad_;
    double a, b, R, T;  /* Carnahan-Starling EOS, Eq. 15 */
    double G;           /* interaction strength, Eq. 7 and Eq. 13 */
    double eps;         /* Li's forcing coefficient, Eq. 14 */
    double s[9];        /* diagonal of Lambda, Eq. 2, moment order of Eq. 4 */
} oracle_params;

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_ENOMEM = -2, ORACLE_ENONFINITE = -4 };

/* D2Q9 discrete velocities e_a (Section 2.1). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Index of -e_a, for halfway bounce-back (Section 4.1). */
static int opposite(int a)
{
    for (int b = 0; b < 9; ++b)
        if (EX[b] == -EX[a] && EY[b] == -EY[a])
            return b;
    return -1;
}

/* Interaction weights of Eq. 7: 1/3 on the axes, 1/12 on the diagonals. */
static double force_weight(int a)
{
    if (a == 0) return 0.0;
    return (a <= 4) ? 1.0 / 3.0 : 1.0 / 12.0;
}

/* Lattice weights of the rest-state equilibrium f_a = w_a rho. */
static double lattice_weight(int a)
{
    if (a == 0) return 4.0 / 9.0;
    return (a <= 4) ? 1.0 / 9.0 : 1.0 / 36.0;
}

/* Orthogonal D2Q9 transformation matrix M (Eq. 1, m = M f), rows in the
 * moment order of Eq. 4. */
static const double M[9][9] = {
    { 1,  1,  1,  1,  1,  1,  1,  1,  1},   /* rho  */
    {-4, -1, -1, -1, -1,  2,  2,  2,  2},   /* e    */
    { 4, -2, -2, -2, -2,  1,  1,  1,  1},   /* zeta */
    { 0,  1,  0, -1,  0,  1, -1, -1,  1},   /* jx   */
    { 0, -2,  0,  2,  0,  1, -1, -1,  1},   /* qx   */
    { 0,  0,  1,  0, -1,  1,  1, -1, -1},   /* jy   */
    { 0,  0, -2,  0,  2,  1,  1, -1, -1},   /* qy   */
    { 0,  1, -1,  1, -1,  0,  0,  0,  0},   /* pxx  */
    { 0,  0,  0,  0,  0,  1, -1,  1, -1},   /* pxy  */
};

static double MINV[9][9];
static int minv_ready = 0;

/* M^-1 by Gauss-Jordan elimination with partial pivoting. */
static void compute_minv(void)
{
    double A[9][18];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 18; ++j)
            A[i][j] = (j < 9) ? M[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 18; ++j) {
                double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t;
            }
        double d = A[c][c];
        for (int j = 0; j < 18; ++j) A[c][j] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            double q = A[r][c];
            if (q == 0.0) continue;
            for (int j = 0; j < 18; ++j) A[r][j] -= q * A[c][j];
        }
    }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j)
            MINV[i][j] = A[i][j + 9];
    minv_ready = 1;
}

static void ensure_minv(void)
{
    if (!minv_ready) compute_minv();
}

/* ---- Equation of state and pseudopotential ------------------------------ */

/* Carnahan-Starling EOS, Eq. 15: p = rho R T (1+eta+eta^2-eta^3)/(1-eta)^3 - a rho^2,
 * eta = b rho / 4. */
double oracle_eos_pressure(const oracle_params *P, double rho)
{
    double eta = P->b * rho / 4.0;
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    return rho * P->R * P->T * num / den - P->a * rho * rho;
}

/* Pseudopotential of the second strategy, Eq. 13, with c = 1 and
 * c_s^2 = 1/3: psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)). */
double oracle_psi(const oracle_params *P, double rho)
{
    const double c = 1.0, cs2 = 1.0 / 3.0;
    double p = oracle_eos_pressure(P, rho);
    return sqrt(2.0 * (p - rho * cs2) / (P->G * c * c));
}

/* ---- Per-field steps ------------------------------------------------------ */

/* Density rho = sum_a f_a (after Eq. 4). */
void oracle_density(const oracle_params *P, const double *f, double *rho)
{
    long n = (long)P->nx * P->ny;
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += f[i * 9 + a];
        rho[i] = s;
    }
}

/* psi at lattice site (x, y), with periodic wrap in x, and in y either periodic
 * wrap or, for walls, the mirror reading (a solid site takes the psi of the
 * fluid row next to it). */
static double psi_site(const oracle_params *P, const double *psi, int x, int y)
{
    int nx = P->nx, ny = P->ny;
    x = ((x % nx) + nx) % nx;
    if (P->walls) {
        if (y < 0) y = 0;
        if (y > ny - 1) y = ny - 1;
    } else {
        y = ((y % ny) + ny) % ny;
    }
    return psi[(long)y * nx + x];
}

/* Pseudopotential interaction force, Eq. 7:
 * F(x) = -G psi(x) sum_{a=1..8} w_a psi(x + e_a) e_a. */
void oracle_force(const oracle_params *P, const double *psi, double *Fx, double *Fy)
{
    int nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0.0, sy = 0.0;
            for (int a = 1; a < 9; ++a) {
                double pn = psi_site(P, psi, x + EX[a], y + EY[a]);
                sx += force_weight(a) * pn * EX[a];
                sy += force_weight(a) * pn * EY[a];
            }
            long i = (long)y * nx + x;
            Fx[i] = -P->G * psi[i] * sx;
            Fy[i] = -P->G * psi[i] * sy;
        }
}

/* m = M f. */
void oracle_moments(const double *f, double *m)
{
    for (int k = 0; k < 9; ++k) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += M[k][a] * f[a];
        m[k] = s;
    }
}

/* Equilibrium moments, Eq. 4. */
void oracle_equilibrium_moments(double rho, double vx, double vy, double *meq)
{
    double v2 = vx * vx + vy * vy;
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * v2);
    meq[2] = rho * (1.0 - 3.0 * v2);
    meq[3] = rho * vx;
    meq[4] = -rho * vx;
    meq[5] = rho * vy;
    meq[6] = -rho * vy;
    meq[7] = rho * (vx * vx - vy * vy);
    meq[8] = rho * vx * vy;
}

/* Li's modified forcing term in moment space, Eq. 14 (Eq. 8 when eps = 0),
 * with delta_t = 1, tau_e = 1/s_e and tau_zeta = 1/s_zeta. */
void oracle_source(const oracle_params *P, double vx, double vy, double Fx, double Fy,
                   double psi, double *S)
{
    const double dt = 1.0;
    double tau_e = 1.0 / P->s[1];
    double tau_z = 1.0 / P->s[2];
    double vF = vx * Fx + vy * Fy;
    double F2 = Fx * Fx + Fy * Fy;
    S[0] = 0.0;
    S[1] = 6.0 * vF + 0.75 * P->eps * F2 / (psi * psi * dt * (tau_e - 0.5));
    S[2] = -6.0 * vF - 0.75 * P->eps * F2 / (psi * psi * dt * (tau_z - 0.5));
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (vx * Fx - vy * Fy);
    S[8] = vx * Fy + vy * Fx;
}

/* One node of the collision: velocity (Eq. 6), moments, equilibrium (Eq. 4),
 * source (Eq. 14), relaxation (Eq. 3), back-transform f* = M^-1 m*. */
void oracle_collide_node(const oracle_params *P, const double *f, double psi,
                         double Fx, double Fy, double *fstar)
{
    const double dt = 1.0;
    ensure_minv();
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += f[a];
        jx += EX[a] * f[a];
        jy += EY[a] * f[a];
    }
    double vx = (jx + 0.5 * dt * Fx) / rho;
    double vy = (jy + 0.5 * dt * Fy) / rho;
    double m[9], meq[9], S[9], ms[9];
    oracle_moments(f, m);
    oracle_equilibrium_moments(rho, vx, vy, meq);
    oracle_source(P, vx, vy, Fx, Fy, psi, S);
    for (int k = 0; k < 9; ++k)
        ms[k] = m[k] - P->s[k] * (m[k] - meq[k]) + dt * (1.0 - 0.5 * P->s[k]) * S[k];
    for (int a = 0; a < 9; ++a) {
        double s = 0.0;
        for (int k = 0; k < 9; ++k) s += MINV[a][k] * ms[k];
        fstar[a] = s;
    }
}

/* Collision of every node. */
void oracle_collide(const oracle_params *P, const double *f, const double *psi,
                    const double *Fx, const double *Fy, double *fstar)
{
    long n = (long)P->nx * P->ny;
    ensure_minv();
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i)
        oracle_collide_node(P, f + i * 9, psi[i], Fx[i], Fy[i], fstar + i * 9);
}

/* Streaming, Eq. 5: f_a(x + e_a, t + 1) = f*_a(x, t); x always periodic; y
 * periodic, or halfway bounce-back: a population that would leave through a
 * wall returns to its own node in the opposite direction. */
void oracle_stream(const oracle_params *P, const double *fstar, double *fnew)
{
    int nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int a = 0; a < 9; ++a) {
                long src = ((long)y * nx + x) * 9 + a;
                int xd = ((x + EX[a]) % nx + nx) % nx;
                int yd = y + EY[a];
                if (P->walls && (yd < 0 || yd > ny - 1)) {
                    fnew[((long)y * nx + x) * 9 + opposite(a)] = fstar[src];
                } else {
                    yd = ((yd % ny) + ny) % ny;
                    fnew[((long)yd * nx + xd) * 9 + a] = fstar[src];
                }
            }
}

/* ---- Whole steps ----------------------------------------------------------- */

static int all_finite(const double *v, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Largest pressure of Eq. 15 over the two wall rows (y = 0 and y = ny-1) of
 * a density field: the wall-pressure reading of the collapse runs (the paper
 * plots a wall pressure but does not define a sampled value). */
static double wall_row_pressure_max(const oracle_params *P, const double *rho)
{
    double best = -INFINITY;
    const int rows[2] = {0, P->ny - 1};
    for (int k = 0; k < 2; ++k)
        for (int x = 0; x < P->nx; ++x) {
            double pw = oracle_eos_pressure(P, rho[(long)rows[k] * P->nx + x]);
            if (pw > best) best = pw;
        }
    return best;
}

static int run_steps(const oracle_params *P, double *f, int64_t nsteps, double *wall_p);

/* nsteps full timesteps in place on f (post-streaming populations).  The
 * order within a step: rho and psi of every node (Eqs. 15, 13), the force of
 * every node (Eq. 7), the collision of every node (Eqs. 6, 4, 14, 3), then
 * streaming (Eq. 5).  Returns ORACLE_ENONFINITE, and stops, at the first step
 * whose psi or populations are not finite. */
int oracle_step(const oracle_params *P, double *f, int64_t nsteps)
{
    return run_steps(P, f, nsteps, NULL);
}

/* The same steps, also writing to wall_p[t] (t = 0 .. nsteps-1) the largest
 * pressure of Eq. 15 on the wall rows of the state at the start of step t. */
int oracle_step_wall_pressure(const oracle_params *P, double *f, int64_t nsteps, double *wall_p)
{
    if (!wall_p) return ORACLE_EINVAL;
    return run_steps(P, f, nsteps, wall_p);
}

static int run_steps(const oracle_params *P, double *f, int64_t nsteps, double *wall_p)
{
    if (P->nx < 1 || P->ny < 1 || nsteps < 0) return ORACLE_EINVAL;
    long n = (long)P->nx * P->ny;
    double *rho = malloc(sizeof(double) * n);
    double *psi = malloc(sizeof(double) * n);
    double *Fx = malloc(sizeof(double) * n);
    double *Fy = malloc(sizeof(double) * n);
    double *fstar = malloc(sizeof(double) * n * 9);
    int rc = ORACLE_OK;
    if (!rho || !psi || !Fx || !Fy || !fstar) { rc = ORACLE_ENOMEM; goto done; }
    ensure_minv();
    for (int64_t t = 0; t < nsteps; ++t) {
        oracle_density(P, f, rho);
        if (wall_p) wall_p[t] = wall_row_pressure_max(P, rho);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) psi[i] = oracle_psi(P, rho[i]);
        if (!all_finite(psi, n)) { rc = ORACLE_ENONFINITE; goto done; }
        oracle_force(P, psi, Fx, Fy);
        oracle_collide(P, f, psi, Fx, Fy, fstar);
        oracle_stream(P, fstar, f);
        if (!all_finite(f, n * 9)) { rc = ORACLE_ENONFINITE; goto done; }
    }
done:
    free(rho); free(psi); free(Fx); free(Fy); free(fstar);
    return rc;
}

/* Macroscopic fields of a post-streaming state: rho, v of Eq. 6 (with the
 * force of Eq. 7 from this state's psi), p of Eq. 15. */
int oracle_macros(const oracle_params *P, const double *f, double *rho, double *vx,
                  double *vy, double *p)
{
    long n = (long)P->nx * P->ny;
    double *psi = malloc(sizeof(double) * n);
    double *Fx = malloc(sizeof(double) * n);
    double *Fy = malloc(sizeof(double) * n);
    if (!psi || !Fx || !Fy) { free(psi); free(Fx); free(Fy); return ORACLE_ENOMEM; }
    oracle_density(P, f, rho);
    for (long i = 0; i < n; ++i) psi[i] = oracle_psi(P, rho[i]);
    oracle_force(P, psi, Fx, Fy);
    for (long i = 0; i < n; ++i) {
        double jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            jx += EX[a] * f[i * 9 + a];
            jy += EY[a] * f[i * 9 + a];
        }
        vx[i] = (jx + 0.5 * Fx[i]) / rho[i];
        vy[i] = (jy + 0.5 * Fy[i]) / rho[i];
        p[i] = oracle_eos_pressure(P, rho[i]);
    }
    free(psi); free(Fx); free(Fy);
    return ORACLE_OK;
}

/* ---- Initial state --------------------------------------------------------- */

/* SplitMix64 (Steele, Lea and Flood, 2014): one output of the generator
 * seeded with s. */
static uint64_t splitmix64(uint64_t s)
{
    uint64_t z = s + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform deviate in [0, 1) for node index i under the given seed. */
double oracle_uniform(uint64_t seed, uint64_t i)
{
    return (double)(splitmix64(seed ^ i) >> 11) * (1.0 / 9007199254740992.0);
}

/* Density field of Eq. 16.  bubbles holds nb triples (x0, y0, r0).  With
 * slab_rows > 0 the state is instead a flat liquid slab of that many rows
 * centred on (ny-1)/2, gas outside.  The liquid side takes rho_l (1 + delta)
 * (Section 4.1), then every node is scaled by 1 + noise_amp (2u - 1).  For
 * several bubbles the signed distance is that to the nearest bubble edge. */
void oracle_init_density(const oracle_params *P, const double *bubbles, int nb, int slab_rows,
                         double rho_l, double rho_g, double W, double delta,
                         double noise_amp, uint64_t seed, double *rho)
{
    int nx = P->nx, ny = P->ny;
    double rl = rho_l * (1.0 + delta);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            /* d: signed distance, positive on the liquid side */
            double d;
            if (slab_rows > 0) {
                d = 0.5 * slab_rows - fabs(y - 0.5 * (ny - 1));
            } else {
                d = INFINITY;
                for (int k = 0; k < nb; ++k) {
                    double dx = x - bubbles[3 * k], dy = y - bubbles[3 * k + 1];
                    double dk = sqrt(dx * dx + dy * dy) - bubbles[3 * k + 2];
                    if (dk < d) d = dk;
                }
            }
            double r = 0.5 * (rl + rho_g) + 0.5 * (rl - rho_g) * tanh(2.0 * d / W);
            long i = (long)y * nx + x;
            if (noise_amp != 0.0)
                r *= 1.0 + noise_amp * (2.0 * oracle_uniform(seed, (uint64_t)i) - 1.0);
            rho[i] = r;
        }
}

/* Populations at rest equilibrium, f_a = w_a rho. */
void oracle_init_populations(const oracle_params *P, const double *rho, double *f)
{
    long n = (long)P->nx * P->ny;
    for (long i = 0; i < n; ++i)
        for (int a = 0; a < 9; ++a) f[i * 9 + a] = lattice_weight(a) * rho[i];
}

/* Exposes M and M^-1 to the tests. */
void oracle_transform(double *m_out, double *minv_out)
{
    ensure_minv();
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            if (m_out) m_out[i * 9 + j] = M[i][j];
            if (minv_out) minv_out[i * 9 + j] = MINV[i][j];
        }
}

/* Exposes the velocity set (ex, ey interleaved) to the tests. */
void oracle_velocities(int *e_out)
{
    for (int a = 0; a < 9; ++a) {
        e_out[2 * a] = EX[a];
        e_out[2 * a + 1] = EY[a];
    }
}

/* Threads the OpenMP loops use, and a way to change it (for timing the oracle
 * on one core and on all of them). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
