/*
 * lbdem_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference of the coupled lattice-Boltzmann /
 * discrete-element method of Cheng, Luding, Rivas, Harting and Magnanimo,
 * "Hydro-micromechanical modeling of wave propagation in saturated granular media"
 * (arXiv 1808.08921).  It exists so that the GPU library can be checked against
 * something obviously correct.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library never links it and
 * shares no code, header or table with it.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. "Verification", lattice units).
 *   - Node (i,j,k) sits at coordinate (i,j,k); cell index n = (k*ny + j)*nx + i.
 *   - Direction index d = 0..18 is the paper's d = 1..19 minus one (Eq. 3d19q);
 *     d = 18 is the rest direction.
 *   - Populations are stored post-collision, f~_d(x,t), as [19][ncell].
 *
 * One step t -> t+1 (the paper gives no order; this is the order used throughout):
 *   1. link pass: the link force of Eq. (fFS) with the bounce-back of Eq. (mem)
 *      substituted is 2 c_d f~_d(x,t) minus a term linear in the particle's velocities;
 *      per particle the first part (F0, T0) and the matrix Z of the second are summed;
 *   2. DEM: Hertz normal / Mindlin tangential contacts (Eqs. fdLawn, fdLaws) at X(t),
 *      Newton-Euler (Eqs. translate, rotate) with symplectic Euler, dt = 1, the velocity
 *      of the step solved together with the momentum the fluid exchanges in it (the
 *      implicit update of the momentum-exchange scheme of Ladd and Verberg, which the
 *      paper cites for its coupling); the conversion impulses of the last re-projection
 *      act here (Eqs. coupleF, coupleT);
 *   3. pull streaming (Eq. stream) with half-way bounce-back on the particle surfaces at
 *      X(t) moving with the new velocities (Eq. mem) and the link force (Eq. fFS);
 *   4. pressure / density boundary on the z faces (Sec. "Acoustic source",
 *      non-equilibrium bounce-back) driven by the waveform (Eq. source, Table source);
 *   5. BGK collision (Eqs. bgk, BGKequili, rhoAndU);
 *   6. cross-section probes (Sec. "Pressure wave ..." and "Model parameters");
 *   7. the particles move, X(t+1) = X(t) + V(t+1);
 *   8. re-projection of the particles on the lattice and conversion of covered /
 *      uncovered nodes (Eqs. convertFS, convertSF); the conversion impulses act on the
 *      particles in the next step's DEM update (Eqs. coupleF, coupleT).
 *
 * Readings taken where the paper is silent, ambiguous or garbled are listed in the
 * repository design notes and are restated at the place they are used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_PRESSURE = 2 };
enum { WAVE_NONE = 0, WAVE_SINE = 1, WAVE_COSINE = 2, WAVE_STEP = 3 };

/* ------------------------------------------------------------------------- */
/* D3Q19 velocity set: the columns of the matrix of Eq. (3d19q).             */
/* ------------------------------------------------------------------------- */
static const int CX[Q] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
static const int CZ[Q] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
static const double CS2 = 1.0 / 3.0; /* c_s = dx / (sqrt(3) dt) */

/* weight w_d by |c_d| (Sec. "Hydrodynamics", lattice weights) */
static double weight(int d)
{
    int c2 = CX[d] * CX[d] + CY[d] * CY[d] + CZ[d] * CZ[d];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* d* : the direction with c_{d*} = -c_d (Sec. "Fluid-solid coupling"), found by search */
static int opposite(int d)
{
    for (int e = 0; e < Q; ++e)
        if (CX[e] == -CX[d] && CY[e] == -CY[d] && CZ[e] == -CZ[d]) return e;
    return -1;
}

/* f_d^eq = w_d rho [1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)]   Eq. (BGKequili) */
static void equilibrium(double rho, const double u[3], double feq[Q])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int d = 0; d < Q; ++d) {
        double cu = CX[d] * u[0] + CY[d] * u[1] + CZ[d] * u[2];
        feq[d] = weight(d) * rho * (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* rho = sum_d f_d ; rho u = sum_d f_d c_d                               Eq. (rhoAndU) */
static void moments(const double f[Q], double *rho, double j[3])
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int d = 0; d < Q; ++d) {
        r += f[d];
        jx += f[d] * CX[d];
        jy += f[d] * CY[d];
        jz += f[d] * CZ[d];
    }
    *rho = r;
    j[0] = jx; j[1] = jy; j[2] = jz;
}

/* f~_d = f_d + (dt/tau)(f_d^eq - f_d)                                     Eq. (bgk) */
static void collide(const double f[Q], double tau, double out[Q])
{
    double rho, j[3], u[3], feq[Q];
    moments(f, &rho, j);
    u[0] = j[0] / rho; u[1] = j[1] / rho; u[2] = j[2] / rho;
    equilibrium(rho, u, feq);
    for (int d = 0; d < Q; ++d) out[d] = f[d] + (1.0 / tau) * (feq[d] - f[d]);
}

/*
 * Density boundary on a z face (Sec. "Acoustic source": Zou-He / Hecht-Harting D3Q19,
 * non-equilibrium bounce-back of f - f^eq).  Paper indices are used through P(k).
 * Readings: tangential velocity u_x = u_y = 0 at the boundary; f5 is built from its
 * opposite f6 (the printed f3 is a typo); the transverse corrections carry -rho u_x/3,
 * which vanishes for u_x = u_y = 0; u_z follows from the prescribed density.
 * outlet = 0: bottom face z = 0, unknowns 5, 9, 13, 15, 17 (c_z = +1).
 * outlet = 1: top face z = nz-1, unknowns 6, 10, 14, 16, 18 (c_z = -1).
 */
#define P(k) f[(k) - 1]
static void zou_he(double f[Q], double rho, int outlet)
{
    double s0 = P(1) + P(2) + P(3) + P(4) + P(7) + P(8) + P(11) + P(12) + P(19); /* c_z = 0 */
    double nx = 0.5 * (P(1) + P(7) + P(8) - P(2) - P(11) - P(12));
    double ny = 0.5 * (P(3) + P(7) + P(11) - P(4) - P(8) - P(12));
    if (!outlet) {
        double sm = P(6) + P(10) + P(14) + P(16) + P(18); /* c_z = -1, known */
        double ruz = rho - (s0 + 2.0 * sm);
        P(5) = P(6) + ruz / 3.0;
        P(9) = P(14) + ruz / 6.0 - nx;
        P(13) = P(10) + ruz / 6.0 + nx;
        P(15) = P(18) + ruz / 6.0 - ny;
        P(17) = P(16) + ruz / 6.0 + ny;
    } else {
        double sp = P(5) + P(9) + P(13) + P(15) + P(17); /* c_z = +1, known */
        double ruz = (s0 + 2.0 * sp) - rho;
        P(6) = P(5) - ruz / 3.0;
        P(14) = P(9) - ruz / 6.0 + nx;
        P(10) = P(13) - ruz / 6.0 - nx;
        P(18) = P(15) - ruz / 6.0 + ny;
        P(16) = P(17) - ruz / 6.0 - ny;
    }
}
#undef P

/* ------------------------------------------------------------------------- */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    double tau, rho_f;
    int bc[6]; /* faces -x,+x,-y,+y,-z,+z */
    int wave;
    double amp, omega;
    long t_n;
    double E, nu, mu, rho_p;
    int n_probe;
    int probe_z[64];
} orc_params;

typedef struct {
    int j;          /* partner particle */
    double ft[3];   /* tangential spring force acting on the owner of this record */
} contact_rec;

typedef struct {
    orc_params p;
    long ncell;
    double *f;      /* post-collision populations f~(x,t), [19][ncell] */
    double *fs;     /* pre-collision populations f(x,t+1) under construction */
    int *owner;     /* -1 fluid, else index of the particle covering the node */
    int *owner_new;
    double *best_d2;
    long t;
    /* particles */
    int np;
    double *X, *V, *W, *R, *m, *I, *Fg, *Fh, *Th, *Ph, *Lh, *Fl, *Tl;
    unsigned char *fixed;
    contact_rec *hist;  /* [np][hist_cap] tangential history, one record per partner */
    int *nhist;
    int hist_cap;
    /* probes: [t][n_probe][4] = n_fluid, sum rho', sum rho u_z, sum rho */
    double *probe;
    long probe_cap;
    int frozen;     /* 1: particles keep X, V, Omega; no DEM and no re-projection */
    int fluid_off;  /* 1: hydrodynamics switched off (Sec. 3.2, dry granular chain): DEM only */
    int rest_free;  /* 1: link forces without the rest state's part (see orc_set_rest_free) */
} orc_sim;

static int axis_n(const orc_sim *s, int a) { return a == 0 ? s->p.nx : (a == 1 ? s->p.ny : s->p.nz); }
static int periodic(const orc_sim *s, int a) { return s->p.bc[2 * a] == BC_PERIODIC; }

/* minimum-image separation along a periodic axis; plain difference otherwise */
static double min_image(const orc_sim *s, int a, double dx)
{
    if (periodic(s, a)) {
        double n = (double)axis_n(s, a);
        if (dx > 0.5 * n) dx -= n;
        else if (dx < -0.5 * n) dx += n;
    }
    return dx;
}

static double dist2_node(const orc_sim *s, int i, int j, int k, const double *X)
{
    double dx = min_image(s, 0, (double)i - X[0]);
    double dy = min_image(s, 1, (double)j - X[1]);
    double dz = min_image(s, 2, (double)k - X[2]);
    /* one fixed evaluation order, no contraction: (dx dx + dy dy) + dz dz */
    return (dx * dx + dy * dy) + dz * dz;
}

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* rho(t) at the driven face: Eq. (source) and the waveforms of Table (source) */
double orc_rho_in_value(int wave, double rho_f, double amp, double omega, long t_n, long t)
{
    if (wave == WAVE_NONE || t > t_n) return rho_f;
    double wt = omega * (double)t;
    if (wave == WAVE_SINE) return rho_f + amp * sin(wt);
    if (wave == WAVE_COSINE) return rho_f + amp * (1.0 - cos(wt));
    return rho_f + amp; /* step */
}

/* ------------------------------------------------------------------------- */
/* Projection of the particles on the lattice (Sec. "Fluid-solid coupling"). */
/* A node is solid when it lies inside a sphere, d^2 <= R^2 (closed ball).   */
/* A node inside several spheres belongs to the one with the smallest d^2,   */
/* then the smallest index.                                                  */
/* ------------------------------------------------------------------------- */
static void classify(orc_sim *s, int *own)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    for (long n = 0; n < s->ncell; ++n) { own[n] = -1; s->best_d2[n] = INFINITY; }
    for (int q = 0; q < s->np; ++q) {
        const double *X = s->X + 3 * q;
        double R = s->R[q], R2 = R * R;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)floor(X[a] - R) - 1;
            hi[a] = (int)ceil(X[a] + R) + 1;
            int n = axis_n(s, a);
            if (!periodic(s, a)) { if (lo[a] < 0) lo[a] = 0; if (hi[a] > n - 1) hi[a] = n - 1; }
            else if (hi[a] - lo[a] + 1 > n) { lo[a] = 0; hi[a] = n - 1; }
        }
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
            for (int jj = lo[1]; jj <= hi[1]; ++jj)
                for (int ii = lo[0]; ii <= hi[0]; ++ii) {
                    int i = (ii % nx + nx) % nx, j = (jj % ny + ny) % ny, k = (kk % nz + nz) % nz;
                    double d2 = dist2_node(s, i, j, k, X);
                    if (d2 <= R2) {
                        long n = ((long)k * ny + j) * nx + i;
                        if (d2 < s->best_d2[n]) { s->best_d2[n] = d2; own[n] = q; }
                    }
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Create / destroy                                                          */
/* ------------------------------------------------------------------------- */
void *orc_create(int nx, int ny, int nz, double tau, double rho_f, const int *bc6, int wave,
                 double amp, double omega, long t_n, double E, double nu, double mu, double rho_p,
                 int n_probe, const int *probe_z)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(tau > 0.5) || n_probe < 0 || n_probe > 64) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p.nx = nx; s->p.ny = ny; s->p.nz = nz;
    s->p.tau = tau; s->p.rho_f = rho_f;
    for (int a = 0; a < 6; ++a) s->p.bc[a] = bc6[a];
    s->p.wave = wave; s->p.amp = amp; s->p.omega = omega; s->p.t_n = t_n;
    s->p.E = E; s->p.nu = nu; s->p.mu = mu; s->p.rho_p = rho_p;
    s->p.n_probe = n_probe;
    for (int k = 0; k < n_probe; ++k) s->p.probe_z[k] = probe_z[k];
    s->ncell = (long)nx * ny * nz;
    s->f = (double *)malloc(sizeof(double) * Q * s->ncell);
    s->fs = (double *)malloc(sizeof(double) * Q * s->ncell);
    s->owner = (int *)malloc(sizeof(int) * s->ncell);
    s->owner_new = (int *)malloc(sizeof(int) * s->ncell);
    s->best_d2 = (double *)malloc(sizeof(double) * s->ncell);
    if (!s->f || !s->fs || !s->owner || !s->owner_new || !s->best_d2) return NULL;
    /* initial fluid at rest with the mean density: f = w_d rho_f */
    for (int d = 0; d < Q; ++d)
        for (long n = 0; n < s->ncell; ++n) s->f[d * s->ncell + n] = weight(d) * rho_f;
    for (long n = 0; n < s->ncell; ++n) s->owner[n] = -1;
    s->t = 0;
    s->probe_cap = 0;
    s->probe = NULL;
    return s;
}

static void free_particles(orc_sim *s)
{
    double **arrs[] = {&s->X, &s->V, &s->W, &s->R, &s->m, &s->I, &s->Fg, &s->Fh, &s->Th,
                       &s->Ph, &s->Lh, &s->Fl, &s->Tl};
    for (unsigned a = 0; a < sizeof(arrs) / sizeof(arrs[0]); ++a) { free(*arrs[a]); *arrs[a] = NULL; }
    free(s->fixed); s->fixed = NULL;
    free(s->hist); s->hist = NULL;
    free(s->nhist); s->nhist = NULL;
    s->np = 0;
}

void orc_destroy(void *h)
{
    orc_sim *s = (orc_sim *)h;
    if (!s) return;
    free_particles(s);
    free(s->f); free(s->fs); free(s->owner); free(s->owner_new); free(s->best_d2); free(s->probe);
    free(s);
}

/* Particles: m = rho_p (4/3) pi R^3, I = (2/5) m R^2 (solid spheres). */
int orc_set_particles(void *h, int n, const double *x, const double *v, const double *w,
                      const double *r, const double *fg, const unsigned char *fixed)
{
    orc_sim *s = (orc_sim *)h;
    free_particles(s);
    s->np = n;
    size_t b3 = sizeof(double) * 3 * (size_t)(n > 0 ? n : 1), b1 = sizeof(double) * (size_t)(n > 0 ? n : 1);
    s->X = malloc(b3); s->V = malloc(b3); s->W = malloc(b3); s->Fg = malloc(b3);
    s->Fh = calloc(1, b3); s->Th = calloc(1, b3); s->Ph = calloc(1, b3); s->Lh = calloc(1, b3);
    s->Fl = calloc(1, b3); s->Tl = calloc(1, b3);
    s->R = malloc(b1); s->m = malloc(b1); s->I = malloc(b1);
    s->fixed = calloc(1, (size_t)(n > 0 ? n : 1));
    s->hist_cap = 32;
    s->hist = calloc((size_t)(n > 0 ? n : 1) * s->hist_cap, sizeof(contact_rec));
    s->nhist = calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    for (int q = 0; q < n; ++q) {
        for (int a = 0; a < 3; ++a) {
            s->X[3 * q + a] = x[3 * q + a];
            s->V[3 * q + a] = v ? v[3 * q + a] : 0.0;
            s->W[3 * q + a] = w ? w[3 * q + a] : 0.0;
            s->Fg[3 * q + a] = fg ? fg[3 * q + a] : 0.0;
        }
        s->R[q] = r[q];
        s->m[q] = s->p.rho_p * (4.0 / 3.0) * M_PI * r[q] * r[q] * r[q];
        s->I[q] = 0.4 * s->m[q] * r[q] * r[q];
        s->fixed[q] = fixed ? fixed[q] : 0;
        if (s->fixed[q]) for (int a = 0; a < 3; ++a) { s->V[3 * q + a] = 0.0; s->W[3 * q + a] = 0.0; }
    }
    classify(s, s->owner);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Streaming with boundaries.                                                */
/* ------------------------------------------------------------------------- */
/* Source classification for incoming direction e at node (i,j,k).
 * Returns 0 and the wrapped source node, 1 for a stationary half-way wall, 2 for a
 * population left unknown for the density boundary.  A source outside a density face
 * is unknown; otherwise outside a wall face it is a wall; periodic faces wrap. */
static int source_of(const orc_sim *s, int i, int j, int k, int e, int *si, int *sj, int *sk)
{
    int c[3] = {i - CX[e], j - CY[e], k - CZ[e]};
    int unknown = 0, wall = 0;
    for (int a = 0; a < 3; ++a) {
        int n = axis_n(s, a);
        if (c[a] < 0 || c[a] >= n) {
            int face = 2 * a + (c[a] >= n ? 1 : 0);
            if (s->p.bc[face] == BC_PRESSURE) unknown = 1;
            else if (s->p.bc[face] == BC_WALL) wall = 1;
            else c[a] = (c[a] % n + n) % n;
        }
    }
    *si = c[0]; *sj = c[1]; *sk = c[2];
    if (unknown) return 2;
    if (wall) return 1;
    return 0;
}

static void stream(orc_sim *s)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long N = s->ncell;
    for (int q = 0; q < 3 * s->np; ++q) { s->Fl[q] = 0.0; s->Tl[q] = 0.0; }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long n = ((long)k * ny + j) * nx + i;
                if (s->owner[n] >= 0) continue;
                for (int e = 0; e < Q; ++e) {
                    if (e == 18) { s->fs[e * N + n] = s->f[e * N + n]; continue; }
                    int si, sj, sk;
                    int kind = source_of(s, i, j, k, e, &si, &sj, &sk);
                    if (kind == 2) { s->fs[e * N + n] = NAN; continue; }
                    int d = opposite(e); /* d points from x toward the (would-be) source */
                    if (kind == 1) { s->fs[e * N + n] = s->f[d * N + n]; continue; }
                    long sn = ((long)sk * ny + sj) * nx + si;
                    int q = s->owner[sn];
                    if (q < 0) { s->fs[e * N + n] = s->f[e * N + sn]; continue; }
                    /* Eq. (mem): f_{d*}(x,t+1) = f~_d(x,t) - 2 (w_d/cs^2) rho V_b.c_d, with d
                     * pointing from the fluid node into the solid one and d* = e.  Reading:
                     * rho is the mean fluid density rho_f; V_b is evaluated midway on the
                     * link, x_b = x + c_d/2, with the particle state at time t. */
                    double xb[3] = {i + 0.5 * CX[d], j + 0.5 * CY[d], k + 0.5 * CZ[d]};
                    double r[3];
                    for (int a = 0; a < 3; ++a) r[a] = min_image(s, a, xb[a] - s->X[3 * q + a]);
                    double wr[3];
                    cross(s->W + 3 * q, r, wr);
                    double vb[3] = {s->V[3 * q] + wr[0], s->V[3 * q + 1] + wr[1], s->V[3 * q + 2] + wr[2]};
                    double vbc = vb[0] * CX[d] + vb[1] * CY[d] + vb[2] * CZ[d];
                    double fnew = s->f[d * N + n] - 2.0 * weight(d) / CS2 * s->p.rho_f * vbc;
                    s->fs[e * N + n] = fnew;
                    /* Eq. (fFS): F = c_d f~_d(x,t) - c_{d*} f_{d*}(x,t+1), acting on the
                     * particle at x_b; torque (x_b - X_p) x F (Eq. coupleT). */
                    double F[3] = {CX[d] * s->f[d * N + n] - CX[e] * fnew,
                                   CY[d] * s->f[d * N + n] - CY[e] * fnew,
                                   CZ[d] * s->f[d * N + n] - CZ[e] * fnew};
                    if (s->rest_free) {
                        /* without the rest state's part: f~_d and f_{d*} each less w_d rho_f */
                        double rest = 2.0 * weight(d) * s->p.rho_f;
                        F[0] -= CX[d] * rest; F[1] -= CY[d] * rest; F[2] -= CZ[d] * rest;
                    }
                    double T[3];
                    cross(r, F, T);
                    for (int a = 0; a < 3; ++a) { s->Fl[3 * q + a] += F[a]; s->Tl[3 * q + a] += T[a]; }
                }
            }
}

/* ------------------------------------------------------------------------- */
/* Density faces, collision, probes.                                         */
/* ------------------------------------------------------------------------- */
static void boundary_collide_probe(orc_sim *s)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long N = s->ncell;
    double rho_in = orc_rho_in_value(s->p.wave, s->p.rho_f, s->p.amp, s->p.omega, s->p.t_n, s->t + 1);
    if (s->t >= s->probe_cap) {
        long cap = s->probe_cap ? 2 * s->probe_cap : 1024;
        while (cap <= s->t) cap *= 2;
        s->probe = (double *)realloc(s->probe, sizeof(double) * 4 * (s->p.n_probe > 0 ? s->p.n_probe : 1) * cap);
        s->probe_cap = cap;
    }
    double *pr = s->probe + 4 * (s->p.n_probe > 0 ? s->p.n_probe : 1) * s->t;
    for (int k = 0; k < 4 * (s->p.n_probe > 0 ? s->p.n_probe : 1); ++k) pr[k] = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long n = ((long)k * ny + j) * nx + i;
                if (s->owner[n] >= 0) continue;
                double f[Q], out[Q];
                for (int d = 0; d < Q; ++d) f[d] = s->fs[d * N + n];
                if (k == 0 && s->p.bc[4] == BC_PRESSURE) zou_he(f, rho_in, 0);
                if (k == nz - 1 && s->p.bc[5] == BC_PRESSURE) zou_he(f, s->p.rho_f, 1);
                double rho, jm[3];
                moments(f, &rho, jm);
                for (int pz = 0; pz < s->p.n_probe; ++pz)
                    if (s->p.probe_z[pz] == k) {
                        pr[4 * pz + 0] += 1.0;
                        pr[4 * pz + 1] += rho - s->p.rho_f;
                        pr[4 * pz + 2] += jm[2];
                        pr[4 * pz + 3] += rho;
                    }
                collide(f, s->p.tau, out);
                for (int d = 0; d < Q; ++d) s->f[d * N + n] = out[d];
            }
}

/* ------------------------------------------------------------------------- */
/* DEM.                                                                      */
/* ------------------------------------------------------------------------- */
/* Contact of particle i with particle j (i's side).  Eq. (fdLawn): Hertz normal force
 * F_n = 2 E u_n sqrt(R* |u_n|) / (3(1 - nu^2)), R* = 1/(1/R_i + 1/R_j).
 * Eq. (fdLaws): incremental Mindlin tangential force dF_t = 2 E du_t sqrt(R*|u_n|) /
 * ((1+nu)(2-nu)) capped at mu |F_n|.  Readings: the tangential force on i opposes the
 * relative tangential displacement of i's contact point over the step; the stored
 * spring is first projected on the current tangent plane; the contact point is the
 * middle of the overlap.  Returns 1 if in contact. */
int orc_contact(const double *Xi, const double *Xj, double Ri, double Rj, const double *Vi,
                const double *Vj, const double *Wi, const double *Wj, double E, double nu, double mu,
                const double *box /* per-axis period or 0 */, const double *ft_old, double *F,
                double *T, double *ft_new)
{
    double d[3];
    for (int a = 0; a < 3; ++a) {
        double dx = Xj[a] - Xi[a];
        if (box[a] > 0.0) {
            if (dx > 0.5 * box[a]) dx -= box[a];
            else if (dx < -0.5 * box[a]) dx += box[a];
        }
        d[a] = dx;
    }
    double dist = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    double un = Ri + Rj - dist;
    for (int a = 0; a < 3; ++a) { F[a] = 0.0; T[a] = 0.0; ft_new[a] = 0.0; }
    if (!(un > 0.0)) return 0;
    double n[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
    double rstar = 1.0 / (1.0 / Ri + 1.0 / Rj);
    double fn = 2.0 * E * un * sqrt(rstar * un) / (3.0 * (1.0 - nu * nu));
    for (int a = 0; a < 3; ++a) F[a] = -fn * n[a];
    if (mu > 0.0) {
        double ai[3], aj[3], wai[3], waj[3], vrel[3];
        for (int a = 0; a < 3; ++a) { ai[a] = (Ri - 0.5 * un) * n[a]; aj[a] = -(Rj - 0.5 * un) * n[a]; }
        cross(Wi, ai, wai);
        cross(Wj, aj, waj);
        for (int a = 0; a < 3; ++a) vrel[a] = (Vi[a] + wai[a]) - (Vj[a] + waj[a]);
        double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
        double fo = ft_old[0] * n[0] + ft_old[1] * n[1] + ft_old[2] * n[2];
        double kt = 2.0 * E * sqrt(rstar * un) / ((1.0 + nu) * (2.0 - nu));
        double ft[3];
        for (int a = 0; a < 3; ++a) ft[a] = (ft_old[a] - fo * n[a]) - kt * (vrel[a] - vn * n[a]);
        double fm = sqrt(ft[0] * ft[0] + ft[1] * ft[1] + ft[2] * ft[2]);
        if (fm > mu * fn) for (int a = 0; a < 3; ++a) ft[a] *= mu * fn / fm;
        double tq[3];
        cross(ai, ft, tq);
        for (int a = 0; a < 3; ++a) { F[a] += ft[a]; T[a] = tq[a]; ft_new[a] = ft[a]; }
    }
    return 1;
}

/* Link pass.  For a link (fluid node x, direction e whose source x - c_e lies in particle
 * q, d = e* pointing into q), Eq. (fFS) with Eq. (mem) substituted is
 *   F = c_d f~_d(x,t) - c_e f_e(x,t+1) = 2 c_d f~_d(x,t) - (2 w_d / c_s^2) rho_f c_d (c_d . V_b),
 * V_b = V_q + Omega_q x r_b, r_b = x_b - X_q, x_b = x + c_d/2.  With a_d = (c_d, r_b x c_d),
 * c_d . V_b = a_d . (V, Omega), so the force and its torque r_b x F about X_q are
 *   (F, T) = F0 - Z (V, Omega),   F0 = sum 2 f~_d(x,t) a_d,   Z = sum (2 w_d / c_s^2) rho_f a_d a_d^T.
 * F0 [np][6] and Z [np][6][6] are summed here from f~(t) and the node map of time t. */
static void link_pass(const orc_sim *s, double *F0, double *Z)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long N = s->ncell;
    for (long q = 0; q < 6L * s->np; ++q) F0[q] = 0.0;
    for (long q = 0; q < 36L * s->np; ++q) Z[q] = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long n = ((long)k * ny + j) * nx + i;
                if (s->owner[n] >= 0) continue;
                for (int e = 0; e < Q - 1; ++e) {
                    int si, sj, sk;
                    if (source_of(s, i, j, k, e, &si, &sj, &sk) != 0) continue;
                    int q = s->owner[((long)sk * ny + sj) * nx + si];
                    if (q < 0) continue;
                    int d = opposite(e);
                    double xb[3] = {i + 0.5 * CX[d], j + 0.5 * CY[d], k + 0.5 * CZ[d]};
                    double r[3], c[3] = {CX[d], CY[d], CZ[d]}, rc[3];
                    for (int a = 0; a < 3; ++a) r[a] = min_image(s, a, xb[a] - s->X[3 * q + a]);
                    cross(r, c, rc);
                    double av[6] = {c[0], c[1], c[2], rc[0], rc[1], rc[2]};
                    /* (rest_free: without the rest state's part w_d rho_f) */
                    double f2 = 2.0 * (s->f[d * N + n] - (s->rest_free ? weight(d) * s->p.rho_f : 0.0));
                    double kz = 2.0 * weight(d) / CS2 * s->p.rho_f;
                    for (int a = 0; a < 6; ++a) {
                        F0[6 * q + a] += f2 * av[a];
                        for (int b = 0; b < 6; ++b) Z[36 * q + 6 * a + b] += kz * av[a] * av[b];
                    }
                }
            }
}

/* Solves A x = b for a symmetric positive definite 6 x 6 A by the Cholesky factorisation
 * A = L L^T (forward, then backward substitution); b is overwritten by x. */
static void cholesky_solve6(double A[6][6], double b[6])
{
    double L[6][6] = {{0}};
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = A[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    for (int i = 0; i < 6; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * b[k];
        b[i] = v / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double v = b[i];
        for (int k = i + 1; k < 6; ++k) v -= L[k][i] * b[k];
        b[i] = v / L[i][i];
    }
}

/* DEM update of the velocities.  Eqs. (translate), (rotate) with symplectic Euler over the
 * step, dt = 1: M (V', Omega') = M (V, Omega) + (F, T), where the hydrodynamic part of
 * (F, T) is the momentum the fluid exchanges in this step, F0 - Z (V', Omega') (link pass),
 * plus the conversion impulses of the last re-projection (Eqs. coupleF, coupleT); contacts
 * (Hertz normal, Mindlin tangential) are evaluated at X(t), V(t), Omega(t), plus the
 * external force.  Reading (the implicit update of the Ladd-Verberg momentum-exchange
 * scheme): the fluid's bounce-back of this step uses the same velocities V', Omega' that
 * this update produces, so (M + Z)(V', Omega') = M (V, Omega) + F0 + contacts + F_g +
 * pending impulses, solved per particle.  (The explicit alternative, bounce-back at V(t)
 * and the particle updated afterwards, lets a period-two mode of the thin fluid
 * filaments next to the contacts of a dense packing grow.)  Fixed particles keep
 * V = Omega = 0.  F_h, T_h first receive the pending impulses used here (the link part
 * is added by the streaming step). */
static void dem(orc_sim *s, const double *F0, const double *Z)
{
    int np = s->np;
    double box[3];
    for (int a = 0; a < 3; ++a) box[a] = periodic(s, a) ? (double)axis_n(s, a) : 0.0;
    double *rhs = calloc((size_t)6 * (np > 0 ? np : 1), sizeof(double));
    contact_rec *nh = calloc((size_t)(np > 0 ? np : 1) * s->hist_cap, sizeof(contact_rec));
    int *nn = calloc((size_t)(np > 0 ? np : 1), sizeof(int));
    for (int i = 0; i < np; ++i) {
        for (int a = 0; a < 3; ++a) {
            s->Fh[3 * i + a] = s->Ph[3 * i + a];
            s->Th[3 * i + a] = s->Lh[3 * i + a];
            rhs[6 * i + a] = (F0 ? F0[6 * i + a] : 0.0) + s->Ph[3 * i + a] + s->Fg[3 * i + a];
            rhs[6 * i + 3 + a] = (F0 ? F0[6 * i + 3 + a] : 0.0) + s->Lh[3 * i + a];
        }
        for (int j = 0; j < np; ++j) {
            if (j == i) continue;
            double ft_old[3] = {0.0, 0.0, 0.0};
            for (int h = 0; h < s->nhist[i]; ++h)
                if (s->hist[i * s->hist_cap + h].j == j)
                    for (int a = 0; a < 3; ++a) ft_old[a] = s->hist[i * s->hist_cap + h].ft[a];
            double F[3], T[3], ftn[3];
            if (orc_contact(s->X + 3 * i, s->X + 3 * j, s->R[i], s->R[j], s->V + 3 * i, s->V + 3 * j,
                            s->W + 3 * i, s->W + 3 * j, s->p.E, s->p.nu, s->p.mu, box, ft_old, F, T, ftn)) {
                for (int a = 0; a < 3; ++a) { rhs[6 * i + a] += F[a]; rhs[6 * i + 3 + a] += T[a]; }
                if (s->p.mu > 0.0 && nn[i] < s->hist_cap) {
                    contact_rec *rec = nh + i * s->hist_cap + nn[i]++;
                    rec->j = j;
                    for (int a = 0; a < 3; ++a) rec->ft[a] = ftn[a];
                }
            }
        }
    }
    for (int i = 0; i < np; ++i) {
        if (s->fixed[i]) continue;
        double A[6][6], b[6];
        for (int a = 0; a < 6; ++a) {
            for (int c = 0; c < 6; ++c) A[a][c] = Z ? Z[36 * i + 6 * a + c] : 0.0;
            double inertia = a < 3 ? s->m[i] : s->I[i];
            A[a][a] += inertia;
            b[a] = inertia * (a < 3 ? s->V[3 * i + a] : s->W[3 * i + a - 3]) + rhs[6 * i + a];
        }
        cholesky_solve6(A, b);
        for (int a = 0; a < 3; ++a) { s->V[3 * i + a] = b[a]; s->W[3 * i + a] = b[3 + a]; }
    }
    for (int i = 0; i < 3 * np; ++i) { s->Ph[i] = 0.0; s->Lh[i] = 0.0; }
    free(s->hist);
    free(s->nhist);
    s->hist = nh;
    s->nhist = nn;
    free(rhs);
}

/* Positions after the step: X(t+1) = X(t) + V(t+1) (symplectic Euler), wrapped on
 * periodic axes; fixed particles stay. */
static void move(orc_sim *s)
{
    for (int i = 0; i < s->np; ++i) {
        if (s->fixed[i]) continue;
        for (int a = 0; a < 3; ++a) {
            double x = s->X[3 * i + a] + s->V[3 * i + a];
            if (periodic(s, a)) {
                double n = (double)axis_n(s, a);
                if (x >= n) x -= n;
                else if (x < 0.0) x += n;
            }
            s->X[3 * i + a] = x;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Re-projection with covered / uncovered node conversion.                   */
/* ------------------------------------------------------------------------- */
/* Readings of Eqs. (convertFS), (convertSF): the printed signs contradict the stated
 * purpose (momentum conservation); the conversions are applied so that fluid plus
 * particle momentum is conserved: a covered node hands +rho u to its new owner, an
 * uncovered node is refilled with f^eq(rho_bar, V_b) and takes rho_bar V_b from its old
 * owner.  rho_bar is the mean density of the D3Q19 neighbours that are fluid both before
 * and after the re-projection (rho_f if there are none).  Torque arms are x - X_p with
 * the particle at its new position. */
static void remap(orc_sim *s)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long N = s->ncell;
    classify(s, s->owner_new);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long n = ((long)k * ny + j) * nx + i;
                int o = s->owner[n], q = s->owner_new[n];
                if (o < 0 && q >= 0) {
                    double f[Q], rho, ju[3], r[3], L[3];
                    for (int d = 0; d < Q; ++d) f[d] = s->f[d * N + n];
                    moments(f, &rho, ju);
                    double x[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a) r[a] = min_image(s, a, x[a] - s->X[3 * q + a]);
                    cross(r, ju, L);
                    for (int a = 0; a < 3; ++a) { s->Ph[3 * q + a] += ju[a]; s->Lh[3 * q + a] += L[a]; }
                } else if (o >= 0 && q < 0) {
                    double sum = 0.0;
                    int cnt = 0;
                    for (int e = 0; e < 18; ++e) {
                        int c[3] = {i + CX[e], j + CY[e], k + CZ[e]};
                        int ok = 1;
                        for (int a = 0; a < 3; ++a) {
                            int na = axis_n(s, a);
                            if (c[a] < 0 || c[a] >= na) {
                                if (periodic(s, a)) c[a] = (c[a] % na + na) % na;
                                else ok = 0;
                            }
                        }
                        if (!ok) continue;
                        long m = ((long)c[2] * ny + c[1]) * nx + c[0];
                        if (s->owner[m] >= 0 || s->owner_new[m] >= 0) continue;
                        double rr = 0.0;
                        for (int d = 0; d < Q; ++d) rr += s->f[d * N + m];
                        sum += rr;
                        cnt += 1;
                    }
                    double rbar = cnt > 0 ? sum / cnt : s->p.rho_f;
                    double x[3] = {i, j, k}, r[3], wr[3], vb[3], feq[Q], L[3], mom[3];
                    for (int a = 0; a < 3; ++a) r[a] = min_image(s, a, x[a] - s->X[3 * o + a]);
                    cross(s->W + 3 * o, r, wr);
                    for (int a = 0; a < 3; ++a) vb[a] = s->V[3 * o + a] + wr[a];
                    equilibrium(rbar, vb, feq);
                    for (int d = 0; d < Q; ++d) s->f[d * N + n] = feq[d];
                    for (int a = 0; a < 3; ++a) mom[a] = rbar * vb[a];
                    cross(r, mom, L);
                    for (int a = 0; a < 3; ++a) { s->Ph[3 * o + a] -= mom[a]; s->Lh[3 * o + a] -= L[a]; }
                }
            }
    int *tmp = s->owner;
    s->owner = s->owner_new;
    s->owner_new = tmp;
}

/* One full coupled step t -> t+1. */
void orc_step(void *h, long nsteps)
{
    orc_sim *s = (orc_sim *)h;
    for (long it = 0; it < nsteps; ++it) {
        if (s->fluid_off) {
            /* no fluid step: the particles feel contacts and their own forces only */
            if (s->np > 0) {
                const size_t b3 = (size_t)3 * s->np * sizeof(double);
                memset(s->Ph, 0, b3); memset(s->Lh, 0, b3);
                if (!s->frozen) { dem(s, NULL, NULL); move(s); }
            }
            s->t += 1;
            continue;
        }
        if (s->frozen) {
            stream(s);
            boundary_collide_probe(s);
            s->t += 1;
            continue;
        }
        double *F0 = calloc((size_t)6 * (s->np > 0 ? s->np : 1), sizeof(double));
        double *Z = calloc((size_t)36 * (s->np > 0 ? s->np : 1), sizeof(double));
        link_pass(s, F0, Z);
        dem(s, F0, Z);
        free(F0);
        free(Z);
        stream(s);
        for (int q = 0; q < 3 * s->np; ++q) { s->Fh[q] += s->Fl[q]; s->Th[q] += s->Tl[q]; }
        boundary_collide_probe(s);
        move(s);
        remap(s);
        s->t += 1;
    }
}

/* ------------------------------------------------------------------------- */
/* Accessors                                                                 */
/* ------------------------------------------------------------------------- */
long orc_time(void *h) { return ((orc_sim *)h)->t; }
long orc_ncell(void *h) { return ((orc_sim *)h)->ncell; }

void orc_get_populations(void *h, double *f)
{
    orc_sim *s = (orc_sim *)h;
    memcpy(f, s->f, sizeof(double) * Q * s->ncell);
}

void orc_set_populations(void *h, const double *f)
{
    orc_sim *s = (orc_sim *)h;
    memcpy(s->f, f, sizeof(double) * Q * s->ncell);
}

void orc_get_owner(void *h, int *own)
{
    orc_sim *s = (orc_sim *)h;
    memcpy(own, s->owner, sizeof(int) * s->ncell);
}

/* Re-project at the current positions (used by tests of the projection alone). */
void orc_classify(void *h, int *own)
{
    orc_sim *s = (orc_sim *)h;
    classify(s, own);
}

void orc_get_particles(void *h, double *x, double *v, double *w, double *fh, double *th)
{
    orc_sim *s = (orc_sim *)h;
    size_t b = sizeof(double) * 3 * (size_t)s->np;
    if (x) memcpy(x, s->X, b);
    if (v) memcpy(v, s->V, b);
    if (w) memcpy(w, s->W, b);
    if (fh) memcpy(fh, s->Fh, b);
    if (th) memcpy(th, s->Th, b);
}

/* pending conversion impulses (momentum, angular momentum) */
void orc_get_pending(void *h, double *ph, double *lh)
{
    orc_sim *s = (orc_sim *)h;
    size_t b = sizeof(double) * 3 * (size_t)s->np;
    memcpy(ph, s->Ph, b);
    memcpy(lh, s->Lh, b);
}

int orc_get_probes(void *h, long first, long n, double *out)
{
    orc_sim *s = (orc_sim *)h;
    if (first < 0 || first + n > s->t) return -1;
    int np = s->p.n_probe > 0 ? s->p.n_probe : 1;
    memcpy(out, s->probe + 4 * np * first, sizeof(double) * 4 * np * n);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Node-level entry points (the same functions the step uses), for pin tests. */
/* ------------------------------------------------------------------------- */
void orc_velocity_set(int *c, double *w, int *opp)
{
    for (int d = 0; d < Q; ++d) {
        c[3 * d] = CX[d]; c[3 * d + 1] = CY[d]; c[3 * d + 2] = CZ[d];
        w[d] = weight(d);
        opp[d] = opposite(d);
    }
}
void orc_equilibrium(double rho, const double *u, double *feq) { equilibrium(rho, u, feq); }
void orc_collide_node(const double *f, double tau, double *out) { collide(f, tau, out); }
void orc_zou_he(double *f, double rho, int outlet) { zou_he(f, rho, outlet); }

/* ------------------------------------------------------------------------- */
/* Adjoint of the fluid step over frozen particle geometry.                  */
/* ------------------------------------------------------------------------- */
/* Frozen geometry: the particles keep their position, velocity and angular velocity,
 * the node map does not change, and one step is streaming with the walls of Eq. (mem),
 * the density faces and the collision (steps 1-3 above).  The probe signal of step n is
 * the plane average of rho - rho_f over the fluid nodes of each probe plane, taken from
 * the pre-collision moments of time level n+1.  For a loss L(P) the discrete adjoint
 * lambda^n = (dS/df^n)^T lambda^{n+1} + dL/df^n is propagated backwards through the
 * stored forward states, and dL/dtau, dL/dA (the waveform amplitude) and dL/dV (particle
 * velocities, through the moving-wall term) are accumulated.  Each transpose is taken of
 * the plain definition: the collision Jacobian differentiated term by term, the density
 * faces through the columns of their affine map, streaming by following every
 * population to its single consumer. */
void orc_set_frozen(void *h, int frozen) { ((orc_sim *)h)->frozen = frozen; }
void orc_set_fluid_off(void *h, int off) { ((orc_sim *)h)->fluid_off = off; }

/* rest_free = 1: the link force of Eq. (fFS) without the part of the rest state
 * f_d = w_d rho_f (a reading for touching particles; identical for separated ones) */
void orc_set_rest_free(void *h, int on) { ((orc_sim *)h)->rest_free = on; }

void orc_set_velocities(void *h, const double *V, const double *W)
{
    orc_sim *s = (orc_sim *)h;
    for (int q = 0; q < 3 * s->np; ++q) {
        if (V) s->V[q] = V[q];
        if (W) s->W[q] = W[q];
    }
}

/* d f~_d / d f_e of the BGK collision at one node, from Eqs. (bgk), (BGKequili),
 * (rhoAndU): (1 - 1/tau) delta_de + (1/tau) d f^eq_d / d f_e, with d rho / d f_e = 1 and
 * d u / d f_e = (c_e - u) / rho. */
static void collide_jacobian(const double f[Q], double tau, double J[Q][Q])
{
    double rho, j[3], u[3];
    moments(f, &rho, j);
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int d = 0; d < Q; ++d) {
        double cu = CX[d] * u[0] + CY[d] * u[1] + CZ[d] * u[2];
        double base = 1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
        for (int e = 0; e < Q; ++e) {
            double du[3] = {(CX[e] - u[0]) / rho, (CY[e] - u[1]) / rho, (CZ[e] - u[2]) / rho};
            double cdu = CX[d] * du[0] + CY[d] * du[1] + CZ[d] * du[2];
            double udu = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
            double dfeq = weight(d) * (base + rho * (cdu / CS2 + cu * cdu / (CS2 * CS2) - udu / CS2));
            J[d][e] = (d == e ? 1.0 - 1.0 / tau : 0.0) + dfeq / tau;
        }
    }
}

/* The density face as an affine map g = M f + b rho: column e of M is the face applied to
 * the unit vector e with rho = 0, b is the face applied to zero with rho = 1. */
static void zou_he_affine(int outlet, double M[Q][Q], double b[Q])
{
    for (int e = 0; e < Q; ++e) {
        double v[Q] = {0};
        v[e] = 1.0;
        zou_he(v, 0.0, outlet);
        for (int d = 0; d < Q; ++d) M[d][e] = v[d];
    }
    double z[Q] = {0};
    zou_he(z, 1.0, outlet);
    for (int d = 0; d < Q; ++d) b[d] = z[d];
}

/* Forward nsteps from the current state with relaxation time tau, waveform amplitude amp
 * and the current particle velocities; P[n * n_probe + k] receives the probe signals.
 * Then, for the loss gradient dLdP (same layout), g_tau, g_amp and g_v[np][3] receive
 * dL/dtau, dL/damp and dL/dV.  The simulation ends at time t + nsteps.  Returns 0, or -1
 * when memory runs out. */
int orc_adjoint(void *h, long nsteps, double tau, double amp, const double *dLdP, double *P, double *g_tau,
                double *g_amp, double *g_v)
{
    orc_sim *s = (orc_sim *)h;
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz, np = s->p.n_probe;
    const long N = s->ncell;
    const long t0 = s->t;
    s->p.tau = tau;
    s->p.amp = amp;
    int frozen = s->frozen;
    s->frozen = 1;
    double *traj = (double *)malloc(sizeof(double) * Q * N * (size_t)(nsteps > 0 ? nsteps : 1));
    double *lam = (double *)calloc((size_t)Q * N, sizeof(double));
    double *lam_prev = (double *)calloc((size_t)Q * N, sizeof(double));
    double *mu = (double *)calloc((size_t)Q * N, sizeof(double));
    double *nfl = (double *)calloc((size_t)(np > 0 ? np : 1), sizeof(double));
    if (!traj || !lam || !lam_prev || !mu || !nfl) {
        free(traj); free(lam); free(lam_prev); free(mu); free(nfl);
        s->frozen = frozen;
        return -1;
    }
    /* forward, keeping every state f^n */
    for (long n = 0; n < nsteps; ++n) {
        memcpy(traj + (size_t)Q * N * n, s->f, sizeof(double) * Q * N);
        orc_step(s, 1);
        const double *pr = s->probe + 4 * (np > 0 ? np : 1) * (t0 + n);
        for (int k = 0; k < np; ++k) {
            P[n * np + k] = pr[4 * k + 1] / pr[4 * k + 0];
            nfl[k] = pr[4 * k + 0];
        }
    }
    double Mz[2][Q][Q], bz[2][Q];
    zou_he_affine(0, Mz[0], bz[0]);
    zou_he_affine(1, Mz[1], bz[1]);
    double gw = 0.0, ga = 0.0;
    for (int q = 0; q < 3 * s->np; ++q) g_v[q] = 0.0;
    /* backward: lambda holds dL/df^{n+1} (zero after the last step) */
    for (long n = nsteps - 1; n >= 0; --n) {
        const double *fn = traj + (size_t)Q * N * n;
        const double shape = orc_rho_in_value(s->p.wave, 0.0, 1.0, s->p.omega, s->p.t_n, t0 + n + 1);
        const double rho_in = s->p.rho_f + amp * shape;
        for (long q = 0; q < (long)Q * N; ++q) mu[q] = 0.0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    long x = ((long)k * ny + j) * nx + i;
                    if (s->owner[x] >= 0) continue;
                    /* pre-face populations: streaming and walls from f^n */
                    double g0[Q], g[Q];
                    for (int e = 0; e < Q; ++e) {
                        if (e == 18) { g0[e] = fn[e * N + x]; continue; }
                        int si, sj, sk;
                        int kind = source_of(s, i, j, k, e, &si, &sj, &sk);
                        int d = opposite(e);
                        if (kind == 2) { g0[e] = 0.0; continue; }
                        if (kind == 1) { g0[e] = fn[d * N + x]; continue; }
                        long sn = ((long)sk * ny + sj) * nx + si;
                        int q = s->owner[sn];
                        if (q < 0) { g0[e] = fn[e * N + sn]; continue; }
                        double xb[3] = {i + 0.5 * CX[d], j + 0.5 * CY[d], k + 0.5 * CZ[d]};
                        double r[3], wr[3];
                        for (int a = 0; a < 3; ++a) r[a] = min_image(s, a, xb[a] - s->X[3 * q + a]);
                        cross(s->W + 3 * q, r, wr);
                        double vbc = (s->V[3 * q] + wr[0]) * CX[d] + (s->V[3 * q + 1] + wr[1]) * CY[d] +
                                     (s->V[3 * q + 2] + wr[2]) * CZ[d];
                        g0[e] = fn[d * N + x] - 2.0 * weight(d) / CS2 * s->p.rho_f * vbc;
                    }
                    int face = -1;
                    if (k == 0 && s->p.bc[4] == BC_PRESSURE) face = 0;
                    if (k == nz - 1 && s->p.bc[5] == BC_PRESSURE) face = 1;
                    for (int e = 0; e < Q; ++e) g[e] = g0[e];
                    if (face >= 0) zou_he(g, face == 0 ? rho_in : s->p.rho_f, face);
                    /* dL/dg: collision transpose and the probe term */
                    double J[Q][Q], rho, jm[3], u[3], feq[Q];
                    collide_jacobian(g, tau, J);
                    moments(g, &rho, jm);
                    for (int a = 0; a < 3; ++a) u[a] = jm[a] / rho;
                    equilibrium(rho, u, feq);
                    double dg[Q];
                    for (int e = 0; e < Q; ++e) {
                        double acc = 0.0;
                        for (int d = 0; d < Q; ++d) acc += lam[d * N + x] * J[d][e];
                        dg[e] = acc;
                    }
                    for (int pz = 0; pz < np; ++pz)
                        if (s->p.probe_z[pz] == k)
                            for (int e = 0; e < Q; ++e) dg[e] += dLdP[n * np + pz] / nfl[pz];
                    /* d f~ / d(1/tau) = f^eq - f */
                    for (int d = 0; d < Q; ++d) gw += lam[d * N + x] * (feq[d] - g[d]);
                    /* through the density face */
                    double dg0[Q];
                    if (face >= 0) {
                        for (int e = 0; e < Q; ++e) {
                            double acc = 0.0;
                            for (int d = 0; d < Q; ++d) acc += dg[d] * Mz[face][d][e];
                            dg0[e] = acc;
                        }
                        if (face == 0)
                            for (int d = 0; d < Q; ++d) ga += dg[d] * bz[0][d] * shape;
                    } else {
                        for (int e = 0; e < Q; ++e) dg0[e] = dg[e];
                    }
                    /* moving walls: d g0_e / dV_q = -2 (w_d / cs^2) rho_f c_d */
                    for (int e = 0; e < 18; ++e) {
                        int si, sj, sk;
                        if (source_of(s, i, j, k, e, &si, &sj, &sk) != 0) continue;
                        int q = s->owner[((long)sk * ny + sj) * nx + si];
                        if (q < 0) continue;
                        int d = opposite(e);
                        double c = -2.0 * weight(d) / CS2 * s->p.rho_f;
                        g_v[3 * q + 0] += dg0[e] * c * CX[d];
                        g_v[3 * q + 1] += dg0[e] * c * CY[d];
                        g_v[3 * q + 2] += dg0[e] * c * CZ[d];
                    }
                    for (int e = 0; e < Q; ++e) mu[e * N + x] = dg0[e];
                }
        /* streaming transpose: every f~_e(y) has one consumer */
        for (long q = 0; q < (long)Q * N; ++q) lam_prev[q] = 0.0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    long x = ((long)k * ny + j) * nx + i;
                    if (s->owner[x] >= 0) continue;
                    for (int e = 0; e < Q; ++e) {
                        if (e == 18) { lam_prev[e * N + x] += mu[e * N + x]; continue; }
                        int si, sj, sk;
                        int kind = source_of(s, i, j, k, e, &si, &sj, &sk);
                        if (kind == 2) continue;
                        int d = opposite(e);
                        if (kind == 1) { lam_prev[d * N + x] += mu[e * N + x]; continue; }
                        long sn = ((long)sk * ny + sj) * nx + si;
                        if (s->owner[sn] >= 0) lam_prev[d * N + x] += mu[e * N + x];
                        else lam_prev[e * N + sn] += mu[e * N + x];
                    }
                }
        double *tmp = lam; lam = lam_prev; lam_prev = tmp;
    }
    *g_tau = gw * (-1.0 / (tau * tau));
    *g_amp = ga;
    free(traj); free(lam); free(lam_prev); free(mu); free(nfl);
    s->frozen = frozen;
    return 0;
}
