/*
 * FP64 CPU oracle for the two-component Shan-Chen lattice Boltzmann model of
 * Milan, Biferale, Sbragaglia and Toschi, "Sub-Kolmogorov droplet dynamics in
 * isotropic turbulence using a multiscale Lattice Boltzmann scheme"
 * (arXiv 2112.09972).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library.
 *
 * Arithmetic: IEEE double, compiled with -ffp-contract=off (no FMA contraction).
 * Every phase of a time step is a separate loop over all lattice nodes, in the
 * order the method defines it, so a reader can check it against the paper:
 *
 *   state        f[s][i](x) at time n, the populations of component s after
 *                streaming (the left side of the lattice Boltzmann equation,
 *                Sec. 2 Eq. 9).
 *   1. moments   rho_s = sum_i f_i, j_s = sum_i f_i c_i             (Sec. 2 Eq. 6)
 *   2. force     F_s = -G rho_s sum_{i>0} w_i rho_{s'}(x + c_i) c_i  (Sec. 2 Eq. 7)
 *   3. velocity  u' = (sum_s j_s/tau_s) / (sum_s rho_s/tau_s),
 *                u_eq,s = u' + tau_s F_s / rho_s  (Shan-Chen velocity shift; the
 *                paper cites Shan & Chen for the model and is silent on how F
 *                enters the collision)
 *   4. collide   p_i = f_i - (f_i - g_eq_i(rho_s, u_eq,s)) / tau_s   (Sec. 2 Eq. 9
 *                with the single-rate reading of the multi-relaxation operator,
 *                Eq. 10 fixes tau; equilibrium Sec. 2 Eq. 8)
 *   5. stream    f_i(x, n+1) = p_i(x - c_i, n) when x - c_i is a lattice node;
 *                otherwise x - c_i is a ghost node holding the equilibrium of the
 *                boundary density and the imposed linear velocity
 *                u = A (x - c_i - x_c)    (Sec. 2 Eq. 8, Sec. 3 Eq. 14, Fig. 1)
 *                In periodic mode x - c_i wraps around the box instead.
 *
 * The ghost density of component s is rho_b[s]; the same value stands in for
 * the neighbour density of the force stencil at a ghost position.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19: every c in {-1,0,1}^3 with |c|^2 <= 2; weights 1/3, 1/18, 1/36 by |c|^2.
 * Filled at run time from that definition (orc_stencil_init) so the table is not
 * typed by hand. */
static int C[Q][3];
static double W[Q];
static int OPP[Q];
static int stencil_ready = 0;

static void orc_stencil_init(void) {
    if (stencil_ready) return;
    int q = 0;
    /* rest velocity first, then the rest in lexicographic order */
    C[q][0] = C[q][1] = C[q][2] = 0;
    W[q] = 1.0 / 3.0;
    q++;
    for (int cz = -1; cz <= 1; cz++)
        for (int cy = -1; cy <= 1; cy++)
            for (int cx = -1; cx <= 1; cx++) {
                int n2 = cx * cx + cy * cy + cz * cz;
                if (n2 == 0 || n2 > 2) continue;
                C[q][0] = cx;
                C[q][1] = cy;
                C[q][2] = cz;
                W[q] = (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
                q++;
            }
    for (int i = 0; i < Q; i++)
        for (int k = 0; k < Q; k++)
            if (C[k][0] == -C[i][0] && C[k][1] == -C[i][1] && C[k][2] == -C[i][2]) OPP[i] = k;
    stencil_ready = 1;
}

/* ---------------------------------------------------------------- state --- */

typedef struct {
    int nx, ny, nz;
    int periodic;     /* 1: periodic box, 0: ghost boundary with linear flow */
    double tau[2];
    double g;         /* G_AB = G_BA; G_AA = G_BB = 0 */
    double rho_b[2];  /* ghost densities of components A and B */
    double xc[3];     /* reference point of the linear flow (box centre) */
    size_t n;         /* nodes */
    double *f;        /* [2][Q][nz][ny][nx] */
    double *fn;       /* next state */
    double *rho;      /* [2][n] scratch */
    double *j;        /* [2][3][n] scratch */
    double *F;        /* [2][3][n] scratch */
    int64_t step;
} orc_state;

static size_t nid(const orc_state *s, int x, int y, int z) {
    return ((size_t)z * s->ny + y) * s->nx + x;
}
static double *fptr(const orc_state *s, double *base, int comp, int i) {
    return base + ((size_t)comp * Q + i) * s->n;
}

/* Second-order equilibrium, Sec. 2 Eq. 8: w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2). */
static double geq(int i, double rho, const double u[3]) {
    double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

int orc_q(void) { return Q; }

/* Threads the OpenMP loops of this oracle use. */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads of the following OpenMP loops (timing on 1 core and on all). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_stencil(int *c_out /* [Q][3] */, double *w_out /* [Q] */) {
    orc_stencil_init();
    for (int i = 0; i < Q; i++) {
        for (int k = 0; k < 3; k++) c_out[3 * i + k] = C[i][k];
        w_out[i] = W[i];
    }
}

void orc_equilibrium(double rho, const double *u, double *out /* [Q] */) {
    orc_stencil_init();
    for (int i = 0; i < Q; i++) out[i] = geq(i, rho, u);
}

orc_state *orc_create(int nx, int ny, int nz, int periodic, double tau_a, double tau_b, double g,
                      double rho_b_a, double rho_b_b) {
    orc_stencil_init();
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->periodic = periodic;
    s->tau[0] = tau_a;
    s->tau[1] = tau_b;
    s->g = g;
    s->rho_b[0] = rho_b_a;
    s->rho_b[1] = rho_b_b;
    /* the droplet sits at the box centre (Sec. 3, Fig. 1) */
    s->xc[0] = 0.5 * (nx - 1);
    s->xc[1] = 0.5 * (ny - 1);
    s->xc[2] = 0.5 * (nz - 1);
    s->n = (size_t)nx * ny * nz;
    s->f = (double *)calloc(2 * Q * s->n, sizeof(double));
    s->fn = (double *)calloc(2 * Q * s->n, sizeof(double));
    s->rho = (double *)calloc(2 * s->n, sizeof(double));
    s->j = (double *)calloc(6 * s->n, sizeof(double));
    s->F = (double *)calloc(6 * s->n, sizeof(double));
    if (!s->f || !s->fn || !s->rho || !s->j || !s->F) {
        free(s->f); free(s->fn); free(s->rho); free(s->j); free(s->F); free(s);
        return NULL;
    }
    return s;
}

void orc_destroy(orc_state *s) {
    if (!s) return;
    free(s->f); free(s->fn); free(s->rho); free(s->j); free(s->F);
    free(s);
}

int64_t orc_get_step(const orc_state *s) { return s->step; }
void orc_set_step(orc_state *s, int64_t n) { s->step = n; }

/* Raw populations in the oracle's own layout [2][Q][nz][ny][nx] and velocity order. */
void orc_get_f(const orc_state *s, double *out) { memcpy(out, s->f, 2 * Q * s->n * sizeof(double)); }
void orc_set_f(orc_state *s, const double *in) { memcpy(s->f, in, 2 * Q * s->n * sizeof(double)); }

/* Initial state from arbitrary fields: f_i^s = g_eq_i(rho_s, u) at every node. */
void orc_init_fields(orc_state *s, const double *rho_a, const double *rho_b, const double *u /* [3][n] */) {
    for (size_t k = 0; k < s->n; k++) {
        double uu[3] = {u[k], u[s->n + k], u[2 * s->n + k]};
        for (int i = 0; i < Q; i++) {
            fptr(s, s->f, 0, i)[k] = geq(i, rho_a[k], uu);
            fptr(s, s->f, 1, i)[k] = geq(i, rho_b[k], uu);
        }
    }
    s->step = 0;
}

/* Spherical droplet of component A at centre `ctr`: a tanh profile of width xi
 * between rho_in (inside) and rho_out (outside); component B is the mirror
 * profile so that rho_A + rho_B = rho_in + rho_out everywhere.  Velocity
 * u = A0 (x - x_c).  The paper only says the droplet sits at the centre of the
 * box; the tanh profile is a reading. */
void orc_init_droplet(orc_state *s, const double *ctr, double radius, double xi, double rho_in,
                      double rho_out, const double *A0 /* 9, row-major, A_ij = d_j u_i */) {
    double *ra = (double *)malloc(s->n * sizeof(double));
    double *rb = (double *)malloc(s->n * sizeof(double));
    double *u = (double *)malloc(3 * s->n * sizeof(double));
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = nid(s, x, y, z);
                double dx = x - ctr[0], dy = y - ctr[1], dz = z - ctr[2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                ra[k] = 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * tanh((r - radius) / xi);
                rb[k] = rho_in + rho_out - ra[k];
                double d[3] = {x - s->xc[0], y - s->xc[1], z - s->xc[2]};
                for (int a = 0; a < 3; a++)
                    u[a * s->n + k] = A0[3 * a + 0] * d[0] + A0[3 * a + 1] * d[1] + A0[3 * a + 2] * d[2];
            }
    orc_init_fields(s, ra, rb, u);
    free(ra); free(rb); free(u);
}

/* ------------------------------------------------------------- phases ----- */

/* Phase 1, Sec. 2 Eq. 6: per-component density and momentum of the current f. */
static void phase_moments(orc_state *s) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = nid(s, x, y, z);
                for (int c = 0; c < 2; c++) {
                    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
                    for (int i = 0; i < Q; i++) {
                        double v = fptr(s, s->f, c, i)[k];
                        r += v;
                        jx += v * C[i][0];
                        jy += v * C[i][1];
                        jz += v * C[i][2];
                    }
                    s->rho[c * s->n + k] = r;
                    s->j[(c * 3 + 0) * s->n + k] = jx;
                    s->j[(c * 3 + 1) * s->n + k] = jy;
                    s->j[(c * 3 + 2) * s->n + k] = jz;
                }
            }
}

/* Density of component c at lattice position (x,y,z), which may lie outside the
 * box: wrapped in periodic mode, the ghost density otherwise. */
static double rho_at(const orc_state *s, int c, int x, int y, int z) {
    if (s->periodic) {
        x = (x + s->nx) % s->nx;
        y = (y + s->ny) % s->ny;
        z = (z + s->nz) % s->nz;
    } else if (x < 0 || x >= s->nx || y < 0 || y >= s->ny || z < 0 || z >= s->nz) {
        return s->rho_b[c];
    }
    return s->rho[c * s->n + nid(s, x, y, z)];
}

/* Phase 2, Sec. 2 Eq. 7: F_s = -rho_s sum_{s' != s} G_{ss'} sum_i w_i rho_{s'}(x + c_i) c_i. */
static void phase_force(orc_state *s) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = nid(s, x, y, z);
                for (int c = 0; c < 2; c++) {
                    int other = 1 - c;
                    double sx = 0.0, sy = 0.0, sz = 0.0;
                    for (int i = 1; i < Q; i++) {
                        double r = rho_at(s, other, x + C[i][0], y + C[i][1], z + C[i][2]);
                        sx += W[i] * r * C[i][0];
                        sy += W[i] * r * C[i][1];
                        sz += W[i] * r * C[i][2];
                    }
                    double pre = -s->g * s->rho[c * s->n + k];
                    s->F[(c * 3 + 0) * s->n + k] = pre * sx;
                    s->F[(c * 3 + 1) * s->n + k] = pre * sy;
                    s->F[(c * 3 + 2) * s->n + k] = pre * sz;
                }
            }
}

/* Phases 3 and 4: velocity shift and single-rate collision; result into s->fn
 * at the same node (post-collision, not yet streamed). */
static void phase_collide(orc_state *s) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = nid(s, x, y, z);
                double num[3] = {0.0, 0.0, 0.0}, den = 0.0;
                for (int c = 0; c < 2; c++) {
                    for (int a = 0; a < 3; a++) num[a] += s->j[(c * 3 + a) * s->n + k] / s->tau[c];
                    den += s->rho[c * s->n + k] / s->tau[c];
                }
                double up[3] = {num[0] / den, num[1] / den, num[2] / den};
                for (int c = 0; c < 2; c++) {
                    double r = s->rho[c * s->n + k];
                    double ueq[3];
                    for (int a = 0; a < 3; a++) ueq[a] = up[a] + s->tau[c] * s->F[(c * 3 + a) * s->n + k] / r;
                    for (int i = 0; i < Q; i++) {
                        double fi = fptr(s, s->f, c, i)[k];
                        fptr(s, s->fn, c, i)[k] = fi - (fi - geq(i, r, ueq)) / s->tau[c];
                    }
                }
            }
}

/* Phase 5: streaming of the post-collision populations (held in s->fn) into
 * s->f, with ghost equilibria for sources outside the box. */
static void phase_stream(orc_state *s, const double *A) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = nid(s, x, y, z);
                for (int i = 0; i < Q; i++) {
                    int sx = x - C[i][0], sy = y - C[i][1], sz = z - C[i][2];
                    int inside = sx >= 0 && sx < s->nx && sy >= 0 && sy < s->ny && sz >= 0 && sz < s->nz;
                    if (s->periodic || inside) {
                        sx = (sx + s->nx) % s->nx;
                        sy = (sy + s->ny) % s->ny;
                        sz = (sz + s->nz) % s->nz;
                        size_t ks = nid(s, sx, sy, sz);
                        for (int c = 0; c < 2; c++) fptr(s, s->f, c, i)[k] = fptr(s, s->fn, c, i)[ks];
                    } else {
                        /* ghost node at (sx,sy,sz): boundary density, velocity A (x_g - x_c) */
                        double d[3] = {sx - s->xc[0], sy - s->xc[1], sz - s->xc[2]};
                        double u[3];
                        for (int a = 0; a < 3; a++) u[a] = A[3 * a + 0] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2];
                        for (int c = 0; c < 2; c++) fptr(s, s->f, c, i)[k] = geq(i, s->rho_b[c], u);
                    }
                }
            }
}

/* One time step n -> n+1.  A (9 doubles, row-major, A_ij = d_j u_i) is the
 * velocity gradient the ghost nodes carry during this step's streaming; it is
 * ignored in periodic mode. */
void orc_step(orc_state *s, const double *A) {
    static const double zero[9] = {0};
    if (!A) A = zero;
    phase_moments(s);
    phase_force(s);
    phase_collide(s);
    phase_stream(s, A);
    s->step++;
}

void orc_run(orc_state *s, const double *Atab /* [nsteps][9] or NULL */, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; t++) orc_step(s, Atab ? Atab + 9 * t : NULL);
}

/* ---------------------------------------------------------- observables --- */

/* Density fields, force fields and barycentric velocity of the current state.
 * u = (j_A + j_B + (F_A + F_B)/2) / (rho_A + rho_B): Sec. 2 Eq. 6 plus the half
 * force that the Shan-Chen model adds to the fluid velocity. */
void orc_fields(orc_state *s, double *rho_a, double *rho_b, double *u /* [3][n] or NULL */,
                double *force /* [2][3][n] or NULL */) {
    phase_moments(s);
    phase_force(s);
    for (size_t k = 0; k < s->n; k++) {
        if (rho_a) rho_a[k] = s->rho[k];
        if (rho_b) rho_b[k] = s->rho[s->n + k];
        double rt = s->rho[k] + s->rho[s->n + k];
        for (int a = 0; a < 3; a++) {
            double m = s->j[(0 * 3 + a) * s->n + k] + s->j[(1 * 3 + a) * s->n + k] +
                       0.5 * (s->F[(0 * 3 + a) * s->n + k] + s->F[(1 * 3 + a) * s->n + k]);
            if (u) u[a * s->n + k] = m / rt;
        }
        if (force)
            for (int c = 0; c < 2; c++)
                for (int a = 0; a < 3; a++) force[(c * 3 + a) * s->n + k] = s->F[(c * 3 + a) * s->n + k];
    }
}

/* Total mass of each component and total momentum sum_x (j_A + j_B), summed in
 * node order. */
void orc_totals(orc_state *s, double *mass /* 2 */, double *mom /* 3 */) {
    phase_moments(s);
    mass[0] = mass[1] = 0.0;
    mom[0] = mom[1] = mom[2] = 0.0;
    for (size_t k = 0; k < s->n; k++) {
        mass[0] += s->rho[k];
        mass[1] += s->rho[s->n + k];
        for (int a = 0; a < 3; a++) mom[a] += s->j[(0 * 3 + a) * s->n + k] + s->j[(1 * 3 + a) * s->n + k];
    }
}

/* Droplet moments of the indicator phi = [rho_A > rho_B] about the point ctr:
 * out = {S0, S1x, S1y, S1z, S2xx, S2xy, S2xz, S2yy, S2yz, S2zz}. */
void orc_droplet_moments(int nx, int ny, int nz, const double *rho_a, const double *rho_b,
                         const double *ctr, double *out) {
    for (int k = 0; k < 10; k++) out[k] = 0.0;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                size_t k = ((size_t)z * ny + y) * nx + x;
                if (!(rho_a[k] > rho_b[k])) continue;
                double d[3] = {x - ctr[0], y - ctr[1], z - ctr[2]};
                out[0] += 1.0;
                out[1] += d[0];
                out[2] += d[1];
                out[3] += d[2];
                out[4] += d[0] * d[0];
                out[5] += d[0] * d[1];
                out[6] += d[0] * d[2];
                out[7] += d[1] * d[1];
                out[8] += d[1] * d[2];
                out[9] += d[2] * d[2];
            }
}

/* ---------------------------------------------- droplet surface and mass --- */

/* Zero-level-set point on the edge from p (phi_p > 0) to q (phi_q <= 0). */
static void edge_point(const double *p, const double *q, double fp, double fq, double *out) {
    double t = fp / (fp - fq);
    for (int a = 0; a < 3; a++) out[a] = p[a] + t * (q[a] - p[a]);
}

static double tri_area(const double *a, const double *b, const double *c) {
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; k++) {
        u[k] = b[k] - a[k];
        v[k] = c[k] - a[k];
    }
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

static double tet_volume(const double *a, const double *b, const double *c, const double *d) {
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; k++) {
        u[k] = b[k] - a[k];
        v[k] = c[k] - a[k];
        w[k] = d[k] - a[k];
    }
    double det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                 u[2] * (v[0] * w[1] - v[1] * w[0]);
    return fabs(det) / 6.0;
}

/* Area of {phi = 0} and volume of {phi > 0} inside one tetrahedron (phi linear
 * between the four vertex values). */
static void tet_surface(double P[4][3], const double *phi, double *area, double *vol) {
    int pos[4], neg[4], np = 0, nn = 0;
    for (int i = 0; i < 4; i++) {
        if (phi[i] > 0.0)
            pos[np++] = i;
        else
            neg[nn++] = i;
    }
    if (np == 0) return;
    if (np == 4) {
        *vol += tet_volume(P[0], P[1], P[2], P[3]);
        return;
    }
    if (np == 1) {
        /* a corner tetrahedron cut off around the one positive vertex */
        int a = pos[0];
        double X[3][3];
        for (int k = 0; k < 3; k++) edge_point(P[a], P[neg[k]], phi[a], phi[neg[k]], X[k]);
        *area += tri_area(X[0], X[1], X[2]);
        *vol += tet_volume(P[a], X[0], X[1], X[2]);
    } else if (np == 3) {
        /* the whole tetrahedron minus the corner around the one non-positive vertex */
        int d = neg[0];
        double X[3][3];
        for (int k = 0; k < 3; k++) edge_point(P[pos[k]], P[d], phi[pos[k]], phi[d], X[k]);
        *area += tri_area(X[0], X[1], X[2]);
        *vol += tet_volume(P[0], P[1], P[2], P[3]) - tet_volume(P[d], X[0], X[1], X[2]);
    } else {
        /* two and two: a quadrilateral cut; the positive part is a prism with the
         * triangles (a, Xac, Xad) and (b, Xbc, Xbd) as ends */
        int a = pos[0], b = pos[1], c = neg[0], d = neg[1];
        double Xac[3], Xad[3], Xbc[3], Xbd[3];
        edge_point(P[a], P[c], phi[a], phi[c], Xac);
        edge_point(P[a], P[d], phi[a], phi[d], Xad);
        edge_point(P[b], P[c], phi[b], phi[c], Xbc);
        edge_point(P[b], P[d], phi[b], phi[d], Xbd);
        /* quadrilateral Xac - Xad - Xbd - Xbc (consecutive corners share a face) */
        *area += tri_area(Xac, Xad, Xbd) + tri_area(Xac, Xbd, Xbc);
        *vol += tet_volume(P[a], Xac, Xad, P[b]) + tet_volume(Xac, Xad, P[b], Xbd) + tet_volume(Xac, P[b], Xbc, Xbd);
    }
}

/* Surface area of the droplet, the level set rho_A = rho_B, and the volume it
 * encloses, for the D_LBM measure of Sec. 5 Eq. 17 (which needs the surface
 * area of the deformed droplet and of the sphere of equal volume).  The paper
 * does not say how the area is measured; here phi = rho_A - rho_B is taken as
 * linear inside each of the six tetrahedra of every lattice cell (the cells
 * split along their main diagonal), the zero set in each tetrahedron is a
 * triangle or a planar quadrilateral, and the areas and the volumes of
 * {phi > 0} are summed over all cells in node order.  out = {area, volume}. */
void orc_droplet_surface(int nx, int ny, int nz, const double *rho_a, const double *rho_b, double *out) {
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    double area = 0.0, vol = 0.0;
    for (int z = 0; z + 1 < nz; z++)
        for (int y = 0; y + 1 < ny; y++)
            for (int x = 0; x + 1 < nx; x++) {
                for (int t = 0; t < 6; t++) {
                    double P[4][3], phi[4];
                    int v[3] = {x, y, z};
                    for (int i = 0; i < 4; i++) {
                        if (i > 0) v[perms[t][i - 1]] += 1;
                        size_t k = ((size_t)v[2] * ny + v[1]) * nx + v[0];
                        P[i][0] = v[0];
                        P[i][1] = v[1];
                        P[i][2] = v[2];
                        phi[i] = rho_a[k] - rho_b[k];
                    }
                    tet_surface(P, phi, &area, &vol);
                }
            }
    out[0] = area;
    out[1] = vol;
}

/* Droplet mass of component A: sum of rho_A over the nodes with rho_A > rho_B
 * (node order). */
double orc_droplet_mass(orc_state *s) {
    phase_moments(s);
    double m = 0.0;
    for (size_t k = 0; k < s->n; k++)
        if (s->rho[k] > s->rho[s->n + k]) m += s->rho[k];
    return m;
}

/* Mass reinjection (Sec. 2: the boundary scheme does not conserve mass, and mass
 * is reinjected into the droplet to keep its density fixed).  Reading: every A
 * population at the droplet nodes (rho_A > rho_B) is multiplied by
 * target / M, M the droplet mass of orc_droplet_mass, so that the droplet mass
 * becomes target; the velocity of component A is unchanged.  Returns M. */
double orc_reinject(orc_state *s, double target) {
    double m = orc_droplet_mass(s);
    double scale = target / m;
    for (size_t k = 0; k < s->n; k++) {
        if (!(s->rho[k] > s->rho[s->n + k])) continue;
        for (int i = 0; i < Q; i++) fptr(s, s->f, 0, i)[k] *= scale;
    }
    return m;
}
