/*
 * Memory and undefined-behaviour check of the FP64 oracle (TEST INFRASTRUCTURE):
 * a driver that exercises every entry point of sclbm_oracle.c on small ragged
 * boxes, built together with it under -fsanitize=address,undefined by
 * tests/test_oracle_sanitized.py.  Any sanitizer report ends the program with a
 * non-zero status.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_state orc_state;
orc_state *orc_create(int nx, int ny, int nz, int periodic, double tau_a, double tau_b, double g, double rho_b_a,
                      double rho_b_b);
void orc_destroy(orc_state *s);
void orc_init_droplet(orc_state *s, const double *ctr, double radius, double xi, double rho_in, double rho_out,
                      const double *A0);
void orc_init_fields(orc_state *s, const double *rho_a, const double *rho_b, const double *u);
void orc_run(orc_state *s, const double *Atab, int64_t nsteps);
void orc_fields(orc_state *s, double *rho_a, double *rho_b, double *u, double *force);
void orc_totals(orc_state *s, double *mass, double *mom);
void orc_droplet_moments(int nx, int ny, int nz, const double *rho_a, const double *rho_b, const double *center,
                         double *out);
void orc_droplet_surface(int nx, int ny, int nz, const double *rho_a, const double *rho_b, double *out);
double orc_droplet_mass(orc_state *s);
double orc_reinject(orc_state *s, double target);
void orc_get_f(const orc_state *s, double *out);
void orc_set_f(orc_state *s, const double *in);

static int run_case(int nx, int ny, int nz, int periodic) {
    const int64_t n = (int64_t)nx * ny * nz;
    orc_state *s = orc_create(nx, ny, nz, periodic, 1.0, 1.3, 1.6417, 0.05, 1.0);
    if (!s) return 1;
    const double ctr[3] = {0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1)};
    const double A[9] = {0.001, 0.0, 0.003, 0.0, -0.0005, 0.0, 0.0004, 0.0, -0.0005};
    double *tab = malloc(sizeof(double) * 9 * 7);
    double *ra = malloc(sizeof(double) * n), *rb = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * 3 * n);
    double *F = malloc(sizeof(double) * 6 * n), *f = malloc(sizeof(double) * 2 * 19 * n);
    if (!tab || !ra || !rb || !u || !F || !f) return 1;
    for (int t = 0; t < 7; ++t)
        for (int k = 0; k < 9; ++k) tab[9 * t + k] = A[k];
    const double rest[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    orc_init_droplet(s, ctr, 2.5, 2.0, 1.0, 0.04, periodic ? rest : A);
    orc_run(s, periodic ? NULL : tab, 7);
    orc_fields(s, ra, rb, u, F);
    orc_fields(s, ra, rb, NULL, NULL);
    double mass[2], mom[3], mom10[10], surf[2];
    orc_totals(s, mass, mom);
    orc_droplet_moments(nx, ny, nz, ra, rb, ctr, mom10);
    orc_droplet_surface(nx, ny, nz, ra, rb, surf);
    const double m = orc_droplet_mass(s);
    orc_reinject(s, 1.01 * m);
    orc_get_f(s, f);
    orc_set_f(s, f);
    orc_init_fields(s, ra, rb, u);
    orc_run(s, periodic ? NULL : tab, 3);
    printf("%dx%dx%d %s: mass %.6f %.6f droplet %.4f area %.4f\n", nx, ny, nz, periodic ? "periodic" : "ghost",
           mass[0], mass[1], m, surf[0]);
    free(tab); free(ra); free(rb); free(u); free(F); free(f);
    orc_destroy(s);
    return 0;
}

int main(void) {
    int bad = 0;
    bad |= run_case(9, 7, 5, 0);
    bad |= run_case(9, 7, 5, 1);
    bad |= run_case(3, 4, 6, 0);
    bad |= run_case(4, 3, 3, 1);
    return bad;
}
