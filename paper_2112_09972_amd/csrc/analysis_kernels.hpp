// Droplet surface (for D_LBM, Sec. 5 Eq. 17), droplet mass and mass reinjection
// (Sec. 2: the open boundary does not conserve mass; mass is put back into the
// droplet so that its density stays fixed).
#pragma once

#include "aux_kernels.hpp"

namespace sclbm {

constexpr int SURF_T = 16;               // cells per tile edge (x and y); one thread per cell
constexpr int SURF_P = SURF_T + 1;       // nodes per tile edge

// Zero set of phi (linear inside the tetrahedron with corners p[0..3], values s[0..3]):
// adds its area and the volume of {phi > 0}.  The volume uses the edge fractions of the
// cut (barycentric closed forms); the tetrahedron's volume is 1/6 (one sixth of a cell).
__device__ __forceinline__ double tri_area2(const double *a, const double *b, const double *c) {
    const double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    const double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
    const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
    return sqrt(wx * wx + wy * wy + wz * wz);  // twice the area
}

__device__ __forceinline__ void cut_point(const double *p, const double *q, double t, double *x) {
    x[0] = p[0] + t * (q[0] - p[0]);
    x[1] = p[1] + t * (q[1] - p[1]);
    x[2] = p[2] + t * (q[2] - p[2]);
}

__device__ __forceinline__ void tet_cut(const double (&p)[4][3], const double (&s)[4], double &area, double &vol) {
    int ip[4], in[4], np = 0, nn = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (s[i] > 0.0) ip[np++] = i;
        else in[nn++] = i;
    }
    constexpr double V6 = 1.0 / 6.0;
    if (np == 0) return;
    if (np == 4) {
        vol += V6;
        return;
    }
    if (np == 1 || np == 3) {
        // one vertex v alone on its side; t_k = fraction from v along the edge to the others
        const int v = np == 1 ? ip[0] : in[0];
        const int o0 = np == 1 ? in[0] : ip[0], o1 = np == 1 ? in[1] : ip[1], o2 = np == 1 ? in[2] : ip[2];
        const double t0 = s[v] / (s[v] - s[o0]), t1 = s[v] / (s[v] - s[o1]), t2 = s[v] / (s[v] - s[o2]);
        double x0[3], x1[3], x2[3];
        cut_point(p[v], p[o0], t0, x0);
        cut_point(p[v], p[o1], t1, x1);
        cut_point(p[v], p[o2], t2, x2);
        area += 0.5 * tri_area2(x0, x1, x2);
        const double corner = V6 * t0 * t1 * t2;
        vol += np == 1 ? corner : V6 - corner;
        return;
    }
    // two and two: a, b positive, c, d not
    const int a = ip[0], b = ip[1], c = in[0], d = in[1];
    const double al = s[a] / (s[a] - s[c]), be = s[a] / (s[a] - s[d]);
    const double ga = s[b] / (s[b] - s[c]), de = s[b] / (s[b] - s[d]);
    double xac[3], xad[3], xbc[3], xbd[3];
    cut_point(p[a], p[c], al, xac);
    cut_point(p[a], p[d], be, xad);
    cut_point(p[b], p[c], ga, xbc);
    cut_point(p[b], p[d], de, xbd);
    // planar quadrilateral xac, xad, xbd, xbc: half the cross product of its diagonals
    const double ex = xbd[0] - xac[0], ey = xbd[1] - xac[1], ez = xbd[2] - xac[2];
    const double fx = xbc[0] - xad[0], fy = xbc[1] - xad[1], fz = xbc[2] - xad[2];
    const double cx = ey * fz - ez * fy, cy = ez * fx - ex * fz, cz = ex * fy - ey * fx;
    area += 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    // the positive part is a prism; its three tetrahedra have volume fractions
    // al be, al de (1 - be) and (1 - al) ga de of the whole
    vol += V6 * (al * be + al * de * (1.0 - be) + (1.0 - al) * ga * de);
}

// Area of {phi = 0} and volume of {phi > 0}, phi = rho_A - rho_B, over the cells of each
// box.  Grid (tile blocks, boxes); a block takes tiles of 16 x 16 cells, marching in z
// with two planes of phi in LDS (each node's populations read about 1.13 times).
template <int P>
__global__ __launch_bounds__(NRED_THREADS) void k_surface(const typename Prec<P>::S *f, const __half *ref, BoxGeom g,
                                                          int b0, int ntx, int ntiles, double *partial) {
    static_assert(NRED_THREADS == SURF_T * SURF_T, "one thread per cell of a tile");
    const int box = b0 + blockIdx.y;
    f += (int64_t)box * 2 * Q * g.nnode;
    if (Prec<P>::DEV) ref += (int64_t)box * 2 * g.nnode;
    __shared__ double ph[2][SURF_P * SURF_P];
    const int ci = threadIdx.x % SURF_T, cj = threadIdx.x / SURF_T;
    double v[2] = {0.0, 0.0};
    // the six tetrahedra of a cell: corner 0, then one unit step along each axis in turn
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % ntx) * SURF_T, y0 = (tile / ntx) * SURF_T;
        for (int z = 0; z < g.nz; ++z) {
            double *dst = ph[z & 1];
            for (int n = threadIdx.x; n < SURF_P * SURF_P; n += NRED_THREADS) {
                const int x = x0 + n % SURF_P, y = y0 + n / SURF_P;
                double val = 0.0;
                if (x < g.nx && y < g.ny) {
                    double rho[2], j[2][3];
                    node_moments<P>(f, ref, g, ((int64_t)z * g.ny + y) * g.nx + x, rho, j);
                    val = rho[0] - rho[1];
                }
                dst[n] = val;
            }
            __syncthreads();
            const int x = x0 + ci, y = y0 + cj;
            if (z > 0 && x + 1 < g.nx && y + 1 < g.ny) {
                const double *lo = ph[(z - 1) & 1], *hi = ph[z & 1];
                double c8[2][2][2];  // [dz][dy][dx]
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        c8[0][dy][dx] = lo[(cj + dy) * SURF_P + ci + dx];
                        c8[1][dy][dx] = hi[(cj + dy) * SURF_P + ci + dx];
                    }
                bool any_pos = false, any_neg = false;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double s = c8[q >> 2][(q >> 1) & 1][q & 1];
                    any_pos |= s > 0.0;
                    any_neg |= !(s > 0.0);
                }
                if (any_pos && !any_neg) {
                    v[1] += 1.0;                 // a cell wholly inside
                } else if (any_pos) {
                    // coordinates relative to the cell's corner (the sums are translation invariant)
#pragma unroll
                    for (int t = 0; t < 6; ++t) {
                        double pp[4][3], ss[4];
                        int o[3] = {0, 0, 0};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (k > 0) o[perm[t][k - 1]] = 1;
                            pp[k][0] = o[0];
                            pp[k][1] = o[1];
                            pp[k][2] = o[2];
                            ss[k] = c8[o[2]][o[1]][o[0]];
                        }
                        tet_cut(pp, ss, v[0], v[1]);
                    }
                }
            }
            __syncthreads();
        }
    }
    block_reduce_store<2>(v, partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2);
}

// Per-block partial sums of rho_A over the droplet nodes (rho_A > rho_B); grid (blocks, boxes).
template <int P>
__global__ __launch_bounds__(NRED_THREADS) void k_drop_mass(const typename Prec<P>::S *f, const __half *ref,
                                                            BoxGeom g, int b0, double *partial) {
    const int box = b0 + blockIdx.y;
    f += (int64_t)box * 2 * Q * g.nnode;
    if (Prec<P>::DEV) ref += (int64_t)box * 2 * g.nnode;
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < g.nnode; k += stride) {
        double rho[2], j[2][3];
        node_moments<P>(f, ref, g, k, rho, j);
        if (rho[0] > rho[1]) v[0] += rho[0];
    }
    block_reduce_store<1>(v, partial + (int64_t)blockIdx.y * gridDim.x + blockIdx.x);
}

// Reinjection: at every droplet node of box b0 + blockIdx.y, scale component A by
// target[box] / mass[box] (every population; for the deviation formats, whose
// populations are w_i rho_ref (1 + d_i), the node's reference density instead).
template <int P>
__global__ __launch_bounds__(256) void k_reinject(typename Prec<P>::S *f, __half *ref, BoxGeom g, int b0,
                                                  const double *mass, const double *target) {
    using R = typename Prec<P>::R;
    const int box = b0 + blockIdx.y;
    f += (int64_t)box * 2 * Q * g.nnode;
    if (Prec<P>::DEV) ref += (int64_t)box * 2 * g.nnode;
    const double scale = target[box] / mass[box];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < g.nnode; k += stride) {
        double rho[2], j[2][3];
        node_moments<P>(f, ref, g, k, rho, j);
        if (!(rho[0] > rho[1])) continue;
        if (Prec<P>::DEV) {
            ref_store(ref + ref_index(k, 0), float(double(ref_load(ref + ref_index(k, 0))) * scale));
        } else {
            const int64_t e = pop_base(g, k);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                typename Prec<P>::S *p = f + e + (int64_t)i * g.nx;
                Prec<P>::store(p, R(double(Prec<P>::load(p, R(0))) * scale), R(0));
            }
        }
    }
}

}  // namespace sclbm
