// Fused stream-and-collide step of the two-component Shan-Chen model
// (arXiv 2112.09972, Sec. 2 Eqs. 6-9, ghost boundary of Sec. 2 Eq. 8 and Sec. 3
// Eq. 14) for gfx950.
//
// State: f(n), the populations of both components after streaming, SoA
// [box][component][direction][z][y][x] with x fastest.  One launch computes
// f(n+1) into the other buffer:
//   moments (Eq. 6) -> pair force from neighbour densities (Eq. 7) ->
//   velocity shift -> single-rate collision (Eq. 9) -> push to x + c_i, and on
//   boundary nodes the populations that stream in from the ghost nodes.
//
// Tiling.  A workgroup owns a tile of 64 x TY nodes in (x, y) (one wavefront per
// row, so every population stream is a coalesced 64-wide access) and marches
// along z through a chunk of planes.  The force at plane z needs the densities
// of planes z-1, z, z+1 including a one-node ring around the tile; those
// densities live in a 4-slot rolling buffer in LDS.  Each plane's populations
// are loaded once into registers, held for one plane while the next plane's
// densities arrive, then collided and stored.  Ring densities (and the two
// chunk-end planes) are recomputed from HBM/L2 rather than exchanged between
// workgroups, so a step is a single launch with no grid-wide synchronisation.
#pragma once

#include "lattice.hpp"

namespace sclbm {

struct StepArgs {
    const void *src;          // f(n), all boxes
    void *dst;                // f(n+1), all boxes
    const double *atab;       // [nbox][table_len][9] velocity-gradient rows (ghost mode)
    const int64_t *tab_first; // [nbox] step of row 0
    const int64_t *clk_in;    // time n (device counter, read)
    int64_t *clk_out;         // time n+1 (device counter, written once)
    int64_t table_len;
    int64_t nnode;            // nodes per box
    int nx, ny, nz, nzc, zchunk;
    int ghost;
    double omega[2];          // 1/tau
    double tau[2];
    double g;                 // G_AB
    double rho_b[2];          // ghost densities
    double rho_ref[2];        // reference densities of the deviation formats
    double xc[3];             // box centre
};

// Density of both components at an in-box node (x,y,z) of one box.
template <int P>
__device__ __forceinline__ void node_density(const typename Prec<P>::S *f, int64_t N, int64_t idx,
                                             const typename Prec<P>::R wref[2][Q],
                                             typename Prec<P>::R out[2]) {
    using R = typename Prec<P>::R;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        R acc = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += R(Prec<P>::load(f + (int64_t)(s * Q + i) * N + idx, wref[s][i]));
        out[s] = acc;
    }
}

template <int P, int TY>
__global__ __launch_bounds__(64 * TY) void k_step(StepArgs a) {
    using S = typename Prec<P>::S;
    using W = typename Prec<P>::W;
    using R = typename Prec<P>::R;
    constexpr int LW = 66;  // 64 + ring
    __shared__ R lds[4][2][TY + 2][LW];

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 + lx;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * TY;
    const int box = blockIdx.z / a.nzc;
    const int zs = (blockIdx.z % a.nzc) * a.zchunk;
    const int ze = min(zs + a.zchunk, a.nz);
    const int x = x0 + lx, y = y0 + ly;
    const bool valid = (x < a.nx) && (y < a.ny);
    const int tw = min(64, a.nx - x0), th = min(TY, a.ny - y0);  // valid tile extent
    const int64_t N = a.nnode;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const S *src = (const S *)a.src + (int64_t)box * 2 * Q * N;
    S *dst = (S *)a.dst + (int64_t)box * 2 * Q * N;

    const int64_t n = *a.clk_in;
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tid == 0) *a.clk_out = n + 1;

    R wref[2][Q];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i) wref[s][i] = w_of<R>(i) * R(a.rho_ref[s]);

    const R om[2] = {R(a.omega[0]), R(a.omega[1])};
    const R tau[2] = {R(a.tau[0]), R(a.tau[1])};
    const R G = R(a.g);
    const R rhob[2] = {R(a.rho_b[0]), R(a.rho_b[1])};

    R Am[9];
    if (a.ghost) {
        const double *row = a.atab + ((int64_t)box * a.table_len + (n - a.tab_first[box])) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) Am[k] = R(row[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Am[k] = R(0);
    }

    W fprev[2][Q], fcur[2][Q];
    R rho_p[2] = {R(0), R(0)}, j_p[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
    const int ringN = 2 * (tw + 2) + 2 * th;
    const int nplanes = (ze - zs) + 2;

    for (int k = 0; k < nplanes; ++k) {
        const int z = zs - 1 + k;
        const int slot = k & 3;
        // ---- 1. own node of plane z: populations into registers, moments ----
        R rho_c[2] = {R(0), R(0)}, j_c[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
        if (valid) {
            int zz = z;
            bool inside = (z >= 0) && (z < nz);
            if (!inside && !a.ghost) {
                zz = (z + nz) % nz;
                inside = true;
            }
            if (inside) {
                const int64_t idx = ((int64_t)zz * ny + y) * nx + x;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) fcur[s][i] = Prec<P>::load(src + (int64_t)(s * Q + i) * N + idx, wref[s][i]);
                    R r = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const R v = R(fcur[s][i]);
                        r += v;
                        if (cx_of(i)) jx += R(cx_of(i)) * v;
                        if (cy_of(i)) jy += R(cy_of(i)) * v;
                        if (cz_of(i)) jz += R(cz_of(i)) * v;
                    }
                    rho_c[s] = r;
                    j_c[s][0] = jx;
                    j_c[s][1] = jy;
                    j_c[s][2] = jz;
                }
            } else {
                rho_c[0] = rhob[0];
                rho_c[1] = rhob[1];
            }
            lds[slot][0][ly + 1][lx + 1] = rho_c[0];
            lds[slot][1][ly + 1][lx + 1] = rho_c[1];
        }
        // ---- 2. ring densities of plane z ----
        for (int r = tid; r < ringN; r += 64 * TY) {
            int sx, sy;
            if (r < tw + 2) {
                sx = r;
                sy = 0;
            } else if (r < 2 * (tw + 2)) {
                sx = r - (tw + 2);
                sy = th + 1;
            } else if (r < 2 * (tw + 2) + th) {
                sx = 0;
                sy = r - 2 * (tw + 2) + 1;
            } else {
                sx = tw + 1;
                sy = r - 2 * (tw + 2) - th + 1;
            }
            int gx = x0 - 1 + sx, gy = y0 - 1 + sy, gz = z;
            bool inside = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            R rr[2];
            if (!inside && !a.ghost) {
                gx = (gx + nx) % nx;
                gy = (gy + ny) % ny;
                gz = (gz + nz) % nz;
                inside = true;
            }
            if (inside) {
                node_density<P>(src, N, ((int64_t)gz * ny + gy) * nx + gx, wref, rr);
            } else {
                rr[0] = rhob[0];
                rr[1] = rhob[1];
            }
            lds[slot][0][sy][sx] = rr[0];
            lds[slot][1][sy][sx] = rr[1];
        }
        __syncthreads();

        // ---- 3. collide plane z-1 and push ----
        if (k >= 2 && valid) {
            const int zc = z - 1;
            // pair force, Eq. 7: F_s = -G rho_s sum_i w_i rho_s'(x + c_i) c_i
            R F[2][3];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int o = 1 - s;
                R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const R nb = lds[(k - 1 + cz_of(i)) & 3][o][ly + 1 + cy_of(i)][lx + 1 + cx_of(i)];
                    const R wn = w_of<R>(i) * nb;
                    if (cx_of(i)) sx += R(cx_of(i)) * wn;
                    if (cy_of(i)) sy += R(cy_of(i)) * wn;
                    if (cz_of(i)) sz += R(cz_of(i)) * wn;
                }
                const R pre = -G * rho_p[s];
                F[s][0] = pre * sx;
                F[s][1] = pre * sy;
                F[s][2] = pre * sz;
            }
            // common velocity and per-component shifted equilibrium velocity
            const R den = rho_p[0] * om[0] + rho_p[1] * om[1];
            const R inv_den = R(1) / den;
            const R up[3] = {(j_p[0][0] * om[0] + j_p[1][0] * om[1]) * inv_den,
                             (j_p[0][1] * om[0] + j_p[1][1] * om[1]) * inv_den,
                             (j_p[0][2] * om[0] + j_p[1][2] * om[1]) * inv_den};
            const bool bx = (x == 0) || (x == nx - 1);
            const bool by = (y == 0) || (y == ny - 1);
            const bool bz = (zc == 0) || (zc == nz - 1);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const R sh = tau[s] / rho_p[s];
                const R ux = up[0] + sh * F[s][0];
                const R uy = up[1] + sh * F[s][1];
                const R uz = up[2] + sh * F[s][2];
                const R usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const R fe = equilibrium<R>(i, rho_p[s], ux, uy, uz, usq);
                    const R fi = R(fprev[s][i]);
                    const R p = fi - om[s] * (fi - fe);
                    int dx = x + cx_of(i), dy = y + cy_of(i), dz = zc + cz_of(i);
                    bool ok = true;
                    if (a.ghost) {
                        ok = dx >= 0 && dx < nx && dy >= 0 && dy < ny && dz >= 0 && dz < nz;
                    } else {
                        dx = dx < 0 ? dx + nx : (dx >= nx ? dx - nx : dx);
                        dy = dy < 0 ? dy + ny : (dy >= ny ? dy - ny : dy);
                        dz = dz < 0 ? dz + nz : (dz >= nz ? dz - nz : dz);
                    }
                    if (ok) Prec<P>::store(dst + (int64_t)(s * Q + i) * N + ((int64_t)dz * ny + dy) * nx + dx, p, wref[s][i]);
                }
            }
            // populations streaming in from ghost nodes (boundary nodes only)
            if (a.ghost && (bx || by || bz)) {
                const int64_t idx = ((int64_t)zc * ny + y) * nx + x;
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int gx = x - cx_of(i), gy = y - cy_of(i), gz = zc - cz_of(i);
                    const bool out = gx < 0 || gx >= nx || gy < 0 || gy >= ny || gz < 0 || gz >= nz;
                    if (out) {
                        const R dxg = R(gx) - R(a.xc[0]), dyg = R(gy) - R(a.xc[1]), dzg = R(gz) - R(a.xc[2]);
                        const R ux = Am[0] * dxg + Am[1] * dyg + Am[2] * dzg;
                        const R uy = Am[3] * dxg + Am[4] * dyg + Am[5] * dzg;
                        const R uz = Am[6] * dxg + Am[7] * dyg + Am[8] * dzg;
                        const R usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
                        for (int s = 0; s < 2; ++s)
                            Prec<P>::store(dst + (int64_t)(s * Q + i) * N + idx,
                                           equilibrium<R>(i, rhob[s], ux, uy, uz, usq), wref[s][i]);
                    }
                }
            }
        }
        // ---- 4. roll the register window ----
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int i = 0; i < Q; ++i) fprev[s][i] = fcur[s][i];
            rho_p[s] = rho_c[s];
            j_p[s][0] = j_c[s][0];
            j_p[s][1] = j_c[s][1];
            j_p[s][2] = j_c[s][2];
        }
    }
}

}  // namespace sclbm
