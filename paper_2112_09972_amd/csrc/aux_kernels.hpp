// Initialisation, observables and FP64 reductions (arXiv 2112.09972, Sec. 2
// Eqs. 6-8, Sec. 4 Eq. 16; droplet inertia tensor for Sec. 2 Eq. 4).
//
// Reductions are deterministic: a fixed grid of NRED_BLOCKS workgroups, each
// thread accumulating a fixed strided subset of nodes in FP64, a wavefront
// butterfly (64 lanes), a fixed-order pass over the wavefronts in LDS, one
// partial per workgroup, then one workgroup summing the partials in a fixed
// order.  No atomics anywhere, so repeated runs give identical bits.
#pragma once

#include "lattice.hpp"

namespace sclbm {

constexpr int NRED_BLOCKS = 512;        // workgroups of the single-box diagnostic reductions
constexpr int NRED_MAX_PER_BOX = 1024;  // workgroups per box of the statistics reduction
constexpr int NRED_THREADS = 256;
constexpr int NSTAT = 16;  // mass 2, momentum 3, S0, S1 3, S2 6, bad-node count

struct Mat3 {
    double a[9];  // row-major, a[3*i + j] = d u_i / d x_j
};

struct BoxGeom {
    int nx, ny, nz;
    int64_t nnode;
    double xc[3];
};

// Element offset of direction 0 of node k = (z ny + y) nx + x in one component's
// population block (row-blocked order [z][y][direction][x]); direction i adds i nx.
__device__ __forceinline__ int64_t pop_base(const BoxGeom &g, int64_t k) {
    const int64_t row = k / g.nx;
    return row * (int64_t)(Q * g.nx) + (k - row * g.nx);
}

__device__ __forceinline__ void node_xyz(const BoxGeom &g, int64_t k, int &x, int &y, int &z) {
    x = (int)(k % g.nx);
    int64_t t = k / g.nx;
    y = (int)(t % g.ny);
    z = (int)(t / g.ny);
}

struct DropletInit {
    double ctr[3], radius, width, rho_in, rho_out;
    Mat3 A0;
    double u0[3];  // mode 2: uniform velocity (densities rho_in for A, rho_out for B)
};

// mode 0: tanh droplet (DropletInit); mode 1: FP64 fields rho_a, rho_b, u;
// mode 2: uniform densities (rho_in, rho_out) moving with u0.
template <int P>
__global__ __launch_bounds__(256) void k_init(typename Prec<P>::S *f, __half *ref, BoxGeom g, int mode, DropletInit d,
                                              const double *rho_a, const double *rho_b, const double *u) {
    using R = typename Prec<P>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.nnode) return;
    int x, y, z;
    node_xyz(g, k, x, y, z);
    double ra, rb, ux, uy, uz;
    if (mode == 0) {
        // tanh droplet, linear velocity about the box centre
        const double dx = x - d.ctr[0], dy = y - d.ctr[1], dz = z - d.ctr[2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        ra = 0.5 * (d.rho_in + d.rho_out) - 0.5 * (d.rho_in - d.rho_out) * tanh((r - d.radius) / d.width);
        rb = d.rho_in + d.rho_out - ra;
        const double ex = x - g.xc[0], ey = y - g.xc[1], ez = z - g.xc[2];
        const double *A = d.A0.a;
        ux = A[0] * ex + A[1] * ey + A[2] * ez;
        uy = A[3] * ex + A[4] * ey + A[5] * ez;
        uz = A[6] * ex + A[7] * ey + A[8] * ez;
    } else if (mode == 2) {
        ra = d.rho_in;
        rb = d.rho_out;
        ux = d.u0[0];
        uy = d.u0[1];
        uz = d.u0[2];
    } else {
        ra = rho_a[k];
        rb = rho_b[k];
        if (u) {
            ux = u[k];
            uy = u[g.nnode + k];
            uz = u[2 * g.nnode + k];
        } else {
            ux = uy = uz = 0.0;
        }
    }
    const double usq = ux * ux + uy * uy + uz * uz;
    const double rr[2] = {ra, rb};
    const int64_t e = pop_base(g, k);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        double rref = 0.0;
        if (Prec<P>::DEV) {
            ref_store(ref + ref_index(k, s), float(rr[s]));
            rref = ref_load(ref + ref_index(k, s));
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double fe = equilibrium<double>(i, rr[s], ux, uy, uz, usq);
            Prec<P>::store(f + pop_index<P>(g.nnode, e + (int64_t)i * g.nx, s), R(fe), R(w_of<R>(i) * R(rref)));
        }
    }
}

template <int P>
__device__ __forceinline__ void node_moments(const typename Prec<P>::S *f, const __half *ref, const BoxGeom &g,
                                             int64_t k, double rho[2], double j[2][3]) {
    using R = typename Prec<P>::R;
    const int64_t N = g.nnode;
    const int64_t e = pop_base(g, k);
    // the populations as stored (decoded in the format's arithmetic type), summed in FP64
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        const R rref = Prec<P>::DEV ? R(ref_load(ref + ref_index(k, s))) : R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double v = double(Prec<P>::load(f + pop_index<P>(N, e + (int64_t)i * g.nx, s), w_of<R>(i) * rref));
            r += v;
            if (cx_of(i)) jx += double(cx_of(i)) * v;
            if (cy_of(i)) jy += double(cy_of(i)) * v;
            if (cz_of(i)) jz += double(cz_of(i)) * v;
        }
        rho[s] = r;
        j[s][0] = jx;
        j[s][1] = jy;
        j[s][2] = jz;
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_density(const typename Prec<P>::S *f, const __half *ref, BoxGeom g,
                                                 double *rho_a, double *rho_b) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.nnode) return;
    double rho[2], j[2][3];
    node_moments<P>(f, ref, g, k, rho, j);
    rho_a[k] = rho[0];
    rho_b[k] = rho[1];
}

// Barycentric velocity with the half-force term; force from the FP64 density
// arrays written by k_density (same neighbour rules as the step kernel).
template <int P>
__global__ __launch_bounds__(256) void k_velocity(const typename Prec<P>::S *f, const __half *ref, BoxGeom g,
                                                  const double *rho_a, const double *rho_b, int ghost, double gab,
                                                  double rb0, double rb1, double *u) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.nnode) return;
    double rho[2], j[2][3];
    node_moments<P>(f, ref, g, k, rho, j);
    int x, y, z;
    node_xyz(g, k, x, y, z);
    const double *rf[2] = {rho_a, rho_b};
    const double rbnd[2] = {rb0, rb1};
    double Ft[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int o = 1 - s;
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            int nxp = x + cx_of(i), nyp = y + cy_of(i), nzp = z + cz_of(i);
            double nb;
            const bool inside = nxp >= 0 && nxp < g.nx && nyp >= 0 && nyp < g.ny && nzp >= 0 && nzp < g.nz;
            if (inside || !ghost) {
                nxp = (nxp + g.nx) % g.nx;
                nyp = (nyp + g.ny) % g.ny;
                nzp = (nzp + g.nz) % g.nz;
                nb = rf[o][((int64_t)nzp * g.ny + nyp) * g.nx + nxp];
            } else {
                nb = rbnd[o];
            }
            const double wn = w_of<double>(i) * nb;
            sx += cx_of(i) * wn;
            sy += cy_of(i) * wn;
            sz += cz_of(i) * wn;
        }
        const double pre = -gab * rho[s];
        Ft[0] += pre * sx;
        Ft[1] += pre * sy;
        Ft[2] += pre * sz;
    }
    const double rt = rho[0] + rho[1];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c * g.nnode + k] = (j[0][c] + j[1][c] + 0.5 * Ft[c]) / rt;
}

template <int K>
__device__ __forceinline__ void block_reduce_store(double (&v)[K], double *out /* K values */) {
    // wavefront butterfly, fixed order
#pragma unroll
    for (int c = 0; c < K; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_down(v[c], off, 64);
    }
    __shared__ double part[NRED_THREADS / 64][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < K; ++c) part[wv][c] = v[c];
    __syncthreads();
    if (threadIdx.x < K) {
        double acc = 0.0;
        for (int w = 0; w < NRED_THREADS / 64; ++w) acc += part[w][threadIdx.x];
        out[threadIdx.x] = acc;
    }
}

// Per-workgroup partials of: mass A, mass B, momentum (3), indicator moments
// S0, S1 (3), S2 (6) about the box centre, and the count of bad nodes.
// Grid (blocks per box, boxes): box b0 + blockIdx.y, partials [box][block][NSTAT].
template <int P>
__global__ __launch_bounds__(NRED_THREADS) void k_stats(const typename Prec<P>::S *f, const __half *ref, BoxGeom g,
                                                        int b0, double *partial) {
    using S = typename Prec<P>::S;
    using R = typename Prec<P>::R;
    const int box = b0 + blockIdx.y;
    f += (int64_t)box * 2 * Q * g.nnode;
    if (Prec<P>::DEV) ref += (int64_t)box * 2 * g.nnode;
    double v[NSTAT];
#pragma unroll
    for (int c = 0; c < NSTAT; ++c) v[c] = 0.0;
    // Thread t takes nodes k = t, t + stride, ... (k = (z ny + y) nx + x), carrying (x, y, z) from
    // one to the next, so that the loop does no integer division; a box holds fewer than 2^31 nodes.
    const uint32_t nn = uint32_t(g.nnode), nx = uint32_t(g.nx), ny = uint32_t(g.ny);
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x = k % nx, y = (k / nx) % ny, z = k / nx / ny;
    const uint32_t sx = stride % nx, sy = (stride / nx) % ny, sz = stride / nx / ny;
    // FP64 and FP32 storage: raw buffer loads, one byte offset per node and a uniform one per
    // direction (the 16-bit formats take the decoding loads of node_moments)
    constexpr uint32_t EB = sizeof(S);
    const uint32_t comp_bytes = uint32_t(Q) * nn * EB, plane_bytes = nx * EB;
    const rsrc_t rs[2] = {make_rsrc(f, comp_bytes), make_rsrc(f + (int64_t)Q * g.nnode, comp_bytes)};
    // the node's contributions, in a fixed order (one node after the other)
    auto accumulate = [&](const double (&rho)[2], const double (&j)[2][3], uint32_t xx, uint32_t yy, uint32_t zz) {
        v[0] += rho[0];
        v[1] += rho[1];
        v[2] += j[0][0] + j[1][0];
        v[3] += j[0][1] + j[1][1];
        v[4] += j[0][2] + j[1][2];
        if (!(rho[0] > 0.0) || !(rho[1] > 0.0) || !isfinite(rho[0]) || !isfinite(rho[1])) v[15] += 1.0;
        if (rho[0] > rho[1]) {
            const double dx = double(xx) - g.xc[0], dy = double(yy) - g.xc[1], dz = double(zz) - g.xc[2];
            v[5] += 1.0;
            v[6] += dx;
            v[7] += dy;
            v[8] += dz;
            v[9] += dx * dx;
            v[10] += dx * dy;
            v[11] += dx * dz;
            v[12] += dy * dy;
            v[13] += dy * dz;
            v[14] += dz * dz;
        }
    };
    // the next node's coordinates: add (sx, sy, sz) with carries (sx < nx, sy < ny)
    auto advance = [&](uint32_t &xx, uint32_t &yy, uint32_t &zz) {
        xx += sx;
        const uint32_t carry_x = xx >= nx ? 1u : 0u;
        xx -= carry_x * nx;
        yy += sy + carry_x;
        const uint32_t carry_y = yy >= ny ? 1u : 0u;
        yy -= carry_y * ny;
        zz += sz + carry_y;
    };
    // density and momentum of a node from its 2 x 19 populations, summed in FP64
    auto moments = [&](const auto &w, double (&rho)[2], double (&j)[2][3]) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double wi = double(w[s][i]);
                r += wi;
                if (cx_of(i)) jx += double(cx_of(i)) * wi;
                if (cy_of(i)) jy += double(cy_of(i)) * wi;
                if (cz_of(i)) jz += double(cz_of(i)) * wi;
            }
            rho[s] = r;
            j[s][0] = jx;
            j[s][1] = jy;
            j[s][2] = jz;
        }
    };
    auto node_vo = [&](uint32_t xx, uint32_t yy, uint32_t zz) { return ((zz * ny + yy) * uint32_t(Q) * nx + xx) * EB; };
    if constexpr (Prec<P>::DEV) {
        for (; k < nn; k += stride) {
            double rho[2], j[2][3];
            node_moments<P>(f, ref, g, k, rho, j);
            accumulate(rho, j, x, y, z);
            advance(x, y, z);
        }
    } else if constexpr (sizeof(S) == 4) {
        // FP32 storage: the loads of node k + stride go out while node k is summed
        float wn[2][Q];
        auto load = [&](uint32_t vo) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) wn[s][i] = Prec<P>::bload(rs[s], vo, uint32_t(i) * plane_bytes, R(0));
        };
        if (k < nn) load(node_vo(x, y, z));
        for (; k < nn; k += stride) {
            float w[2][Q];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) w[s][i] = wn[s][i];
            uint32_t xn = x, yn = y, zn = z;
            advance(xn, yn, zn);
            if (k + stride < nn) load(node_vo(xn, yn, zn));
            double rho[2], j[2][3];
            moments(w, rho, j);
            accumulate(rho, j, x, y, z);
            x = xn;
            y = yn;
            z = zn;
        }
    } else {
        for (; k < nn; k += stride) {
            S w[2][Q];
            const uint32_t vo = node_vo(x, y, z);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) w[s][i] = Prec<P>::bload(rs[s], vo, uint32_t(i) * plane_bytes, R(0));
            double rho[2], j[2][3];
            moments(w, rho, j);
            accumulate(rho, j, x, y, z);
            advance(x, y, z);
        }
    }
    block_reduce_store<NSTAT>(v, partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * NSTAT);
}

// Partials of sum |u - A d|^2 and sum |A d|^2 (Sec. 4 Eq. 16).
__global__ __launch_bounds__(NRED_THREADS) void k_e0(const double *u, BoxGeom g, Mat3 A, double *partial) {
    double v[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < g.nnode; k += stride) {
        int x, y, z;
        node_xyz(g, k, x, y, z);
        const double dx = x - g.xc[0], dy = y - g.xc[1], dz = z - g.xc[2];
        const double vx = A.a[0] * dx + A.a[1] * dy + A.a[2] * dz;
        const double vy = A.a[3] * dx + A.a[4] * dy + A.a[5] * dz;
        const double vz = A.a[6] * dx + A.a[7] * dy + A.a[8] * dz;
        const double ex = u[k] - vx, ey = u[g.nnode + k] - vy, ez = u[2 * g.nnode + k] - vz;
        v[0] += ex * ex + ey * ey + ez * ez;
        v[1] += vx * vx + vy * vy + vz * vz;
    }
    block_reduce_store<2>(v, partial + (int64_t)blockIdx.x * 2);
}

// Fixed-order sum of nblk partials of K values each; workgroup b handles the
// partials of box b ([b][nblk][K] -> out[b][K]).
template <int K>
__global__ __launch_bounds__(NRED_THREADS) void k_final(const double *partial, int nblk, double *out) {
    partial += (int64_t)blockIdx.x * nblk * K;
    out += (int64_t)blockIdx.x * K;
    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NRED_THREADS)
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] += partial[(int64_t)b * K + c];
    block_reduce_store<K>(v, out);
}

}  // namespace sclbm
