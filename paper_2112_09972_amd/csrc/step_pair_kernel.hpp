// Fused stream-and-collide step for the 16-bit deviation formats with two
// nodes per lane (same method and, node by node, the same arithmetic as k_step:
// arXiv 2112.09972, Sec. 2 Eqs. 6-9, ghost boundary of Sec. 2 Eq. 8 and Sec. 3
// Eq. 14).
//
// Why: a 16-bit population access by one node per lane moves 128 bytes per
// wavefront instruction, half of what an FP32 access moves, and these formats
// are bound by their memory instructions (without the collision arithmetic the
// one-node kernel is only 8 % faster).  Here lane l owns the neighbouring nodes
// x0 + 2l and x0 + 2l + 1, so every population and reference-density access of
// a run is a 32-bit pair: a wavefront covers 128 nodes of a row and each of its
// loads and stores moves 256 bytes.
//
// Layout and tiling as in k_step with a 128 WX x TY tile (row-blocked
// populations, march along a z-chunk, 4-slot LDS density window, raw next-plane
// prefetch, streaming loads of rows read once, alternating march directions,
// grouped z-chunks in the tile order), with WX wavefronts per row.  The
// register window holds raw pairs, decoded node by node when the densities are
// summed and again when the plane collides.  Every post-collision value goes to
// LDS; after the second barrier each lane reads, per direction, the pair pushed
// into its two nodes as one aligned 32-bit LDS word and stores it as one 32-bit
// word.  Requires an even nx (pairs 4-byte aligned, the tile's width even).
#pragma once

#include "step_kernel.hpp"

namespace sclbm {

template <int P, int TY, int WX, bool GHOST>
__global__ __launch_bounds__(64 * WX * TY, 2) void k_step_pair(StepArgs a) {
    static_assert(Prec<P>::DEV, "two nodes per lane: the 16-bit deviation formats");
    using R = typename Prec<P>::R;  // float
    using W = typename Prec<P>::W;  // float
    using C = R;
    using L = typename Prec<P>::L;  // unsigned short
    constexpr int TXW = 128 * WX;   // nodes per tile row: WX wavefronts of 64 lanes x 2
    constexpr int LW = TXW + 2;
    constexpr uint32_t EB = 2;
    typedef uint32_t __attribute__((may_alias)) u32a;
    // densities of the planes zc - 1, zc, zc + 1 and the reciprocals of their
    // rounded reference densities (as k_step's deviation formats)
    constexpr int NSLOT = 3;
    __shared__ R lds[NSLOT][2][TY + 2][LW];
    __shared__ float rq[NSLOT][2][TY + 2][LW];
    // every direction's post-collision value by node: node n in column n for the
    // directions with c_x = 0, in column n + 1 for the others, whose columns 0 and
    // tw + 1 hold what streams in across the tile's left and right edges.  The
    // pair pushed into nodes (n0, n0 + 1), n0 even, then starts at an even column.
    __shared__ __attribute__((aligned(16))) unsigned short xq[2][Q][TY][LW];
    auto col0 = [](int i) { return cx_of(i) != 0 ? 1 : 0; };

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 * WX + lx;
    // tile order: as in k_step (contiguous runs per XCD, z-chunks grouped)
    const uint32_t nbx = gridDim.x, nby = gridDim.y;
    const uint32_t nb = nbx * nby * gridDim.z;
    const uint32_t lin = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
    const uint32_t q8 = nb / 8, r8 = nb % 8, xcd = lin % 8, k8 = lin / 8;
    const uint32_t tile = xcd < r8 ? xcd * (q8 + 1) + k8 : r8 * (q8 + 1) + (xcd - r8) * q8 + k8;
    const int bx = int(tile % nbx);
    uint32_t t2 = tile / nbx;
    const uint32_t zg = uint32_t(a.zgroup), ngr = uint32_t(a.nzc) / zg;
    const uint32_t ci = t2 % zg;
    t2 /= zg;
    const int by = int(t2 % nby);
    t2 /= nby;
    const int chunk = int((t2 % ngr) * zg + ci);
    const int bz = int(t2 / ngr) * a.nzc + chunk;
    const int x0 = bx * TXW, y0 = by * TY;
    const int box = bz / a.nzc;
    const int zs = (bz % a.nzc) * a.zchunk;
    const int ze = min(zs + a.zchunk, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tw = min(TXW, nx - x0), th = min(TY, ny - y0);  // both even / any
    const int n0 = 2 * lx;                                      // the lane's first node in the tile
    const int xa = x0 + n0;
    const int y = y0 + ly;
    const bool valid = (y < ny) && (n0 < tw);                   // both nodes (tw is even)
    const bool left_face = x0 == 0, right_face = x0 + tw == nx;
    const bool span = left_face && right_face;
    const uint32_t N = uint32_t(a.nnode);
    const uint32_t nxy = uint32_t(nx) * uint32_t(ny);
    const uint32_t qnx = uint32_t(Q) * uint32_t(nx);
    const uint32_t plane_bytes = uint32_t(nx) * EB;

    const uint32_t comp_bytes = uint32_t(Q) * N * EB;
    const unsigned short *src = (const unsigned short *)a.src + (int64_t)box * 2 * Q * N;
    unsigned short *dst = (unsigned short *)a.dst + (int64_t)box * 2 * Q * N;
    const rsrc_t rs[2] = {make_rsrc(src, comp_bytes), make_rsrc(src + (int64_t)Q * N, comp_bytes)};
    const rsrc_t rd[2] = {make_rsrc(dst, comp_bytes), make_rsrc(dst + (int64_t)Q * N, comp_bytes)};

    const int64_t n = *a.clk_in;
    if (lin == 0 && tid == 0) *a.clk_out = n + 1;

    const __half *ref_in = a.ref_src + (int64_t)box * 2 * N;
    __half *ref_out = a.ref_dst + (int64_t)box * 2 * N;
    const R rhob[2] = {R(a.rho_b[0]), R(a.rho_b[1])};
    R Am[9];
    if (GHOST) {
        const double *Arow = a.atab + ((int64_t)box * a.table_len + (n - a.tab_first[box])) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) Am[q] = R(Arow[q]);
    }
    const int nplanes = (ze - zs) + 2;

    // halves of a raw pair (low half: the first node)
    auto half_of = [](uint32_t p, int j) -> L { return L(j ? (p >> 16) : (p & 0xffffu)); };
    auto ref_of = [&](uint32_t p, int j) -> R { return R(__half2float(__builtin_bit_cast(__half, half_of(p, j)))); };
    // density of node j of a pair from the raw words of one component (the order of pair_density)
    auto pair_node_density = [&](const uint32_t (&f)[Q], uint32_t rp, int j) -> R {
        const R rr = ref_of(rp, j);
        W v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = Prec<P>::dec(half_of(f[i], j), w_of<R>(i) * rr);
        return pair_density<R>(v);
    };

    // the lane's pair in plane z: inside the box (ghost mode), byte offset, node index
    auto own_pair = [&](int z, uint32_t &vo, uint32_t &nd) -> bool {
        int zz = z;
        bool in = (z >= 0) && (z < nz);
        if (!GHOST) {
            zz = z < 0 ? z + nz : (z >= nz ? z - nz : z);
            in = true;
        }
        vo = ((uint32_t(zz) * uint32_t(ny) + uint32_t(y)) * qnx + uint32_t(xa)) * EB;
        nd = uint32_t(zz) * nxy + uint32_t(y) * uint32_t(nx) + uint32_t(xa);
        return in && valid;
    };
    uint32_t fnx[2][Q], rnx[2] = {0u, 0u};
    bool nx_in = false;
    // rows that no other workgroup reads (as in k_step): streaming loads
    const bool row_once = GHOST && span && ly > 0 && ly < th - 1;
    auto prefetch = [&](int z) {
        uint32_t vo, nd;
        nx_in = own_pair(z, vo, nd);
        if (nx_in) {
            const bool once = row_once && z > zs && z < ze - 1;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rnx[s] = *reinterpret_cast<const u32a *>(ref_in + s * N + nd);
                if (once) {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        fnx[s][i] = __builtin_amdgcn_raw_buffer_load_b32(rs[s], vo, uint32_t(i) * plane_bytes, kLoadNT);
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        fnx[s][i] = __builtin_amdgcn_raw_buffer_load_b32(rs[s], vo, uint32_t(i) * plane_bytes, 0);
                }
            }
        }
    };
    const int dir = (chunk & 1) ? -1 : 1;
    const int zfirst = dir > 0 ? zs - 1 : ze;
    prefetch(zfirst);

    uint32_t fprev[2][Q], fcur[2][Q], rprev[2] = {0u, 0u}, rcur[2] = {0u, 0u};
    for (int k = 0; k < nplanes; ++k) {
        const int z = zfirst + dir * k;
        const int slot = k % NSLOT;
        if constexpr (kDebugFill) {
            // debug build: this plane's density slot and the exchange buffer start as NaN
            __syncthreads();
            lds_fill(&lds[slot][0][0][0], 2 * (TY + 2) * LW, R(__builtin_nanf("")), tid, 64 * WX * TY);
            lds_fill(&rq[slot][0][0][0], 2 * (TY + 2) * LW, __builtin_nanf(""), tid, 64 * WX * TY);
            lds_fill(&xq[0][0][0][0], 2 * Q * TY * LW, nan_bits<unsigned short>(P), tid, 64 * WX * TY);
            __syncthreads();
        }
        // ---- 1. densities of plane z: the lane's pair and the ring around the tile ----
        const bool own_in = nx_in;
        if (own_in) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rcur[s] = rnx[s];
#pragma unroll
                for (int i = 0; i < Q; ++i) fcur[s][i] = fnx[s][i];
            }
        }
        if (valid) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const R d0 = own_in ? pair_node_density(fcur[0], rcur[0], j) : rhob[0];
                const R d1 = own_in ? pair_node_density(fcur[1], rcur[1], j) : rhob[1];
                lds[slot][0][ly + 1][1 + n0 + j] = d0;
                lds[slot][1][ly + 1][1 + n0 + j] = d1;
                rq[slot][0][ly + 1][1 + n0 + j] = ref_rcp(d0);
                rq[slot][1][ly + 1][1 + n0 + j] = ref_rcp(d1);
            }
        }
        // ring rows y0 - 1 and y0 + th as pairs (threads 0 .. TXW - 1), the two ring
        // columns node by node (threads TXW ...)
        static_assert(TXW + 2 * (TY + 2) <= 64 * WX * TY, "one ring pair or node per thread");
        if (tid < TXW) {
            const int p = tid % (TXW / 2), side = tid / (TXW / 2);
            const int rsy = side ? th + 1 : 0;
            if (2 * p < tw) {
                int gy = y0 - 1 + rsy, gz = z;
                bool in = gy >= 0 && gy < ny && gz >= 0 && gz < nz;
                if (!GHOST) {
                    gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
                    gz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);
                    in = true;
                }
                R rr[2][2] = {{rhob[0], rhob[1]}, {rhob[0], rhob[1]}};  // [node][component]
                if (in) {
                    const uint32_t gx = uint32_t(x0 + 2 * p);
                    const uint32_t vo = ((uint32_t(gz) * uint32_t(ny) + uint32_t(gy)) * qnx + gx) * EB;
                    const uint32_t nd = uint32_t(gz) * nxy + uint32_t(gy) * uint32_t(nx) + gx;
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const uint32_t rp = *reinterpret_cast<const u32a *>(ref_in + s * N + nd);
                        uint32_t f[Q];
#pragma unroll
                        for (int i = 0; i < Q; ++i)
                            f[i] = __builtin_amdgcn_raw_buffer_load_b32(rs[s], vo, uint32_t(i) * plane_bytes, 0);
                        rr[0][s] = pair_node_density(f, rp, 0);
                        rr[1][s] = pair_node_density(f, rp, 1);
                    }
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    lds[slot][0][rsy][1 + 2 * p + j] = rr[j][0];
                    lds[slot][1][rsy][1 + 2 * p + j] = rr[j][1];
                    rq[slot][0][rsy][1 + 2 * p + j] = ref_rcp(rr[j][0]);
                    rq[slot][1][rsy][1 + 2 * p + j] = ref_rcp(rr[j][1]);
                }
            }
        } else if (tid < TXW + 2 * (th + 2)) {
            const int r = tid - TXW, side = r / (th + 2), rsy = r % (th + 2);
            const int rsx = side ? tw + 1 : 0;
            int gx = x0 - 1 + rsx, gy = y0 - 1 + rsy, gz = z;
            bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            if (!GHOST) {
                gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
                gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
                gz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);
                in = true;
            }
            R rr[2] = {rhob[0], rhob[1]};
            if (in) {
                const uint32_t vo = ((uint32_t(gz) * uint32_t(ny) + uint32_t(gy)) * qnx + uint32_t(gx)) * EB;
                const uint32_t nd = uint32_t(gz) * nxy + uint32_t(gy) * uint32_t(nx) + uint32_t(gx);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const R ref = R(ref_load(ref_in + s * N + nd));
                    W f[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        f[i] = Prec<P>::bload(rs[s], vo, uint32_t(i) * plane_bytes, w_of<R>(i) * ref);
                    rr[s] = pair_density<R>(f);
                }
            }
            lds[slot][0][rsy][rsx] = rr[0];
            lds[slot][1][rsy][rsx] = rr[1];
            rq[slot][0][rsy][rsx] = ref_rcp(rr[0]);
            rq[slot][1][rsy][rsx] = ref_rcp(rr[1]);
        }
        __syncthreads();
        // ---- 2. the next plane's loads land during the collision ----
        if (k + 1 < nplanes) prefetch(z + dir);
        if (k >= 2) {
        // ---- 3. collide plane zc = z - dir, node by node; every value goes to LDS ----
        const int zc = z - dir;
        auto sl = [&](int d) { return (k - 1 + dir * d) % NSLOT; };  // k >= 2: never negative
        const uint32_t nda = uint32_t(zc) * nxy + uint32_t(y) * uint32_t(nx) + uint32_t(xa);
        const uint32_t vo = ((uint32_t(zc) * uint32_t(ny) + uint32_t(y)) * qnx + uint32_t(xa)) * EB;
        const bool ylo = y == 0, yhi = y == ny - 1;
        const bool zlo = zc == 0, zhi = zc == nz - 1;
        if (valid) {
            R rho_keep[2][2];  // [node][component], for the reference densities
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int nn = n0 + j;  // node within the tile
                const R rref[2] = {ref_of(rprev[0], j), ref_of(rprev[1], j)};
                R rho[2], jm[2][3];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    W f[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) f[i] = Prec<P>::dec(half_of(fprev[s][i], j), w_of<R>(i) * rref[s]);
                    R d[10];
#pragma unroll
                    for (int p = 1; p <= 9; ++p) d[p] = R(f[2 * p - 1]) - R(f[2 * p]);
                    rho[s] = pair_density<R>(f);
                    jm[s][0] = d[1] + d[4] + d[5] + d[6] + d[7];
                    jm[s][1] = d[2] + d[4] - d[5] + d[8] + d[9];
                    jm[s][2] = d[3] + d[6] - d[7] + d[8] - d[9];
                }
                R sig[2][3];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int o = 1 - s;
                    R e[10];
#pragma unroll
                    for (int p = 1; p <= 9; ++p) {
                        const int i = 2 * p - 1;
                        const R hi = lds[sl(cz_of(i))][o][ly + 1 + cy_of(i)][1 + nn + cx_of(i)];
                        const R lo = lds[sl(-cz_of(i))][o][ly + 1 - cy_of(i)][1 + nn - cx_of(i)];
                        e[p] = hi - lo;
                    }
                    const R w1 = R(1) / R(18), w2 = R(1) / R(36);
                    sig[s][0] = w1 * e[1] + w2 * (e[4] + e[5] + e[6] + e[7]);
                    sig[s][1] = w1 * e[2] + w2 * (e[4] - e[5] + e[8] + e[9]);
                    sig[s][2] = w1 * e[3] + w2 * (e[6] - e[7] + e[8] - e[9]);
                }
                const R om0 = R(a.omega[0]), om1 = R(a.omega[1]);
                const R inv_den = R(1) / (rho[0] * om0 + rho[1] * om1);
                const R up[3] = {(jm[0][0] * om0 + jm[1][0] * om1) * inv_den,
                                 (jm[0][1] * om0 + jm[1][1] * om1) * inv_den,
                                 (jm[0][2] * om0 + jm[1][2] * om1) * inv_den};
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    rho_keep[j][s] = rho[s];
                    const C om = C(s ? om1 : om0);
                    const R gt = R(a.g) * R(a.tau[s]);
                    const C ux = C(up[0] - gt * sig[s][0]);
                    const C uy = C(up[1] - gt * sig[s][1]);
                    const C uz = C(up[2] - gt * sig[s][2]);
                    const C usq = ux * ux + uy * uy + uz * uz;
                    const C r = C(rho[s]);
                    const C aa = r - C(1.5) * r * usq;
                    const C r3 = C(3) * r, r45 = C(4.5) * r;
                    // FP32 arithmetic: the rest population closes the mass balance (as in k_step)
                    C psum = C(0);
                    auto push = [&](int i, C geq) {
                        // decoded again here rather than kept from the moments (registers);
                        // the empty asm keeps the compiler from reusing the first decode
                        uint32_t raw = fprev[s][i];
                        asm volatile("" : "+v"(raw));
                        const C fi = C(Prec<P>::dec(half_of(raw, j), w_of<R>(i) * rref[s]));
                        C pst = fi + om * (geq - fi);
                        if (i == 0) pst = C(rho[s]) - psum;
                        else psum += pst;
                        const C scale = inv_w_of<C>(i) * C(rq[sl(cz_of(i))][s][ly + 1 + cy_of(i)][1 + nn + cx_of(i)]);
                        const unsigned short bits = (unsigned short)Prec<P>::enc_s(pst, scale);
                        xq[s][i][ly][col0(i) + nn] = bits;
                        if (cx_of(i) != 0 && !GHOST && span) {
                            if (cx_of(i) > 0 && nn == tw - 1) xq[s][i][ly][0] = bits;
                            if (cx_of(i) < 0 && nn == 0) xq[s][i][ly][tw + 1] = bits;
                        }
                    };
                    equilibrium_pairs<C>(ux, uy, uz, r, aa, r3, r45, push);
                }
            }
            // reference densities of the pair (as ref_store rounds them)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const uint32_t lo = __builtin_bit_cast(unsigned short, __float2half_rn(float(rho_keep[0][s])));
                const uint32_t hi = __builtin_bit_cast(unsigned short, __float2half_rn(float(rho_keep[1][s])));
                *reinterpret_cast<u32a *>(ref_out + s * N + nda) = lo | (hi << 16);
            }
        }
        if (GHOST && y < ny) {
            // (a) ghosts beside this row at x = -1 and x = nx, into the edge columns
            // (lanes 0-9: left side, 16-25: right side, as in k_step)
            const int side = lx < 16 ? 0 : 1;
            const int q = lx - 16 * side;
            if (q < 10 && (side ? right_face : left_face)) {
                const int sgn = side ? -1 : 1;
                const int m = q >> 1, s = q & 1;
                const int cyv = m == 1 ? 1 : (m == 2 ? -1 : 0);
                const int czv = m == 3 ? 1 : (m == 4 ? -1 : 0);
                const int idx = sgn > 0 ? (m == 0 ? 1 : m == 1 ? 7 : m == 2 ? 9 : m == 3 ? 11 : 13)
                                        : (m == 0 ? 2 : m == 1 ? 10 : m == 2 ? 8 : m == 3 ? 14 : 12);
                const int fx = side ? nx - 1 : 0;
                const R dxg = R(fx - sgn) - R(a.xc[0]), dyg = R(y) - R(a.xc[1]), dzg = R(zc) - R(a.xc[2]);
                const R gx = Am[0] * dxg + Am[1] * dyg + Am[2] * dzg;
                const R gy = Am[3] * dxg + Am[4] * dyg + Am[5] * dzg;
                const R gz = Am[6] * dxg + Am[7] * dyg + Am[8] * dzg;
                const R cu = R(sgn) * gx + R(cyv) * gy + R(czv) * gz;
                const R usq = gx * gx + gy * gy + gz * gz;
                const R wgt = m == 0 ? R(1) / R(18) : R(1) / R(36);
                const R geq = wgt * (s ? rhob[1] : rhob[0]) * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
                const R gscale = (m == 0 ? R(18) : R(36)) * R(rq[sl(czv)][s][ly + 1 + cyv][fx - x0 + 1]);
                xq[s][idx][ly][side ? tw + 1 : 0] = (unsigned short)Prec<P>::enc_s(geq, gscale);
            }
            // (b) y and z faces: the directions whose source lies outside the box in y
            // or z, for both nodes of the pair (the same directions), one 32-bit store
            if (valid && (ylo || yhi || zlo || zhi)) {
                const R dy0 = R(y) - R(a.xc[1]), dz0 = R(zc) - R(a.xc[2]);
#pragma nounroll
                for (int i = 1; i < Q; ++i) {
                    const int cx = c_rt(0, i), cy = c_rt(1, i), cz = c_rt(2, i);
                    const bool from_yz = (cy > 0 && ylo) || (cy < 0 && yhi) || (cz > 0 && zlo) || (cz < 0 && zhi);
                    if (!from_yz) continue;
                    const R wgt = i < 7 ? R(1) / R(18) : R(1) / R(36);
                    uint32_t word[2] = {0u, 0u};
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const R dxg = (R(xa + j) - R(a.xc[0])) - R(cx), dyg = dy0 - R(cy), dzg = dz0 - R(cz);
                        const R gx = Am[0] * dxg + Am[1] * dyg + Am[2] * dzg;
                        const R gy = Am[3] * dxg + Am[4] * dyg + Am[5] * dzg;
                        const R gz = Am[6] * dxg + Am[7] * dyg + Am[8] * dzg;
                        const R cu = R(cx) * gx + R(cy) * gy + R(cz) * gz;
                        const R usq = gx * gx + gy * gy + gz * gz;
                        const R br = R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq;
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const R oscale = (i < 7 ? R(18) : R(36)) * R(rq[sl(0)][s][ly + 1][1 + n0 + j]);
                            word[s] |= uint32_t(Prec<P>::enc_s(wgt * rhob[s] * br, oscale)) << (16 * j);
                        }
                    }
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        __builtin_amdgcn_raw_buffer_store_b32(word[s], rd[s], vo + uint32_t(i) * plane_bytes, 0, kStoreNT);
                }
            }
        }
        __syncthreads();
        // ---- 4. the stores: per direction, the pair pushed into the lane's two
        // nodes as one aligned 32-bit word (whole cache lines per wavefront);
        // halves whose source lies in another tile are written by that tile.
        if (valid) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
                int yd = y + cy, zd = zc + cz;
                bool out = false;
                if (GHOST) {
                    out = yd < 0 || yd >= ny || zd < 0 || zd >= nz;
                } else {
                    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
                    zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
                }
                if (out) continue;  // the destination row is outside the box
                const uint32_t row = (uint32_t(zd) * uint32_t(ny) + uint32_t(yd)) * qnx + uint32_t(i) * uint32_t(nx);
                bool ok0 = true, ok1 = true;
                if (cx > 0 && n0 == 0) ok0 = GHOST ? left_face : span;
                if (cx < 0 && n0 + 1 == tw - 1) ok1 = GHOST ? right_face : span;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const uint32_t w = *reinterpret_cast<const u32a *>(&xq[s][i][ly][col0(i) + n0 - cx]);
                    if (ok0 && ok1) {
                        __builtin_amdgcn_raw_buffer_store_b32(w, rd[s], (row + uint32_t(xa)) * EB, 0, kStoreNT);
                    } else {
                        if (ok0) Prec<P>::bstore_bits(rd[s], (row + uint32_t(xa)) * EB, 0, w & 0xffffu);
                        if (ok1) Prec<P>::bstore_bits(rd[s], (row + uint32_t(xa) + 1) * EB, 0, w >> 16);
                    }
                }
                if (cx != 0 && !span) {
                    // the value that leaves the tile: c_x = +1 from its last node, -1 from its first
                    const bool edge = cx > 0 ? n0 + 1 == tw - 1 : n0 == 0;
                    int xd = cx > 0 ? x0 + tw : x0 - 1;
                    bool go = edge;
                    if (GHOST) go = go && (cx > 0 ? !right_face : !left_face);
                    else xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
                    if (go) {
#pragma unroll
                        for (int s = 0; s < 2; ++s)
                            Prec<P>::bstore_bits(rd[s], (row + uint32_t(xd)) * EB, 0,
                                                 xq[s][i][ly][cx > 0 ? 1 + n0 + 1 : 1 + n0]);
                    }
                }
            }
        }
        }  // k >= 2
        // ---- 5. roll the window ----
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rprev[s] = rcur[s];
#pragma unroll
            for (int i = 0; i < Q; ++i) fprev[s][i] = fcur[s][i];
        }
    }
}

}  // namespace sclbm
