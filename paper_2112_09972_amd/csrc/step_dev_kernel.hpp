// Fused stream-and-collide step for the 16-bit deviation formats (the method of
// k_step: arXiv 2112.09972, Sec. 2 Eqs. 6-9, ghost boundary of Sec. 2 Eq. 8 and
// Sec. 3 Eq. 14), for gfx950.
//
// Storage.  A population is held as d_i = f_i / (w_i m) - 1 in FP16 or BF16, m the
// node's density one step earlier rounded to FP16 (its reference density, stored
// per node and component).  Both components of one (node, direction) share a
// 32-bit word, A in the low half and B in the high half, in the row-blocked order
// of k_step: [box][z][y][direction][x] words; the reference densities are one
// word per node, [box][node].  With one node per lane every population access is
// then a 32-bit access (256 bytes per wavefront instruction, as in FP32 storage),
// 19 loads and 19 stores per node, and both components of a push go to the same
// destination word.
//
// Arithmetic.  FP32, on the deviations themselves (the dev_* functions below):
// one mixed-precision multiply-add per population for the density, one per
// nonzero velocity component for the momentum, one for the post-collision value
// and one for its encoding.  w_i m is never formed: the weights enter the density
// only through its small relative change and the momentum as the exact integers
// 72 w_i, so their FP32 rounding biases neither mass nor momentum.  The
// functions run with contraction off, so that every tile shape rounds alike.
//
// Tiling, march along z, density ring, x exchange through LDS, tile order and
// stores are those of k_step, with a 3-slot density window (planes zc - 1, zc,
// zc + 1) and, beside every density, the node's (m, 1 / m) per component that a
// value pushed into the node is encoded against.
#pragma once

#include "step_kernel.hpp"

namespace sclbm {

#pragma clang fp contract(off)

// stored 16 bits -> d
template <int P>
__device__ __forceinline__ float dev_of(unsigned short h) {
    if constexpr (P == SCLBM_F16DEV) return __half2float(__builtin_bit_cast(__half, h));
    else return __uint_as_float(uint32_t(h) << 16);
}
// half s of a word (component A: s = 0, low half)
__device__ __forceinline__ unsigned short half_of(uint32_t w, int s) {
    return (unsigned short)(s ? (w >> 16) : (w & 0xffffu));
}

// Density of Sec. 2 Eq. 6: rho = m (1 + sum_i w_i d_i).  The sum is the node's
// relative change since its reference density (a few 1e-4), so the rounding of the
// FP32 weights moves rho by less than 1e-11 of itself.
template <typename DV>
__device__ __forceinline__ float dev_density(DV &&dv, float m) {
    constexpr float W0 = 1.0f / 3.0f, W1 = 1.0f / 18.0f, W2 = 1.0f / 36.0f;
    float sa = __builtin_fmaf(dv(1), W1, 0.0f);
#pragma unroll
    for (int i = 2; i < 7; ++i) sa = __builtin_fmaf(dv(i), W1, sa);
    float sd = __builtin_fmaf(dv(7), W2, 0.0f);
#pragma unroll
    for (int i = 8; i < Q; ++i) sd = __builtin_fmaf(dv(i), W2, sd);
    return __builtin_fmaf(m, __builtin_fmaf(dv(0), W0, sa + sd), m);
}

// First moment of Sec. 2 Eq. 6 up to the factor m / 72: J = sum_i c_i (72 w_i) d_i
// with 72 w_i = 4 on the axes and 2 on the diagonals (sum_i c_i w_i = 0 removes m).
template <typename DV>
__device__ __forceinline__ void dev_momentum(DV &&dv, float (&J)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int c = a == 0 ? cx_of(i) : (a == 1 ? cy_of(i) : cz_of(i));
            if (c != 0) acc = __builtin_fmaf(dv(i), float(c * (i < 7 ? 4 : 2)), acc);
        }
        J[a] = acc;
    }
}

// Pair force of Sec. 2 Eq. 7 as the stencil sum sig_s = sum_i w_i rho_s'(x + c_i) c_i
// (F_s = -G rho_s sig_s) from pair differences of the neighbour densities;
// rho(o, cx, cy, cz) reads component o at x + c.
template <typename Rho>
__device__ __forceinline__ void dev_stencil(Rho &&rho, float (&sig)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int o = 1 - s;
        float e[10];
#pragma unroll
        for (int p = 1; p <= 9; ++p) {
            const int i = 2 * p - 1;
            e[p] = rho(o, cx_of(i), cy_of(i), cz_of(i)) - rho(o, -cx_of(i), -cy_of(i), -cz_of(i));
        }
        constexpr float w1 = 1.0f / 18.0f, w2 = 1.0f / 36.0f;
        sig[s][0] = __builtin_fmaf(w1, e[1], w2 * (e[4] + e[5] + e[6] + e[7]));
        sig[s][1] = __builtin_fmaf(w1, e[2], w2 * (e[4] - e[5] + e[8] + e[9]));
        sig[s][2] = __builtin_fmaf(w1, e[3], w2 * (e[6] - e[7] + e[8] - e[9]));
    }
}

// Shifted velocities u' - G tau_s sig_s (Sec. 2 Eq. 9) of both components, u' the
// common velocity sum_s omega_s j_s / sum_s omega_s rho_s with j_s = m_s J_s / 72.
template <typename DV>
__device__ __forceinline__ void dev_shifted(DV &&dv, const float (&m)[2], const float (&rho)[2],
                                            const float (&sig)[2][3], float om0, float om1, float gt0, float gt1,
                                            float (&u)[2][3]) {
    float J[2][3];
    dev_momentum([&](int i) { return dv(0, i); }, J[0]);
    dev_momentum([&](int i) { return dv(1, i); }, J[1]);
    const float k0 = om0 * m[0], k1 = om1 * m[1];
    const float inv = 1.0f / (72.0f * __builtin_fmaf(rho[0], om0, rho[1] * om1));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float up = __builtin_fmaf(k0, J[0][c], k1 * J[1][c]) * inv;
        u[0][c] = __builtin_fmaf(-gt0, sig[0][c], up);
        u[1][c] = __builtin_fmaf(-gt1, sig[1][c], up);
    }
}

// Post-collision values per weight, t_i = f*_i / w_i (Sec. 2 Eq. 9).  With
// f_i / w_i = m (1 + d_i), t_i = a d_i + (a + omega G_i), a = (1 - omega) m and G_i
// the bracket rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2) of Sec. 2 Eq. 8.  DevColl holds
// one component's constants at one node; dev_pair gives the pair (2p - 1, 2p),
// dev_rest the rest population.
struct DevColl {
    float a, A0, R45, R3, ux, uy, uz;
};
__device__ __forceinline__ DevColl dev_coll(float m, float rho, const float (&u)[3], float om) {
    const float usq = __builtin_fmaf(u[0], u[0], __builtin_fmaf(u[1], u[1], u[2] * u[2]));
    const float orho = om * rho;
    DevColl c;
    c.a = __builtin_fmaf(-om, m, m);
    c.A0 = __builtin_fmaf(orho, __builtin_fmaf(-1.5f, usq, 1.0f), c.a);
    c.R45 = 4.5f * orho;
    c.R3 = 3.0f * orho;
    c.ux = u[0];
    c.uy = u[1];
    c.uz = u[2];
    return c;
}
__device__ __forceinline__ void dev_pair(const DevColl &c, int p, float dplus, float dminus, float &tplus,
                                         float &tminus) {
    const int i = 2 * p - 1;
    float cu = 0.0f;
    if (cx_of(i)) cu += float(cx_of(i)) * c.ux;
    if (cy_of(i)) cu += float(cy_of(i)) * c.uy;
    if (cz_of(i)) cu += float(cz_of(i)) * c.uz;
    const float sp = __builtin_fmaf(c.R45 * cu, cu, c.A0);
    const float ap = c.R3 * cu;
    tplus = __builtin_fmaf(dplus, c.a, sp + ap);
    tminus = __builtin_fmaf(dminus, c.a, sp - ap);
}
__device__ __forceinline__ float dev_rest(const DevColl &c, float d0) { return __builtin_fmaf(d0, c.a, c.A0); }

// Stored bits of a value t = f / w pushed into a node of reference density m with
// r = 1 / m as kept in LDS: d = (t - m) r.  Taking t - m first leaves the
// reciprocal's rounding on d alone; t r - 1 would scale every population pushed
// into the node by m r (1 +- 1e-7, fixed by m), a systematic gain or loss of mass.
template <int P>
__device__ __forceinline__ unsigned short dev_enc(float t, float m, float r) {
    const float d = __builtin_fmaf(t - m, r, 0.0f);
    if constexpr (P == SCLBM_F16DEV) return __builtin_bit_cast(unsigned short, __float2half_rn(d));
    else return __builtin_bit_cast(unsigned short, __float2bfloat16(d));
}
// (m, 1 / m) of a node from its density
__device__ __forceinline__ float2 dev_ref(float rho) {
    const float m = ref_round(rho);
    return make_float2(m, __builtin_amdgcn_rcpf(m));
}

// Bracket 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2 of a ghost population (Sec. 2 Eq. 8),
// its velocity A (x_g - x_c) from the displacement (dx, dy, dz); c = (cx, cy, cz).
__device__ __forceinline__ float ghost_bracket(const float *A, float dx, float dy, float dz, int cx, int cy,
                                               int cz) {
    const float gx = __builtin_fmaf(A[0], dx, __builtin_fmaf(A[1], dy, A[2] * dz));
    const float gy = __builtin_fmaf(A[3], dx, __builtin_fmaf(A[4], dy, A[5] * dz));
    const float gz = __builtin_fmaf(A[6], dx, __builtin_fmaf(A[7], dy, A[8] * dz));
    const float cu = float(cx) * gx + float(cy) * gy + float(cz) * gz;
    const float usq = __builtin_fmaf(gx, gx, __builtin_fmaf(gy, gy, gz * gz));
    return __builtin_fmaf(__builtin_fmaf(4.5f, cu, 3.0f), cu, __builtin_fmaf(-1.5f, usq, 1.0f));
}

#pragma clang fp contract(fast)

template <int P, int TY, int WX, bool GHOST, int WAVES>
__global__ __launch_bounds__(64 * WX * TY, WAVES) void k_step_dev(StepArgs a) {
    static_assert(Prec<P>::DEV, "the 16-bit deviation formats");
    constexpr int TXW = 64 * WX;  // tile width: WX wavefronts per row
    constexpr int LW = TXW + 2;   // with the ring
    constexpr uint32_t EB = 4;    // one word (both components) per node and direction
    constexpr int NSLOT = 3;
    __shared__ float lds[NSLOT][2][TY + 2][LW];
    __shared__ float4 rmq[NSLOT][TY + 2][LW];  // (m_A, 1 / m_A, m_B, 1 / m_B)
    // x exchange: the words with c_x != 0 by slot, row and column lx + 1; columns 0
    // and tw + 1 hold what streams in across the tile's left and right edges
    __shared__ uint32_t xq[NXD][TY][LW];

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * TXW + lx;
    const int lane = lx & 63;
    constexpr int NWAVES = TY * WX;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront in the workgroup
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
    const int x = x0 + lx, y = y0 + ly;
    const bool valid = (x < a.nx) && (y < a.ny);
    const int tw = min(TXW, a.nx - x0), th = min(TY, a.ny - y0);
    const bool left_face = x0 == 0, right_face = x0 + tw == a.nx;
    const bool span = left_face && right_face;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t N = uint32_t(a.nnode);
    const uint32_t nxy = uint32_t(nx) * uint32_t(ny);
    const uint32_t qnx = uint32_t(Q) * uint32_t(nx);
    const uint32_t plane_bytes = uint32_t(nx) * EB;

    // one descriptor per buffer; 19 N words per box (< 4 GiB, checked on the host)
    const rsrc_t rs = make_rsrc((const uint32_t *)a.src + (int64_t)box * Q * N, uint32_t(Q) * N * EB);
    const rsrc_t rd = make_rsrc((uint32_t *)a.dst + (int64_t)box * Q * N, uint32_t(Q) * N * EB);
    const rsrc_t rf_in = make_rsrc(a.ref_src + (int64_t)box * 2 * N, 4u * N);
    const rsrc_t rf_out = make_rsrc(a.ref_dst + (int64_t)box * 2 * N, 4u * N);

    const int64_t n = *a.clk_in;
    if (lin == 0 && tid == 0) *a.clk_out = n + 1;

    // Values that are the same in every lane are taken into scalar registers
    // (readfirstlane): held in vector registers through the march they pushed the
    // kernel past its 128 registers into scratch, and the compiler then waited for
    // all outstanding memory operations several times per plane.
    auto uni = [](float v) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v))); };
    const float rhob[2] = {uni(float(a.rho_b[0])), uni(float(a.rho_b[1]))};
    // velocity gradient of step n (row-major) and box centre, for the ghost nodes
    float gsc[12];
    if (GHOST) {
        const double *Arow = a.atab + ((int64_t)box * a.table_len + (n - a.tab_first[box])) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) gsc[q] = uni(float(Arow[q]));
#pragma unroll
        for (int q = 0; q < 3; ++q) gsc[9 + q] = uni(float(a.xc[q]));
    }
    const float om0 = uni(float(a.omega[0])), om1 = uni(float(a.omega[1]));
    const float gt0 = uni(float(a.g) * float(a.tau[0])), gt1 = uni(float(a.g) * float(a.tau[1]));

    static_assert(2 * (TXW + 2) + 2 * TY <= TXW * TY, "one ring node per thread");
    const int ringN = 2 * (tw + 2) + 2 * th;
    const int nplanes = (ze - zs) + 2;

    auto mval = [](uint32_t r, int s) -> float { return __half2float(__builtin_bit_cast(__half, half_of(r, s))); };
    // density of component s of a node from its words and reference-density word
    auto node_density = [&](const uint32_t (&f)[Q], uint32_t r, int s) -> float {
        return dev_density([&](int i) { return dev_of<P>(half_of(f[i], s)); }, mval(r, s));
    };

    auto own_node = [&](int z, uint32_t &vo, uint32_t &nd) -> bool {
        int zz = z;
        bool in = (z >= 0) && (z < nz);
        if (!GHOST) {
            zz = z < 0 ? z + nz : (z >= nz ? z - nz : z);
            in = true;
        }
        vo = ((uint32_t(zz) * uint32_t(ny) + uint32_t(y)) * qnx + uint32_t(x)) * EB;
        nd = uint32_t(zz) * nxy + uint32_t(y) * uint32_t(nx) + uint32_t(x);
        return in && valid;
    };
    // words of the next plane and its reference-density word
    uint32_t fnx[Q], rnx = 0u;
    bool nx_in = false;
    const bool row_once = GHOST && span && ly > 0 && ly < th - 1;
    auto prefetch = [&](int z) {
        uint32_t vo, nd;
        nx_in = own_node(z, vo, nd);
        if (nx_in) {
            rnx = __builtin_amdgcn_raw_buffer_load_b32(rf_in, 4u * nd, 0, 0);
            if (row_once && z > zs && z < ze - 1) {
#pragma unroll
                for (int i = 0; i < Q; ++i) fnx[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, uint32_t(i) * plane_bytes, kLoadNT);
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) fnx[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, uint32_t(i) * plane_bytes, 0);
            }
        }
    };
    const int dir = (chunk & 1) ? -1 : 1;
    const int zfirst = dir > 0 ? zs - 1 : ze;
    prefetch(zfirst);

    uint32_t fprev[Q], fcur[Q], rprev = 0u, rcur = 0u;
    for (int k = 0; k < nplanes; ++k) {
        const int z = zfirst + dir * k;
        const int slot = k % NSLOT;
        if constexpr (kDebugFill) {
            // debug build: this plane's density slot and the exchange buffer start as NaN
            __syncthreads();
            lds_fill(&lds[slot][0][0][0], 2 * (TY + 2) * LW, __builtin_nanf(""), tid, 64 * WX * TY);
            const float qn = __builtin_nanf("");
            lds_fill(&rmq[slot][0][0], (TY + 2) * LW, make_float4(qn, qn, qn, qn), tid, 64 * WX * TY);
            const uint32_t hn = uint32_t(nan_bits<unsigned short>(P));
            lds_fill(&xq[0][0][0], NXD * TY * LW, hn | (hn << 16), tid, 64 * WX * TY);
            __syncthreads();
        }
        // ---- 1. densities of plane z: own node and one ring node per thread ----
        const bool own_in = nx_in;
        if (own_in) {
            rcur = rnx;
#pragma unroll
            for (int i = 0; i < Q; ++i) fcur[i] = fnx[i];
        }
        if (valid) {
            const float d0 = own_in ? node_density(fcur, rcur, 0) : rhob[0];
            const float d1 = own_in ? node_density(fcur, rcur, 1) : rhob[1];
            lds[slot][0][ly + 1][lx + 1] = d0;
            lds[slot][1][ly + 1][lx + 1] = d1;
            const float2 q0 = dev_ref(d0), q1 = dev_ref(d1);
            rmq[slot][ly + 1][lx + 1] = make_float4(q0.x, q0.y, q1.x, q1.y);
        }
        if (tid < ringN) {
            // threads 0 .. 2 tw - 1: the ring rows y0 - 1 and y0 + th from x0 (whole
            // cache lines), then the ring columns x0 - 1 and x0 + tw with the corners
            int rsx, rsy;
            if (tid < 2 * tw) {
                rsy = tid < tw ? 0 : th + 1;
                rsx = (tid < tw ? tid : tid - tw) + 1;
            } else {
                const int q = tid - 2 * tw;
                rsx = q < th + 2 ? 0 : tw + 1;
                rsy = q < th + 2 ? q : q - (th + 2);
            }
            // (an empty asm keeps the ring node's plane-invariant offsets from being
            // hoisted out of the march: held there, one spilled to scratch in the BF16
            // build, and its reload waited for every outstanding store)
            asm volatile("" : "+v"(rsx), "+v"(rsy));
            int gx = x0 - 1 + rsx, gy = y0 - 1 + rsy, gz = z;
            bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            if (!GHOST) {
                gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
                gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
                gz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);
                in = true;
            }
            float rr[2] = {rhob[0], rhob[1]};
            if (in) {
                const uint32_t vo = ((uint32_t(gz) * uint32_t(ny) + uint32_t(gy)) * qnx + uint32_t(gx)) * EB;
                const uint32_t nd = uint32_t(gz) * nxy + uint32_t(gy) * uint32_t(nx) + uint32_t(gx);
                const uint32_t rw = __builtin_amdgcn_raw_buffer_load_b32(rf_in, 4u * nd, 0, 0);
                uint32_t f[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) f[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, uint32_t(i) * plane_bytes, 0);
                rr[0] = node_density(f, rw, 0);
                rr[1] = node_density(f, rw, 1);
            }
            lds[slot][0][rsy][rsx] = rr[0];
            lds[slot][1][rsy][rsx] = rr[1];
            const float2 q0 = dev_ref(rr[0]), q1 = dev_ref(rr[1]);
            rmq[slot][rsy][rsx] = make_float4(q0.x, q0.y, q1.x, q1.y);
        }
        __syncthreads();
        // ---- 2. the next plane's loads go out now and land during the collision ----
        if (k + 1 < nplanes) prefetch(z + dir);
        if (k >= 2) {
        // ---- 3. collide plane zc = z - dir: c_x = 0 words are pushed now, the others
        // go through LDS ----
        const int zc = z - dir;
        auto sl = [&](int d) { return (k - 1 + dir * d) % NSLOT; };  // k >= 2: never negative
        const uint32_t node = uint32_t(zc) * nxy + uint32_t(y) * uint32_t(nx) + uint32_t(x);
        const uint32_t elem = (uint32_t(zc) * uint32_t(ny) + uint32_t(y)) * qnx + uint32_t(x);
        const uint32_t vo = elem * EB;
        const bool ylo = y == 0, yhi = y == ny - 1;
        const bool zlo = zc == 0, zhi = zc == nz - 1;
        if (valid) {
            const float m[2] = {mval(rprev, 0), mval(rprev, 1)};
            const float rho[2] = {lds[sl(0)][0][ly + 1][lx + 1], lds[sl(0)][1][ly + 1][lx + 1]};
            float sig[2][3], u[2][3];
            dev_stencil([&](int o, int cx, int cy, int cz) -> float { return lds[sl(cz)][o][ly + 1 + cy][lx + 1 + cx]; },
                        sig);
            auto dv = [&](int s, int i) { return dev_of<P>(half_of(fprev[i], s)); };
            dev_shifted(dv, m, rho, sig, om0, om1, gt0, gt1, u);
            // direction i: the two components' values, encoded against the destination's
            // reference densities, as one word
            auto push = [&](int i, float t0, float t1) {
                const float4 q = rmq[sl(cz_of(i))][ly + 1 + cy_of(i)][lx + 1 + cx_of(i)];
                const uint32_t w = uint32_t(dev_enc<P>(t0, q.x, q.y)) | (uint32_t(dev_enc<P>(t1, q.z, q.w)) << 16);
                if (cx_of(i) != 0) {
                    xq[xslot_of(i)][ly][lx + 1] = w;
                    // periodic rows held whole: the wrap across the box's x faces
                    if (!GHOST && span) {
                        if (cx_of(i) > 0 && lx == tw - 1) xq[xslot_of(i)][ly][0] = w;
                        if (cx_of(i) < 0 && lx == 0) xq[xslot_of(i)][ly][tw + 1] = w;
                    }
                    return;
                }
                uint32_t dvo;
                if (GHOST) {
                    const bool out = (cy_of(i) < 0 && ylo) || (cy_of(i) > 0 && yhi) || (cz_of(i) < 0 && zlo) ||
                                     (cz_of(i) > 0 && zhi);
                    const int shift = (cy_of(i) + cz_of(i) * ny) * int(qnx);
                    dvo = out ? kOOB : uint32_t(int(elem) + shift) * EB + uint32_t(i) * plane_bytes;
                } else {
                    int dy = y + cy_of(i), dz = zc + cz_of(i);
                    dy = dy < 0 ? dy + ny : (dy >= ny ? dy - ny : dy);
                    dz = dz < 0 ? dz + nz : (dz >= nz ? dz - nz : dz);
                    dvo = ((uint32_t(dz) * uint32_t(ny) + uint32_t(dy)) * qnx + uint32_t(x)) * EB +
                          uint32_t(i) * plane_bytes;
                }
                __builtin_amdgcn_raw_buffer_store_b32(w, rd, dvo, 0, kStoreNT);
            };
            if constexpr (P == SCLBM_BF16DEV) {
                // BF16 halves are decoded by a shift or a mask, not inside the
                // multiply-add as FP16 halves are; decoding them again here costs
                // less than keeping the momentum's 36 decoded values alive (registers)
#pragma unroll
                for (int i = 0; i < Q; ++i) asm volatile("" : "+v"(fprev[i]));
            }
            const DevColl c0 = dev_coll(m[0], rho[0], u[0], om0);
            const DevColl c1 = dev_coll(m[1], rho[1], u[1], om1);
#pragma unroll
            for (int p = 1; p <= 9; ++p) {
                const int i = 2 * p - 1;
                float tp0, tm0, tp1, tm1;
                dev_pair(c0, p, dv(0, i), dv(0, i + 1), tp0, tm0);
                dev_pair(c1, p, dv(1, i), dv(1, i + 1), tp1, tm1);
                push(i, tp0, tp1);
                push(i + 1, tm0, tm1);
            }
            push(0, dev_rest(c0, dv(0, 0)), dev_rest(c1, dv(1, 0)));
            // the node's reference densities for the next step: its densities now
            const uint32_t rw = uint32_t(__builtin_bit_cast(unsigned short, __float2half_rn(rho[0]))) |
                                (uint32_t(__builtin_bit_cast(unsigned short, __float2half_rn(rho[1]))) << 16);
            __builtin_amdgcn_raw_buffer_store_b32(rw, rf_out, 4u * node, 0, kStoreNT);
        }
        if (GHOST && y < ny) {
            // Populations streaming in from ghost nodes, which hold
            // g_eq(rho_b, A (x_g - x_c)) (values per weight: rho_b times the bracket).
            // The lane's coordinates pass through an empty asm first, so that what this
            // code derives from them is computed here each plane instead of being
            // hoisted out of the march and held in registers (or scratch).
            int x_b = x, y_b = y, lx_b = lx, ly_b = ly;
            asm volatile("" : "+v"(x_b), "+v"(y_b), "+v"(lx_b), "+v"(ly_b));
            const float *A = gsc, *xcf = gsc + 9;
            // (b) y and z faces: the directions whose source lies beyond y = 0, y = ny - 1,
            // z = 0 or z = nz - 1 (edges included) take the ghost equilibrium at the
            // face node itself, both components as one word.  On a z-face plane every
            // lane writes its node's five z directions.
            if (valid && (zlo || zhi)) {
                const float dx0 = float(x_b) - xcf[0], dy0 = float(y_b) - xcf[1], dz0 = float(zc) - xcf[2];
                const float4 qr = rmq[sl(0)][ly_b + 1][lx_b + 1];
                const uint32_t code = zlo ? kZcode[0] : kZcode[1];  // nz >= 3: not both
#pragma nounroll
                for (int mz = 0; mz < 5; ++mz) {
                    const int i = int((code >> (5 * mz)) & 31u);
                    const int cx = c_rt(0, i), cy = c_rt(1, i), cz = c_rt(2, i);
                    const float br = ghost_bracket(A, dx0 - float(cx), dy0 - float(cy), dz0 - float(cz), cx, cy, cz);
                    const uint32_t w = uint32_t(dev_enc<P>(rhob[0] * br, qr.x, qr.y)) |
                                       (uint32_t(dev_enc<P>(rhob[1] * br, qr.z, qr.w)) << 16);
                    __builtin_amdgcn_raw_buffer_store_b32(w, rd, vo + uint32_t(i) * plane_bytes, 0, kStoreNT);
                }
            }
        }
        if (GHOST) {
            // (a) Ghosts beside the tile's rows at x = -1 and x = nx: their five
            // populations with c_x pointing into the box stream into the face nodes of
            // the rows y + c_y, z + c_z, and enter the x exchange at the tile's edge
            // columns.  The 2 x TY x 10 (side, row, direction, component) values go to
            // the tile's last wavefronts, entry g = (side TY + row) 10 + 2m + s in
            // lane g mod 64, so that few wavefronts issue this code; lane pairs (2m,
            // 2m + 1) share a wavefront, and lane 2m writes the word of both components.
            {
                constexpr int NXG = 20 * TY, NXW = (NXG + 63) / 64;
                static_assert(NXW <= NWAVES, "x-face ghosts need more wavefronts than the tile has");
                if (wid >= NWAVES - NXW) {
                    int lane_g = lane;
                    asm volatile("" : "+v"(lane_g));
                    const int g = (wid - (NWAVES - NXW)) * 64 + lane_g;
                    const int side = g / (10 * TY), r = (g / 10) % TY, q = g % 10;
                    if (g < NXG && r < th && (side ? right_face : left_face)) {
                        const float *A = gsc, *xcf = gsc + 9;
                        const int sgn = side ? -1 : 1;  // c_x of the incoming directions
                        const int m = q >> 1, s = q & 1;
                        // m = 0..4 -> (c_y, c_z) = (0,0), (1,0), (-1,0), (0,1), (0,-1)
                        const int cyv = m == 1 ? 1 : (m == 2 ? -1 : 0);
                        const int czv = m == 3 ? 1 : (m == 4 ? -1 : 0);
                        const int idx = sgn > 0 ? (m == 0 ? 1 : m == 1 ? 7 : m == 2 ? 9 : m == 3 ? 11 : 13)
                                                : (m == 0 ? 2 : m == 1 ? 10 : m == 2 ? 8 : m == 3 ? 14 : 12);
                        const int fx = side ? nx - 1 : 0;  // the receiving face node's x
                        const float br = ghost_bracket(A, float(fx - sgn) - xcf[0], float(y0 + r) - xcf[1],
                                                       float(zc) - xcf[2], sgn, cyv, czv);
                        // the receiver (fx, y + c_y, z + c_z) lies in the LDS window
                        const float4 qr = rmq[sl(czv)][r + 1 + cyv][fx - x0 + 1];
                        const uint32_t bits =
                            s ? dev_enc<P>(rhob[1] * br, qr.z, qr.w) : dev_enc<P>(rhob[0] * br, qr.x, qr.y);
                        const uint32_t other = uint32_t(__shfl_xor(int(bits), 1, 64));  // the pair lane's component
                        if (s == 0) xq[xslot_of(idx)][r][side ? tw + 1 : 0] = bits | (other << 16);
                    }
                }
            }
            // A tile holding the row y = 0 or y = ny - 1 writes that row's five y
            // directions (those also beyond a z face went above) as tasks of one
            // direction and one 64-node column each, spread over all its wavefronts
            // (rows beyond the box included), so that the face row's wavefronts do
            // not hold up the tile's barrier.
            const bool fy0 = y0 == 0, fy1 = y0 + th == ny;
            if (fy0 || fy1) {
                int lane_t = lane;
                asm volatile("" : "+v"(lane_t));
                const float *A = gsc, *xcf = gsc + 9;
                // task t: face t / (5 WX), direction (t / WX) mod 5 of its list, column t mod WX
#pragma nounroll
                for (int t = wid; t < 10 * WX; t += NWAVES) {
                    const int f = t / (5 * WX), my = (t / WX) % 5, c = t % WX;
                    if (f ? !fy1 : !fy0) continue;
                    const int i = int(((f ? kYcode[1] : kYcode[0]) >> (5 * my)) & 31u);
                    const int cx = c_rt(0, i), cy = c_rt(1, i), cz = c_rt(2, i);
                    if ((cz > 0 && zlo) || (cz < 0 && zhi)) continue;
                    const int yr = f ? ny - 1 : 0;
                    const int lxn = 64 * c + lane_t, xn = x0 + lxn;
                    // the face node's reference densities (in the window; a column beyond
                    // the tile's nodes reads a cell of the window and stores nothing)
                    const float4 qr = rmq[sl(0)][yr - y0 + 1][lxn + 1];
                    const float br = ghost_bracket(A, (float(xn) - xcf[0]) - float(cx), (float(yr) - xcf[1]) - float(cy),
                                                   (float(zc) - xcf[2]) - float(cz), cx, cy, cz);
                    const uint32_t w = uint32_t(dev_enc<P>(rhob[0] * br, qr.x, qr.y)) |
                                       (uint32_t(dev_enc<P>(rhob[1] * br, qr.z, qr.w)) << 16);
                    const uint32_t off = xn < x0 + tw ? ((uint32_t(zc) * uint32_t(ny) + uint32_t(yr)) * qnx +
                                                         uint32_t(i) * uint32_t(nx) + uint32_t(xn)) * EB
                                                      : kOOB;
                    __builtin_amdgcn_raw_buffer_store_b32(w, rd, off, 0, kStoreNT);
                }
            }
        }
        __syncthreads();
        // ---- 4. the c_x != 0 stores: lane x writes its own slot with the word pushed
        // from x - c_x (whole cache lines per wavefront); a tile that does not hold
        // whole rows also writes the one word that leaves it across each edge.
        if (valid) {
#pragma unroll
            for (int jx = 0; jx < NXD; ++jx) {
                const int i = jx < 2 ? jx + 1 : jx + 5;
                const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
                int yd = y + cy, zd = zc + cz;
                bool out = false;
                if (GHOST) {
                    out = yd < 0 || yd >= ny || zd < 0 || zd >= nz;
                } else {
                    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
                    zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
                }
                const uint32_t row = (uint32_t(zd) * uint32_t(ny) + uint32_t(yd)) * qnx + uint32_t(i) * uint32_t(nx);
                bool ok = !out;
                if (cx > 0 && lx == 0) ok = ok && (GHOST ? left_face : span);
                if (cx < 0 && lx == tw - 1) ok = ok && (GHOST ? right_face : span);
                __builtin_amdgcn_raw_buffer_store_b32(xq[jx][ly][lx + 1 - cx], rd, ok ? (row + uint32_t(x)) * EB : kOOB,
                                                      0, kStoreNT);
                if (!span) {
                    const bool edge = cx > 0 ? lx == tw - 1 : lx == 0;
                    int xd = x + cx;
                    bool go = edge && !out;
                    if (GHOST) go = go && (cx > 0 ? !right_face : !left_face);
                    else xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
                    if (go) __builtin_amdgcn_raw_buffer_store_b32(xq[jx][ly][lx + 1], rd, (row + uint32_t(xd)) * EB, 0, kStoreNT);
                }
            }
        }
        }  // k >= 2
        // ---- 5. roll the register window ----
        rprev = rcur;
#pragma unroll
        for (int i = 0; i < Q; ++i) fprev[i] = fcur[i];
    }
}

}  // namespace sclbm
