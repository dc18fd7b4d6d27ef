// Fused stream-and-collide step of the two-component Shan-Chen model
// (arXiv 2112.09972, Sec. 2 Eqs. 6-9, ghost boundary of Sec. 2 Eq. 8 and Sec. 3
// Eq. 14) for gfx950: FP64 and FP32 storage (the 16-bit deviation formats run
// k_step_dev, which shares the tiling, march and stores described here).
//
// State: f(n), the populations of both components after streaming, in
// row-blocked SoA order [box][component][z][y][direction][x]: for every (y, z)
// row of the box the 19 directions follow one another, each a run of nx values
// (x fastest).  A wavefront's 19 loads of one row then fall in one contiguous
// 19 nx-element block, and its pushes into the neighbouring rows into three
// such blocks, which keeps HBM pages open (measured 8 % more bandwidth than
// one plane per direction on the same access pattern).  One launch computes
// f(n+1) into the other buffer:
//   moments (Eq. 6) -> pair force from neighbour densities (Eq. 7) ->
//   velocity shift -> single-rate collision (Eq. 9) -> push to x + c_i, and on
//   boundary nodes the populations that stream in from the ghost nodes.
//
// Tiling.  A workgroup owns a tile of TY rows of WX wavefronts (64 WX x TY nodes
// in (x, y); 128 x 4 holds whole rows of a 128-wide box) and marches along z
// through a chunk of planes (up in even chunks, down in odd ones).  The force at
// plane z needs the densities of planes
// z-1, z, z+1 including a one-node ring around the tile; those densities live in
// a 4-slot rolling buffer in LDS.  Per plane each thread takes its node's 38
// populations into a register window (FP32 storage: loaded during the
// previous plane's collision) and sums them into densities, the workgroup adds the ring
// densities, and after a barrier the previous plane's window is collided.
// Ring densities (and the two chunk-end planes) are recomputed rather than
// exchanged between workgroups, so a step is a single launch with no grid-wide
// synchronisation.
//
// Stores.  Populations with c_x = 0 are pushed straight to x + c_i.  The ten
// with c_x != 0 pass through an LDS exchange buffer and, after a second barrier,
// each lane stores at its own x the value that x - c_x pushed: every store of a
// wavefront covers 64 aligned consecutive elements, i.e. whole cache lines.
// (Shifted stores leave partial lines that another wavefront completes later;
// the same access pattern without arithmetic runs at 3.7 TB/s with shifted
// stores and 5.1 TB/s with whole-line ones.)  Stores are non-temporal.
//
// Precision.  FP64 storage computes in FP64.  FP32 storage computes the
// collision in FP32 (or FP64: SCLBM_F32D); the densities of the force
// stencil are summed in FP64 (from the FP32 populations, so exactly up to the
// storage rounding): the stencil takes differences of neighbouring densities,
// and an FP32 sum leaves a rounding noise of a few 1e-7 in them that the
// velocity shift tau F / rho multiplies by G tau (measured on the 32^3 droplet
// box at tau = 3: 3e-5 density error after 500 steps with FP32 sums, 3.6e-6 with
// FP64 sums).
//
// Instruction economy (the kernel issues about as many VALU instructions as it
// can hide behind HBM traffic): populations are handled in opposite-velocity
// pairs (c_{2k} = -c_{2k-1}), which shares the symmetric and antisymmetric parts
// of the equilibrium and of the force stencil; the velocity shift
// tau_s F_s / rho_s = -G tau_s sum_i w_i rho_s'(x + c_i) c_i needs no division;
// every access goes through raw-buffer instructions with one 32-bit per-lane
// byte offset.  In ghost mode a push whose destination lies outside the box gets
// an out-of-range offset, which the buffer unit discards, instead of a branch.
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
    int zgroup;               // z-chunks that follow one another in the tile order (divides nzc)
    double omega[2];          // 1/tau
    double tau[2];
    double g;                 // G_AB
    double rho_b[2];          // ghost densities
    const __half *ref_src;    // deviation formats: per-node reference densities of f(n),
                              // [box][node][component]
    __half *ref_dst;          // and of f(n+1); unused otherwise
    double xc[3];             // box centre
};

// Byte offset the buffer unit treats as out of range (every population array
// of one component and box is smaller; checked on the host).
constexpr uint32_t kOOB = 0xFFFFFFF0u;

// Density of one component from its 19 populations, summed in opposite pairs.
// The own-node and ring paths both use this so that a node's density does not
// depend on which tile computed it.
template <typename R, typename W>
__device__ __forceinline__ R pair_density(const W (&f)[Q]) {
    R r = R(f[0]);
#pragma unroll
    for (int k = 1; k < Q; k += 2) r += R(f[k]) + R(f[k + 1]);
    return r;
}

// Equilibrium bracket rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2) of Sec. 2 Eq. 8 for
// both members of the pair (c, -c), as sym +- asym; aa = rho (1 - 3/2 u^2).
template <typename R>
__device__ __forceinline__ void eq_pair(R cu, R aa, R rho3, R rho45, R &plus, R &minus) {
    const R sym = (rho45 * cu) * cu + aa;
    const R asym = rho3 * cu;
    plus = sym + asym;
    minus = sym - asym;
}

// Weighted equilibria w_i g_eq,i (Sec. 2 Eq. 8) of the nine opposite pairs and of
// the rest population, handed to push(i, value) in a fixed order; aa = rho (1 -
// 3/2 u^2), r3 = 3 rho, r45 = 9/2 rho.  In FP64 the pairs go in order 1..9.  In
// FP32 the rounded weights make the first moment of the equilibrium
// 3 (w_1 + 4 w_2) rho u = rho u (1 + 3e-8) instead of rho u; a collision would then
// scale the momentum of every node by that factor at every step (about 1e-5 of
// the densities after 500 steps of the droplet box).  There the face diagonals go
// first and the antisymmetric part of each axis pair is taken as rho u_a / 2
// minus the diagonals' with c_a != 0, so that the first moment is rho u up to
// one rounding (the same equilibrium in exact arithmetic).
template <typename C, typename Push>
__device__ __forceinline__ void equilibrium_pairs(C ux, C uy, C uz, C r, C aa, C r3, C r45, Push &&push) {
    if constexpr (sizeof(C) == 8) {
#pragma unroll
        for (int p = 1; p <= 9; ++p) {
            const int i = 2 * p - 1;
            C cu = C(0);
            if (cx_of(i)) cu += C(cx_of(i)) * ux;
            if (cy_of(i)) cu += C(cy_of(i)) * uy;
            if (cz_of(i)) cu += C(cz_of(i)) * uz;
            C fplus, fminus;
            eq_pair<C>(cu, aa, r3, r45, fplus, fminus);
            push(i, w_of<C>(i) * fplus);
            push(i + 1, w_of<C>(i) * fminus);
        }
    } else {
        C mx = C(0), my = C(0), mz = C(0);  // sum over diagonals of c_a times the antisymmetric part
#pragma unroll
        for (int p = 4; p <= 9; ++p) {
            const int i = 2 * p - 1;
            C cu = C(0);
            if (cx_of(i)) cu += C(cx_of(i)) * ux;
            if (cy_of(i)) cu += C(cy_of(i)) * uy;
            if (cz_of(i)) cu += C(cz_of(i)) * uz;
            const C sym = w_of<C>(i) * ((r45 * cu) * cu + aa);
            const C asym = w_of<C>(i) * (r3 * cu);
            if (cx_of(i)) mx += C(cx_of(i)) * asym;
            if (cy_of(i)) my += C(cy_of(i)) * asym;
            if (cz_of(i)) mz += C(cz_of(i)) * asym;
            push(i, sym + asym);
            push(i + 1, sym - asym);
        }
        const C half = C(0.5) * r;
        const C ua[3] = {ux, uy, uz}, ma[3] = {mx, my, mz};
#pragma unroll
        for (int p = 1; p <= 3; ++p) {
            const int i = 2 * p - 1;
            const C u = ua[p - 1];
            const C sym = w_of<C>(i) * ((r45 * u) * u + aa);
            const C asym = half * u - ma[p - 1];
            push(i, sym + asym);
            push(i + 1, sym - asym);
        }
    }
    push(0, w_of<C>(0) * aa);
}

// The ten directions with c_x != 0 have slots j = 0..9 in the x-exchange
// buffer (odd directions c_x = +1, even ones -1).
constexpr int NXD = 10;
__host__ __device__ constexpr int xslot_of(int i) { return i < 3 ? i - 1 : i - 5; }

// Directions whose source lies beyond a face: [0] beyond y = 0 (c_y = +1) or
// z = 0 (c_z = +1), [1] beyond y = ny - 1 or z = nz - 1 (c = -1).
constexpr int kYin[2][5] = {{3, 7, 10, 15, 17}, {4, 8, 9, 16, 18}};
constexpr int kZin[2][5] = {{5, 11, 14, 15, 18}, {6, 12, 13, 16, 17}};
__host__ __device__ constexpr bool face_lists_ok() {
    for (int f = 0; f < 2; ++f) {
        const int sg = f ? -1 : 1;
        int ny = 0, nz = 0;
        for (int i = 0; i < Q; ++i) {
            ny += cy_of(i) == sg;
            nz += cz_of(i) == sg;
        }
        if (ny != 5 || nz != 5) return false;
        for (int m = 0; m < 5; ++m)
            if (cy_of(kYin[f][m]) != sg || cz_of(kZin[f][m]) != sg) return false;
    }
    return true;
}
static_assert(face_lists_ok(), "face direction lists");
// the lists packed five bits per entry, for loops that are not unrolled
__host__ __device__ constexpr uint32_t pack_dirs(const int (&l)[5]) {
    uint32_t p = 0;
    for (int m = 0; m < 5; ++m) p |= uint32_t(l[m]) << (5 * m);
    return p;
}
constexpr uint32_t kYcode[2] = {pack_dirs(kYin[0]), pack_dirs(kYin[1])};
constexpr uint32_t kZcode[2] = {pack_dirs(kZin[0]), pack_dirs(kZin[1])};

template <int P, int TY, int WX, bool GHOST, int WAVES>
__global__ __launch_bounds__(64 * WX * TY, WAVES) void k_step(StepArgs a) {
    using S = typename Prec<P>::S;
    using W = typename Prec<P>::W;
    using R = typename Prec<P>::R;
    using B = typename Prec<P>::B;
    using L = typename Prec<P>::L;
    using C = R;  // collision arithmetic
    using D = typename Prec<P>::D;  // densities of the force stencil
    constexpr int TXW = 64 * WX;  // tile width: WX wavefronts per row
    constexpr int LW = TXW + 2;   // with the ring
    constexpr uint32_t EB = sizeof(S);
    // the next plane's populations (raw words, decoded when the plane is used, so
    // that nothing waits for them during the collision) are loaded while the
    // current one collides.  FP64 windows leave no registers for a third plane.
    constexpr bool PREFETCH = sizeof(S) < 8;
    // the x-exchange values read from LDS together before their stores (FP32 storage)
    constexpr bool BATCH = PREFETCH;
    static_assert(!Prec<P>::DEV, "the 16-bit deviation formats run k_step_dev");
    // density window: the planes zc - 1, zc, zc + 1 of the collision and one more
    constexpr int NSLOT = 4;
    __shared__ D lds[NSLOT][2][TY + 2][LW];
    // x exchange: post-collision values with c_x != 0, by component, slot, row and
    // column lx + 1; columns 0 and tw + 1 hold what streams in across the tile's
    // left and right edges (ghost populations, or the periodic wrap)
    __shared__ B xq[2][NXD][TY][LW];

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * TXW + lx;
    const int lane = lx & 63;
    // wavefront index within the workgroup, uniform (a scalar register)
    constexpr int NWAVES = TY * WX;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware tile order: workgroups are dispatched round-robin over the 8
    // XCDs by linear id, so give XCD k one contiguous run of tiles, ordered x
    // fastest, then a group of zgroup z-chunks, then y, then the chunk groups,
    // then box.  Tiles that run at the same time on one XCD then cover a block
    // of neighbouring rows (and, for groups of several chunks, chunks): their ring
    // rows hit in that XCD's L2, and since even chunks march up in z and odd ones
    // down, the planes at a chunk boundary inside a group are read by two tiles at
    // about the same time.  (The host passes groups of one chunk: measured faster
    // or equal since the ghost faces were balanced.)
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
    const int tw = min(TXW, a.nx - x0), th = min(TY, a.ny - y0);  // valid tile extent
    const bool left_face = x0 == 0, right_face = x0 + tw == a.nx;
    const bool span = left_face && right_face;                     // the tile holds whole rows
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t N = uint32_t(a.nnode);
    const uint32_t nxy = uint32_t(nx) * uint32_t(ny);
    const uint32_t qnx = uint32_t(Q) * uint32_t(nx);  // elements per (y, z) row, all directions
    const uint32_t plane_bytes = uint32_t(nx) * EB;   // from one direction to the next within a row

    // one descriptor per component and buffer; 19 N elements each (< 4 GiB, checked on the host)
    const uint32_t comp_bytes = uint32_t(Q) * N * EB;
    const S *src = (const S *)a.src + (int64_t)box * 2 * Q * N;
    S *dst = (S *)a.dst + (int64_t)box * 2 * Q * N;
    const rsrc_t rs[2] = {make_rsrc(src, comp_bytes), make_rsrc(src + (int64_t)Q * N, comp_bytes)};
    const rsrc_t rd[2] = {make_rsrc(dst, comp_bytes), make_rsrc(dst + (int64_t)Q * N, comp_bytes)};

    const int64_t n = *a.clk_in;
    if (lin == 0 && tid == 0) *a.clk_out = n + 1;

    const R rhob[2] = {R(a.rho_b[0]), R(a.rho_b[1])};
    const D rhobd[2] = {D(a.rho_b[0]), D(a.rho_b[1])};
    // velocity gradient of step n (ghost mode), read before the first store so
    // that the reads are uniform scalar loads (no wait on the vector-memory queue)
    R Am[9];
    if (GHOST) {
        const double *Arow = a.atab + ((int64_t)box * a.table_len + (n - a.tab_first[box])) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) Am[q] = R(Arow[q]);
    }

    static_assert(2 * (TXW + 2) + 2 * TY <= TXW * TY, "one ring node per thread");
    const int ringN = 2 * (tw + 2) + 2 * th;
    const int nplanes = (ze - zs) + 2;

    // own node of plane z: whether it is inside the box (ghost mode), its
    // population byte offset and node index (periodic mode wraps z)
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
    // raw words of the next plane
    L fnx[2][Q];
    bool nx_in = false;
    // rows that no other workgroup reads: not a tile edge row in y, not a chunk-end
    // plane, in a ghost-mode tile holding whole rows (no ring columns taken from it)
    const bool row_once = GHOST && span && ly > 0 && ly < th - 1;
    auto prefetch = [&](int z) {
        uint32_t vo, nd;
        nx_in = own_node(z, vo, nd);
        if (nx_in) {
            const bool once = row_once && z > zs && z < ze - 1;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (once) {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        fnx[s][i] = Prec<P>::template bload_raw<kLoadNT>(rs[s], vo, uint32_t(i) * plane_bytes);
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i) fnx[s][i] = Prec<P>::bload_raw(rs[s], vo, uint32_t(i) * plane_bytes);
                }
            }
        }
    };
    const int dir = (chunk & 1) ? -1 : 1;  // march direction in z
    const int zfirst = dir > 0 ? zs - 1 : ze;
    if (PREFETCH) prefetch(zfirst);

    W fprev[2][Q], fcur[2][Q];
    for (int k = 0; k < nplanes; ++k) {
        const int z = zfirst + dir * k;
        const int slot = k % NSLOT;
        if constexpr (kDebugFill) {
            // debug build: this plane's density slot and the exchange buffer start as NaN
            __syncthreads();
            lds_fill(&lds[slot][0][0][0], 2 * (TY + 2) * LW, D(__builtin_nan("")), tid, 64 * WX * TY);
            lds_fill(&xq[0][0][0][0], 2 * NXD * TY * LW, nan_bits<B>(P), tid, 64 * WX * TY);
            __syncthreads();
        }
        // ---- 1. densities of plane z: own node (into the register window) and one
        // ring node per thread ----
        bool own_in;
        if (PREFETCH) {
            own_in = nx_in;
            if (own_in) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int i = 0; i < Q; ++i) fcur[s][i] = Prec<P>::dec(fnx[s][i], R(0));
            }
        } else {
            uint32_t own_vo, own_nd;
            own_in = own_node(z, own_vo, own_nd);
            if (own_in) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int i = 0; i < Q; ++i) fcur[s][i] = Prec<P>::bload(rs[s], own_vo, uint32_t(i) * plane_bytes, R(0));
            }
        }
        bool ring_on = false, ring_in = false;
        uint32_t ring_vo = 0;
        int rsx = 0, rsy = 0;
        if (tid < ringN) {
            // threads 0 .. 2 tw - 1: the ring rows y0 - 1 and y0 + th at x0 .. x0 + tw - 1,
            // lane by lane from x0, so that a wavefront's loads of a ring row cover
            // whole cache lines as the own row's do; then the two ring columns
            // x0 - 1 and x0 + tw, corners included, node by node
            const int r = tid;
            if (r < 2 * tw) {
                rsy = r < tw ? 0 : th + 1;
                rsx = (r < tw ? r : r - tw) + 1;
            } else {
                const int q = r - 2 * tw;  // 0 .. 2 (th + 2) - 1
                rsx = q < th + 2 ? 0 : tw + 1;
                rsy = q < th + 2 ? q : q - (th + 2);
            }
            int gx = x0 - 1 + rsx, gy = y0 - 1 + rsy, gz = z;
            ring_in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            if (!GHOST) {
                gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
                gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
                gz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);
                ring_in = true;
            }
            ring_on = true;
            ring_vo = ((uint32_t(gz) * uint32_t(ny) + uint32_t(gy)) * qnx + uint32_t(gx)) * EB;
        }
        if (valid) {
            const D r0 = own_in ? pair_density<D>(fcur[0]) : rhobd[0];
            const D r1 = own_in ? pair_density<D>(fcur[1]) : rhobd[1];
            lds[slot][0][ly + 1][lx + 1] = r0;
            lds[slot][1][ly + 1][lx + 1] = r1;
        }
        if (ring_on) {
            D rr[2] = {rhobd[0], rhobd[1]};
            if (ring_in) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    W f[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) f[i] = Prec<P>::bload(rs[s], ring_vo, uint32_t(i) * plane_bytes, R(0));
                    rr[s] = pair_density<D>(f);
                }
            }
            lds[slot][0][rsy][rsx] = rr[0];
            lds[slot][1][rsy][rsx] = rr[1];
        }
        __syncthreads();
        // ---- 2. the next plane's loads go out now and land during the collision ----
        if (PREFETCH && k + 1 < nplanes) prefetch(z + dir);
        if (k >= 2) {
        // ---- 3. collide the previous plane of the march, zc = z - dir: c_x = 0
        // populations are pushed now, the others go through LDS ----
        const int zc = z - dir;  // plane zc + d sits in LDS slot sl(d)
        auto sl = [&](int d) { return (k - 1 + dir * d) % NSLOT; };  // k >= 2: never negative
        const uint32_t elem = (uint32_t(zc) * uint32_t(ny) + uint32_t(y)) * qnx + uint32_t(x);
        const uint32_t vo = elem * EB;
        const bool ylo = y == 0, yhi = y == ny - 1;
        const bool zlo = zc == 0, zhi = zc == nz - 1;
        if (valid) {
            const W (&f)[2][Q] = fprev;  // populations of plane zc, loaded one plane ago
            // moments, Eq. 6: density and momentum from pair sums and differences
            R rho[2], j[2][3];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                R d[10];
#pragma unroll
                for (int p = 1; p <= 9; ++p) d[p] = R(f[s][2 * p - 1]) - R(f[s][2 * p]);
                // the density summed when the plane was loaded (same value)
                rho[s] = R(lds[sl(0)][s][ly + 1][lx + 1]);
                j[s][0] = d[1] + d[4] + d[5] + d[6] + d[7];
                j[s][1] = d[2] + d[4] - d[5] + d[8] + d[9];
                j[s][2] = d[3] + d[6] - d[7] + d[8] - d[9];
            }
            // pair force, Eq. 7, as the stencil sum sig_s = sum_i w_i rho_s'(x + c_i) c_i
            // (F_s = -G rho_s sig_s) from pair differences of the LDS densities
            D sig[2][3];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int o = 1 - s;
                D e[10];
#pragma unroll
                for (int p = 1; p <= 9; ++p) {
                    const int i = 2 * p - 1;
                    const D hi = lds[sl(cz_of(i))][o][ly + 1 + cy_of(i)][lx + 1 + cx_of(i)];
                    const D lo = lds[sl(-cz_of(i))][o][ly + 1 - cy_of(i)][lx + 1 - cx_of(i)];
                    e[p] = hi - lo;
                }
                const D w1 = D(1) / D(18), w2 = D(1) / D(36);
                sig[s][0] = w1 * e[1] + w2 * (e[4] + e[5] + e[6] + e[7]);
                sig[s][1] = w1 * e[2] + w2 * (e[4] - e[5] + e[8] + e[9]);
                sig[s][2] = w1 * e[3] + w2 * (e[6] - e[7] + e[8] - e[9]);
            }
            // common velocity u' and shifted velocity u' + tau_s F_s / rho_s = u' - G tau_s sig_s
            const R om0 = R(a.omega[0]), om1 = R(a.omega[1]);
            const R inv_den = R(1) / (rho[0] * om0 + rho[1] * om1);
            const R up[3] = {(j[0][0] * om0 + j[1][0] * om1) * inv_den, (j[0][1] * om0 + j[1][1] * om1) * inv_den,
                             (j[0][2] * om0 + j[1][2] * om1) * inv_den};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const C om = C(s ? om1 : om0);
                const D gt = D(a.g) * D(a.tau[s]);
                C ux, uy, uz;
                if constexpr (sizeof(D) > sizeof(C)) {
                    // FP32 arithmetic: the shift from the FP64 stencil sum, rounded once
                    ux = C(up[0]) - C(gt * sig[s][0]);
                    uy = C(up[1]) - C(gt * sig[s][1]);
                    uz = C(up[2]) - C(gt * sig[s][2]);
                } else {
                    ux = C(up[0] - gt * sig[s][0]);
                    uy = C(up[1] - gt * sig[s][1]);
                    uz = C(up[2] - gt * sig[s][2]);
                }
                const C usq = ux * ux + uy * uy + uz * uz;
                const C r = C(rho[s]);
                const C aa = r - C(1.5) * r * usq;
                const C r3 = C(3) * r, r45 = C(4.5) * r;
                // the nine opposite pairs, then the rest population: equilibrium, collision, push
                // In FP32 arithmetic the rounded weights sum to 1 + 3e-8, so the single-rate
                // update would create that much mass per collision; there the rest
                // population takes the mass balance rho - sum_{i>0} p_i instead (equal in
                // exact arithmetic).
                constexpr bool BALANCE = sizeof(C) == 4;
                C psum = C(0);
                auto push = [&](int i, C geq) {
                    const C fi = C(f[s][i]);
                    C pst = fi + om * (geq - fi);
                    if (BALANCE) {
                        if (i == 0) pst = C(rho[s]) - psum;
                        else psum += pst;
                    }
                    const B bits = Prec<P>::enc(pst, C(0));
                    if (cx_of(i) != 0) {
                        xq[s][xslot_of(i)][ly][lx + 1] = bits;
                        // periodic rows held whole: the wrap across the box's x faces
                        if (!GHOST && span) {
                            if (cx_of(i) > 0 && lx == tw - 1) xq[s][xslot_of(i)][ly][0] = bits;
                            if (cx_of(i) < 0 && lx == 0) xq[s][xslot_of(i)][ly][tw + 1] = bits;
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
                    Prec<P>::bstore_bits(rd[s], dvo, 0, bits);
                };
                equilibrium_pairs<C>(ux, uy, uz, r, aa, r3, r45, push);
            }
        }
        // bracket of the ghost equilibrium g_eq(rho_b, A (x_g - x_c)) = w_i rho_b br of
        // direction i (known only at run time: the face loops are not unrolled) at
        // the ghost x_g = (xn, yn, zn) - c_i
        auto ghost_bracket = [&](int i, int xn, int yn, int zn) -> R {
            const int cx = c_rt(0, i), cy = c_rt(1, i), cz = c_rt(2, i);
            const R dxg = (R(xn) - R(a.xc[0])) - R(cx), dyg = (R(yn) - R(a.xc[1])) - R(cy);
            const R dzg = (R(zn) - R(a.xc[2])) - R(cz);
            const R gx = Am[0] * dxg + Am[1] * dyg + Am[2] * dzg;
            const R gy = Am[3] * dxg + Am[4] * dyg + Am[5] * dzg;
            const R gz = Am[6] * dxg + Am[7] * dyg + Am[8] * dzg;
            const R cu = R(cx) * gx + R(cy) * gy + R(cz) * gz;
            const R usq = gx * gx + gy * gy + gz * gz;
            return R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq;
        };
        if (GHOST && y < ny) {
            // Populations streaming in from ghost nodes, which hold
            // g_eq(rho_b, A (x_g - x_c)).
            // (b) y and z faces: the directions whose source lies beyond y = 0, y = ny - 1,
            // z = 0 or z = nz - 1 (edges included) take the ghost equilibrium at the
            // face node itself.  On a z-face plane every lane writes its node's five
            // z directions.
            if (valid && (zlo || zhi)) {
                const uint32_t code = zlo ? kZcode[0] : kZcode[1];  // nz >= 3: not both
#pragma nounroll
                for (int m = 0; m < 5; ++m) {
                    const int i = int((code >> (5 * m)) & 31u);
                    const R br = ghost_bracket(i, x, y, zc);
                    const R wgt = i < 7 ? R(1) / R(18) : R(1) / R(36);
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        Prec<P>::bstore_bits(rd[s], vo + uint32_t(i) * plane_bytes, 0, Prec<P>::enc(wgt * rhob[s] * br, R(0)));
                }
            }
        }
        if (GHOST) {
            // (a) Ghosts beside the tile's rows at x = -1 and x = nx: their five
            // populations with c_x pointing into the box stream into the face nodes of
            // the rows y + c_y, z + c_z, and enter the x exchange at the tile's edge
            // columns.  The 2 x TY x 10 (side, row, direction, component) values go to
            // the tile's last wavefronts, entry g = (side TY + row) 10 + 2m + s in
            // lane g mod 64, so that few wavefronts issue this code.
            {
                constexpr int NXG = 20 * TY, NXW = (NXG + 63) / 64;
                static_assert(NXW <= NWAVES, "x-face ghosts need more wavefronts than the tile has");
                if (wid >= NWAVES - NXW) {
                    const int g = (wid - (NWAVES - NXW)) * 64 + lane;
                    const int side = g / (10 * TY), r = (g / 10) % TY, q = g % 10;
                    if (g < NXG && r < th && (side ? right_face : left_face)) {
                        const int sgn = side ? -1 : 1;  // c_x of the incoming directions
                        const int m = q >> 1, s = q & 1;
                        // m = 0..4 -> (c_y, c_z) = (0,0), (1,0), (-1,0), (0,1), (0,-1)
                        const int cyv = m == 1 ? 1 : (m == 2 ? -1 : 0);
                        const int czv = m == 3 ? 1 : (m == 4 ? -1 : 0);
                        const int idx = sgn > 0 ? (m == 0 ? 1 : m == 1 ? 7 : m == 2 ? 9 : m == 3 ? 11 : 13)
                                                : (m == 0 ? 2 : m == 1 ? 10 : m == 2 ? 8 : m == 3 ? 14 : 12);
                        const int fx = side ? nx - 1 : 0;  // the receiving face node's x
                        const R dxg = R(fx - sgn) - R(a.xc[0]), dyg = R(y0 + r) - R(a.xc[1]), dzg = R(zc) - R(a.xc[2]);
                        const R gx = Am[0] * dxg + Am[1] * dyg + Am[2] * dzg;
                        const R gy = Am[3] * dxg + Am[4] * dyg + Am[5] * dzg;
                        const R gz = Am[6] * dxg + Am[7] * dyg + Am[8] * dzg;
                        const R cu = R(sgn) * gx + R(cyv) * gy + R(czv) * gz;
                        const R usq = gx * gx + gy * gy + gz * gz;
                        const R wgt = m == 0 ? R(1) / R(18) : R(1) / R(36);
                        const R geq =
                            wgt * (s ? rhob[1] : rhob[0]) * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
                        // the receiver (fx, y + c_y, z + c_z) lies in the LDS window (plane slots k-2..k)
                        xq[s][xslot_of(idx)][r][side ? tw + 1 : 0] = Prec<P>::enc(geq, R(0));
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
                // task t: face t / (5 WX), direction (t / WX) mod 5 of its list, column t mod WX
#pragma nounroll
                for (int t = wid; t < 10 * WX; t += NWAVES) {
                    const int f = t / (5 * WX), m = (t / WX) % 5, c = t % WX;
                    if (f ? !fy1 : !fy0) continue;
                    const int i = int(((f ? kYcode[1] : kYcode[0]) >> (5 * m)) & 31u);
                    const int cz = c_rt(2, i);
                    if ((cz > 0 && zlo) || (cz < 0 && zhi)) continue;
                    const int yr = f ? ny - 1 : 0;
                    const int xn = x0 + 64 * c + lane;
                    const uint32_t off = xn < x0 + tw ? ((uint32_t(zc) * uint32_t(ny) + uint32_t(yr)) * qnx +
                                                         uint32_t(i) * uint32_t(nx) + uint32_t(xn)) * EB
                                                      : kOOB;
                    const R br = ghost_bracket(i, xn, yr, zc);
                    const R wgt = i < 7 ? R(1) / R(18) : R(1) / R(36);
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        Prec<P>::bstore_bits(rd[s], off, 0, Prec<P>::enc(wgt * rhob[s] * br, R(0)));
                }
            }
        }
        __syncthreads();
        // ---- 4. the c_x != 0 stores: lane x writes its own slot with the value
        // pushed from x - c_x, so that every store of a wavefront covers 64 aligned
        // consecutive elements (whole cache lines).  A tile that does not hold whole
        // rows also writes the one value that leaves it across each edge.
        if (valid && BATCH) {
            // FP32 storage: all ten values per component first, so that the LDS reads
            // overlap instead of each store waiting for its own read
            B wq[2][NXD];
#pragma unroll
            for (int jx = 0; jx < NXD; ++jx) {
                const int cx = cx_of(jx < 2 ? jx + 1 : jx + 5);
#pragma unroll
                for (int s = 0; s < 2; ++s) wq[s][jx] = xq[s][jx][ly][lx + 1 - cx];
            }
            // destination row of direction i and whether it lies outside the box (ghost mode)
            auto dest_row = [&](int i, bool &out) -> uint32_t {
                int yd = y + cy_of(i), zd = zc + cz_of(i);
                out = false;
                if (GHOST) {
                    out = yd < 0 || yd >= ny || zd < 0 || zd >= nz;
                } else {
                    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
                    zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
                }
                return (uint32_t(zd) * uint32_t(ny) + uint32_t(yd)) * qnx + uint32_t(i) * uint32_t(nx);
            };
#pragma unroll
            for (int jx = 0; jx < NXD; ++jx) {
                const int i = jx < 2 ? jx + 1 : jx + 5;
                const int cx = cx_of(i);
                bool out;
                const uint32_t row = dest_row(i, out);
                bool ok = !out;
                if (cx > 0 && lx == 0) ok = ok && (GHOST ? left_face : span);
                if (cx < 0 && lx == tw - 1) ok = ok && (GHOST ? right_face : span);
#pragma unroll
                for (int s = 0; s < 2; ++s) Prec<P>::bstore_bits(rd[s], ok ? (row + uint32_t(x)) * EB : kOOB, 0, wq[s][jx]);
            }
            // a tile that does not hold whole rows also writes the value leaving it
            // across each edge, in a loop of its own so that no branch separates the
            // reads above from their stores
            if (!span) {
#pragma unroll
                for (int jx = 0; jx < NXD; ++jx) {
                    const int i = jx < 2 ? jx + 1 : jx + 5;
                    const int cx = cx_of(i);
                    bool out;
                    const uint32_t row = dest_row(i, out);
                    const bool edge = cx > 0 ? lx == tw - 1 : lx == 0;
                    int xd = x + cx;
                    bool go = edge && !out;
                    if (GHOST) go = go && (cx > 0 ? !right_face : !left_face);
                    else xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
                    if (go) {
#pragma unroll
                        for (int s = 0; s < 2; ++s)
                            Prec<P>::bstore_bits(rd[s], (row + uint32_t(xd)) * EB, 0, xq[s][jx][ly][lx + 1]);
                    }
                }
            }
        } else if (valid) {
            // FP64 storage (no registers left for the values): one read per store
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
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    Prec<P>::bstore_bits(rd[s], ok ? (row + uint32_t(x)) * EB : kOOB, 0, xq[s][jx][ly][lx + 1 - cx]);
                if (!span) {
                    const bool edge = cx > 0 ? lx == tw - 1 : lx == 0;
                    int xd = x + cx;
                    bool go = edge && !out;
                    if (GHOST) go = go && (cx > 0 ? !right_face : !left_face);
                    else xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
                    if (go) {
#pragma unroll
                        for (int s = 0; s < 2; ++s)
                            Prec<P>::bstore_bits(rd[s], (row + uint32_t(xd)) * EB, 0, xq[s][jx][ly][lx + 1]);
                    }
                }
            }
        }
        }  // k >= 2
        // ---- 5. roll the register window ----
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) fprev[s][i] = fcur[s][i];
    }
}

}  // namespace sclbm
