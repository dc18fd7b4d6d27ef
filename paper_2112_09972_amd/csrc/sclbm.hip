// C-ABI host library of the two-component Shan-Chen lattice Boltzmann solver
// (arXiv 2112.09972).  Declarations and the contract of every call: sclbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "analysis_kernels.hpp"
#include "aux_kernels.hpp"
#include "lattice.hpp"
#include "mm_kernel.hpp"
#include "sclbm.h"
#include "step_kernel.hpp"
#include "step_dev_kernel.hpp"

using namespace sclbm;

namespace {

thread_local std::string g_err;

sclbm_status fail(sclbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(SCLBM_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                          \
    } while (0)

#define HIP_LAUNCHED()                                                                                  \
    do {                                                                                                \
        hipError_t e_ = hipGetLastError();                                                              \
        if (e_ != hipSuccess) return fail(SCLBM_EHIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                          \
    } while (0)

constexpr size_t kAlign = 256;
size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t f0, f1, ref0, ref1, atab, first, clock, partial, result, mass, diag, total;
    size_t fbytes;    // populations of every box, one buffer
    size_t refbytes;  // per-node FP16 reference densities (deviation formats), one buffer
};

bool config_ok(const sclbm_config *c, std::string &why) {
    if (!c) { why = "null config"; return false; }
    if (c->nx < 3 || c->ny < 3 || c->nz < 3) { why = "nx, ny, nz must be >= 3"; return false; }
    if (c->nx > 4096 || c->ny > 65535 || c->nz > 65535) { why = "box too large"; return false; }
    if (c->nbox < 1) { why = "nbox must be >= 1"; return false; }
    if (c->bc != SCLBM_BC_PERIODIC && c->bc != SCLBM_BC_GHOST) { why = "unknown boundary mode"; return false; }
    if (c->prec < SCLBM_F64 || c->prec > SCLBM_F32D) { why = "unknown precision"; return false; }
    if (!(c->tau[0] > 0.5) || !(c->tau[1] > 0.5)) { why = "tau must exceed 1/2"; return false; }
    if (!(c->rho_b[0] > 0.0) || !(c->rho_b[1] > 0.0)) { why = "rho_b must be positive"; return false; }
    if (!std::isfinite(c->g_ab)) { why = "g_ab must be finite"; return false; }
    if (!(c->mach_max >= 0.0)) { why = "mach_max must be >= 0"; return false; }
    if (c->bc == SCLBM_BC_GHOST && c->table_len < 1) { why = "ghost mode needs table_len >= 1"; return false; }
    if (c->table_len < 0) { why = "table_len must be >= 0"; return false; }
    const double nodes = double(c->nx) * c->ny * c->nz * c->nbox;
    if (nodes * 2 * Q * elem_bytes(c->prec) > 250e9) { why = "populations exceed 250 GB"; return false; }
    // the step kernel addresses one component of one box (both, in the deviation
    // formats' shared words) through a raw buffer (32-bit byte offsets)
    if (double(c->nx) * c->ny * c->nz * Q * elem_bytes(c->prec) * (is_dev(c->prec) ? 2 : 1) >= 4294901760.0) {
        why = "one box's populations of one component (both, 16-bit formats) exceed 4 GiB";
        return false;
    }
    return true;
}

// Workgroups per box of the statistics reduction: about 2048 nodes each, at
// least enough to fill the chip when all boxes are reduced together.
size_t stats_blocks(const sclbm_config *c) {
    const size_t N = size_t(c->nx) * c->ny * c->nz;
    size_t b = std::max<size_t>(1, N / 2048);
    b = std::max<size_t>(b, (1024 + c->nbox - 1) / c->nbox);
    return std::min<size_t>(b, NRED_MAX_PER_BOX);
}

Layout make_layout(const sclbm_config *c) {
    Layout L{};
    const size_t N = size_t(c->nx) * c->ny * c->nz;
    L.fbytes = size_t(c->nbox) * 2 * Q * N * elem_bytes(c->prec);
    L.refbytes = is_dev(c->prec) ? size_t(c->nbox) * 2 * N * 2 : 0;
    size_t off = 0;
    L.f0 = off; off += round_up(L.fbytes);
    L.f1 = off; off += round_up(L.fbytes);
    L.ref0 = off; off += round_up(L.refbytes);
    L.ref1 = off; off += round_up(L.refbytes);
    L.atab = off; off += round_up(size_t(c->nbox) * size_t(c->bc == SCLBM_BC_GHOST ? c->table_len : 0) * 9 * 8);
    L.first = off; off += round_up(size_t(c->nbox) * 8);
    L.clock = off; off += round_up(2 * 8);
    L.partial = off; off += round_up(std::max<size_t>(size_t(NRED_BLOCKS), size_t(c->nbox) * stats_blocks(c)) * NSTAT * 8);
    L.result = off; off += round_up(size_t(c->nbox) * NSTAT * 8);
    L.mass = off; off += round_up(size_t(c->nbox) * 2 * 8);  // droplet mass now, reinjection target
    L.diag = off; off += round_up(5 * N * 8);
    L.total = off;
    return L;
}

}  // namespace

// Device memory of the allocation-free droplet moments
// (sclbm_droplet_moments_all_static): the statistics partials and per-box
// results.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` names no device address; the address on a
// device comes from hipGetSymbolAddress with that device current.
constexpr size_t kScratchDoubles = size_t(1) << 18;  // 2 MiB
__device__ __align__(256) static double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, resolved once per device; `dev` must be
// the current device.
sclbm_status scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SCLBM_EINVAL, "device %d out of range [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SCLBM_EHIP, "no device address for the static scratch on device %d", dev);
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return SCLBM_OK;
}

}  // namespace

struct sclbm_ctx {
    sclbm_config cfg;
    Layout lay;
    char *ws;
    hipStream_t stream;
    int64_t n;        // time of the state
    int par;          // which population buffer holds f(n): 0 -> f0
    int tile_rows;    // TY
    int tile_waves;   // WX: wavefronts per tile row (tile width 64 WX)
    int zchunk;
    std::vector<int64_t> tab_first, tab_len;  // host copies, per box
    // captured step loop: valid for (graph_steps, graph_par, graph_ty, graph_wx, graph_zc)
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_steps = 0;
    int graph_par = -1, graph_ty = 0, graph_wx = 0, graph_zc = 0;
    int64_t N;
    BoxGeom geom;
    int device = 0;   // HIP device current at create
    int64_t health_every = 0;  // check every box for NaN/Inf and non-positive densities every so many steps (0: off)

    void *fbuf(int which) { return ws + (which ? lay.f1 : lay.f0); }
    __half *refbuf(int which) {
        return lay.refbytes ? reinterpret_cast<__half *>(ws + (which ? lay.ref1 : lay.ref0)) : nullptr;
    }
    __half *box_ref(int which, int box) { return lay.refbytes ? refbuf(which) + size_t(box) * 2 * size_t(N) : nullptr; }
    size_t box_bytes() const { return size_t(2) * Q * size_t(N) * elem_bytes(cfg.prec); }
    double *partial() { return reinterpret_cast<double *>(ws + lay.partial); }
    double *result() { return reinterpret_cast<double *>(ws + lay.result); }
    double *mass_now() { return reinterpret_cast<double *>(ws + lay.mass); }
    double *mass_target() { return reinterpret_cast<double *>(ws + lay.mass) + cfg.nbox; }
    double *diag() { return reinterpret_cast<double *>(ws + lay.diag); }
    int64_t *clock() { return reinterpret_cast<int64_t *>(ws + lay.clock); }
};

namespace {

void drop_graph(sclbm_ctx *c);

sclbm_status check_ctx(const sclbm_ctx *c) {
    if (!c) return fail(SCLBM_EINVAL, "null context");
    return SCLBM_OK;
}

sclbm_status check_box(const sclbm_ctx *c, int32_t box, bool allow_all) {
    if (allow_all && box == -1) return SCLBM_OK;
    if (box < 0 || box >= c->cfg.nbox) return fail(SCLBM_EINVAL, "box %d out of range [0, %d)", box, c->cfg.nbox);
    return SCLBM_OK;
}

// Waves per SIMD the 16-bit formats' step kernel is compiled for (at most 128 VGPRs).
constexpr int kDevWaves = 4;

// Tile shapes of the step kernels: (rows, 64-node columns).  (4, 4), 256 nodes
// wide in 16 wavefronts, needs four waves per SIMD: the 16-bit formats only.
bool valid_tile(const sclbm_config &c, int ty, int wx) {
    if (ty == 4 && wx == 4) return is_dev(c.prec);
    return (ty == 4 && (wx == 1 || wx == 2)) || (ty == 8 && wx == 1);
}

// Default tile: 128 x 4 (whole 128-wide rows: every x-shifted store writes whole
// cache lines), unless the last 128-wide tile of a row would be at most half
// full; then 64 x 8, which leaves fewer idle lanes (measured at 160^3: 402
// against 463 us per step).
void default_tile(const sclbm_config &c, int &ty, int &wx) {
    const int tail = c.nx % 128;
    const bool wide = c.nx > 64 && (tail == 0 || tail > 64);
    wx = wide ? 2 : 1;
    ty = wide ? 4 : 8;
    // the 16-bit formats: 256-wide tiles where the last 256-wide tile of a row is
    // full or more than 160 nodes long (no ring columns loaded from a neighbouring
    // tile of the row: each such node costs 19 cache lines for 76 bytes)
    const int tail256 = c.nx % 256;
    if (valid_tile(c, 4, 4) && c.nx > 128 && (tail256 == 0 || tail256 > 160)) {
        ty = 4;
        wx = 4;
    }
}

// z-chunk of a launch.  FP64 and FP32: two waves per SIMD are resident (the
// register budget): 256 CUs x 4 SIMDs x 2 = 2048 waves = 2048 / (TY WX)
// workgroups at a time.  A workgroup's time grows with its planes plus the two it
// reads beyond its chunk, so the launch takes the chunk count that minimises
// (rounds of resident workgroups) x (planes per chunk + 2): a grid slightly
// larger than the device would otherwise take a second, nearly empty round
// (measured: 160^3 at 5.4 GLUPS with 320 workgroups).  The 16-bit formats: four
// waves per SIMD, and chunks of at most 64 planes (measured with their default
// tiles, us per step at the rule's choice capped at 32 / at 64 planes, FP16:
// 192^3 305-319 / 305, 200^3 352 / 340, 240^3 525 / 506, 256^3 579-583 / 543-547,
// 288^3 1110-1118 / 1081, 64 boxes of 64^3 548 / 552, 8 boxes of 128^3 571-575 /
// 554-559; longer chunks lose: 256^3 in one 256-wide tile per row needs 256
// workgroups of 64 planes to fill the device once).
int default_zchunk(const sclbm_config &c, int ty, int wx) {
    const long tiles = long((c.nx + 64 * wx - 1) / (64 * wx)) * long((c.ny + ty - 1) / ty) * c.nbox;
    const bool dev = is_dev(c.prec);
    const long resident = (dev ? 1024L * kDevWaves : 2048L) / (ty * wx);
    const long zmax = dev ? 64 : c.nz;
    long best_cost = -1, best_zc = std::min<long>(c.nz, zmax);
    for (long nzc = 1; nzc <= std::max(1, c.nz / 2); ++nzc) {
        const long zc = (c.nz + nzc - 1) / nzc;
        if (zc > zmax) continue;
        const long chunks = (c.nz + zc - 1) / zc;
        const long rounds = (tiles * chunks + resident - 1) / resident;
        const long cost = rounds * (zc + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_zc = zc;
        }
    }
    return int(best_zc);
}

// The z-chunk that puts all workgroups of a launch in one round of resident
// workgroups with as many chunks as fit (0 where even whole-box chunks need more
// than one round).  An autotuner candidate: single rounds of long chunks beat the
// rounds rule's split into two rounds for FP32 at some sizes (192^3: 519 against
// 561 us per step with 64-plane chunks on 64 x 8 tiles; 224^3: 799 against 841 us
// with 112-plane chunks on 128 x 4 tiles).
int one_round_zchunk(const sclbm_config &c, int ty, int wx) {
    const long tiles = long((c.nx + 64 * wx - 1) / (64 * wx)) * long((c.ny + ty - 1) / ty) * c.nbox;
    const long resident = (is_dev(c.prec) ? 1024L * kDevWaves : 2048L) / (ty * wx);
    const long nzc = std::min<long>(resident / tiles, c.nz);
    if (nzc < 1) return 0;
    return int((c.nz + nzc - 1) / nzc);
}

// Launch of the step kernel for precision P and a tile of TY rows of WX wavefronts.
template <int P, int TY, int WX>
hipError_t launch_step_tile(sclbm_ctx *c, const StepArgs &a) {
    dim3 block(64 * WX, TY, 1);
    dim3 grid((c->cfg.nx + 64 * WX - 1) / (64 * WX), (c->cfg.ny + TY - 1) / TY, a.nzc * c->cfg.nbox);
    // register budget: two waves per SIMD (up to 256 VGPRs); a tighter budget spills
    constexpr int WAVES = 2;
    if constexpr (Prec<P>::DEV) {
        // the 16-bit formats fit four waves per SIMD (128 VGPRs)
        if (c->cfg.bc == SCLBM_BC_GHOST)
            hipLaunchKernelGGL((k_step_dev<P, TY, WX, true, kDevWaves>), grid, block, 0, c->stream, a);
        else
            hipLaunchKernelGGL((k_step_dev<P, TY, WX, false, kDevWaves>), grid, block, 0, c->stream, a);
    } else {
        if (c->cfg.bc == SCLBM_BC_GHOST)
            hipLaunchKernelGGL((k_step<P, TY, WX, true, WAVES>), grid, block, 0, c->stream, a);
        else
            hipLaunchKernelGGL((k_step<P, TY, WX, false, WAVES>), grid, block, 0, c->stream, a);
    }
    return hipGetLastError();
}

template <int P>
hipError_t launch_step(sclbm_ctx *c, const StepArgs &a) {
    if constexpr (Prec<P>::DEV) {
        if (c->tile_waves == 4) return launch_step_tile<P, 4, 4>(c, a);
    }
    if (c->tile_waves == 2) return launch_step_tile<P, 4, 2>(c, a);
    if (c->tile_rows == 8) return launch_step_tile<P, 8, 1>(c, a);
    return launch_step_tile<P, 4, 1>(c, a);
}

hipError_t launch_step_prec(sclbm_ctx *c, const StepArgs &a) {
    switch (c->cfg.prec) {
        case SCLBM_F64: return launch_step<SCLBM_F64>(c, a);
        case SCLBM_F32: return launch_step<SCLBM_F32>(c, a);
        case SCLBM_F32D: return launch_step<SCLBM_F32D>(c, a);
        case SCLBM_F16DEV: return launch_step<SCLBM_F16DEV>(c, a);
        default: return launch_step<SCLBM_BF16DEV>(c, a);
    }
}

// Dispatch a per-precision functor.
template <typename Fn>
hipError_t by_prec(int prec, Fn &&fn) {
    switch (prec) {
        case SCLBM_F64: return fn(std::integral_constant<int, SCLBM_F64>{});
        case SCLBM_F32: return fn(std::integral_constant<int, SCLBM_F32>{});
        case SCLBM_F32D: return fn(std::integral_constant<int, SCLBM_F32D>{});
        case SCLBM_F16DEV: return fn(std::integral_constant<int, SCLBM_F16DEV>{});
        default: return fn(std::integral_constant<int, SCLBM_BF16DEV>{});
    }
}

unsigned grid1d(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

sclbm_status init_common(sclbm_ctx *c, int32_t box, int mode, const DropletInit &d, const double *ra, const double *rb,
                         const double *u) {
    const int b0 = box < 0 ? 0 : box, b1 = box < 0 ? c->cfg.nbox : box + 1;
    // written into the buffer that holds the current state of every box
    for (int b = b0; b < b1; ++b) {
        hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            using S = typename Prec<P>::S;
            S *f = reinterpret_cast<S *>(c->fbuf(c->par)) + size_t(b) * 2 * Q * size_t(c->N);
            hipLaunchKernelGGL((k_init<P>), dim3(grid1d(c->N, 256)), dim3(256), 0, c->stream, f, c->box_ref(c->par, b),
                               c->geom, mode, d, ra, rb, u);
            return hipGetLastError();
        });
        if (e != hipSuccess) return fail(SCLBM_EHIP, "init kernel: %s", hipGetErrorString(e));
    }
    c->n = 0;
    drop_graph(c);
    int64_t zero[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(c->clock(), zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));  // `zero` is a stack buffer
    return SCLBM_OK;
}

// Largest ghost speed |A (x_g - x_c)| of a gradient over the ghost nodes that
// streaming reads.  |A d| is convex in d, so the maximum over the face and edge
// ghosts is reached at an end point of an edge ghost line: two coordinates in
// {-1, n} and the third in {0, n-1}.
double max_ghost_speed(const sclbm_config &c, const double *A, const double xc[3]) {
    const int n[3] = {c.nx, c.ny, c.nz};
    double best = 0.0;
    for (int free_axis = 0; free_axis < 3; ++free_axis)
        for (int m = 0; m < 8; ++m) {
            double p[3];
            for (int ax = 0, bit = 0; ax < 3; ++ax, ++bit) {
                const int hi = (m >> bit) & 1;
                if (ax == free_axis)
                    p[ax] = hi ? n[ax] - 1 : 0;
                else
                    p[ax] = hi ? n[ax] : -1;
            }
            const double d[3] = {p[0] - xc[0], p[1] - xc[1], p[2] - xc[2]};
            double s = 0.0;
            for (int i = 0; i < 3; ++i) {
                const double v = A[3 * i] * d[0] + A[3 * i + 1] * d[1] + A[3 * i + 2] * d[2];
                s += v * v;
            }
            best = std::max(best, std::sqrt(s));
        }
    return best;
}

// Eigenvalues of a symmetric 3x3 matrix, descending, by the closed-form
// trigonometric solution of the characteristic cubic.
void sym3_eigenvalues(const double m[6] /* xx xy xz yy yz zz */, double out[3]) {
    const double a00 = m[0], a01 = m[1], a02 = m[2], a11 = m[3], a12 = m[4], a22 = m[5];
    const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
    const double q = (a00 + a11 + a22) / 3.0;
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    if (p2 <= 0.0) {
        out[0] = out[1] = out[2] = q;
        return;
    }
    const double p = std::sqrt(p2 / 6.0);
    // det((A - qI)/p) / 2
    const double c00 = b00 / p, c11 = b11 / p, c22 = b22 / p, c01 = a01 / p, c02 = a02 / p, c12 = a12 / p;
    const double det = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
    double r = det / 2.0;
    r = std::max(-1.0, std::min(1.0, r));
    const double phi = std::acos(r) / 3.0;
    const double two_pi_3 = 2.0943951023931954923;
    out[0] = q + 2.0 * p * std::cos(phi);
    out[2] = q + 2.0 * p * std::cos(phi + two_pi_3);
    out[1] = 3.0 * q - out[0] - out[2];
}

template <int K>
sclbm_status reduce_final(sclbm_ctx *c, int nblk, double *host_out) {
    hipLaunchKernelGGL((k_final<K>), dim3(1), dim3(NRED_THREADS), 0, c->stream, c->partial(), nblk, c->result());
    HIP_LAUNCHED();
    HIP_TRY(hipMemcpyAsync(host_out, c->result(), K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

// Launch the FP64 statistics of boxes [b0, b0 + nb) at time n; the final 16
// values of box b0 + i go to c->result() + 16 i (device).
// Partials [box][block][16] go to `partial` (nb * stats_blocks * 16 doubles) and
// the final values to `result` (nb * 16); by default the workspace's areas.
sclbm_status launch_stats(sclbm_ctx *c, int32_t b0, int32_t nb, double *partial, double *result) {
    const int bpb = int(stats_blocks(&c->cfg));
    if (!partial) partial = c->partial();
    if (!result) result = c->result();
    hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using S = typename Prec<P>::S;
        const S *f = reinterpret_cast<const S *>(c->fbuf(c->par));
        hipLaunchKernelGGL((k_stats<P>), dim3(bpb, nb), dim3(NRED_THREADS), 0, c->stream, f, c->refbuf(c->par),
                           c->geom, b0, partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return fail(SCLBM_EHIP, "stats kernel: %s", hipGetErrorString(e));
    hipLaunchKernelGGL((k_final<NSTAT>), dim3(nb), dim3(NRED_THREADS), 0, c->stream, partial, bpb, result);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

// Droplet mass (sum of rho_A where rho_A > rho_B) of boxes [b0, b0 + nb) into c->mass_now() + b0.
sclbm_status launch_drop_mass(sclbm_ctx *c, int32_t b0, int32_t nb) {
    const int bpb = int(stats_blocks(&c->cfg));
    hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using S = typename Prec<P>::S;
        const S *f = reinterpret_cast<const S *>(c->fbuf(c->par));
        hipLaunchKernelGGL((k_drop_mass<P>), dim3(bpb, nb), dim3(NRED_THREADS), 0, c->stream, f, c->refbuf(c->par),
                           c->geom, b0, c->partial());
        return hipGetLastError();
    });
    if (e != hipSuccess) return fail(SCLBM_EHIP, "droplet mass kernel: %s", hipGetErrorString(e));
    hipLaunchKernelGGL((k_final<1>), dim3(nb), dim3(NRED_THREADS), 0, c->stream, c->partial(), bpb, c->mass_now() + b0);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

sclbm_status fields_into(sclbm_ctx *c, int32_t box, double *ra, double *rb, double *u) {
    hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using S = typename Prec<P>::S;
        const S *f = reinterpret_cast<const S *>(c->fbuf(c->par)) + size_t(box) * 2 * Q * size_t(c->N);
        hipLaunchKernelGGL((k_density<P>), dim3(grid1d(c->N, 256)), dim3(256), 0, c->stream, f,
                           c->box_ref(c->par, box), c->geom, ra, rb);
        hipError_t e1 = hipGetLastError();
        if (e1 != hipSuccess || !u) return e1;
        hipLaunchKernelGGL((k_velocity<P>), dim3(grid1d(c->N, 256)), dim3(256), 0, c->stream, f,
                           c->box_ref(c->par, box), c->geom, ra, rb, int(c->cfg.bc == SCLBM_BC_GHOST), c->cfg.g_ab,
                           c->cfg.rho_b[0], c->cfg.rho_b[1], u);
        return hipGetLastError();
    });
    if (e != hipSuccess) return fail(SCLBM_EHIP, "fields kernels: %s", hipGetErrorString(e));
    return SCLBM_OK;
}

}  // namespace

extern "C" {

const char *sclbm_last_error(void) { return g_err.c_str(); }

sclbm_status sclbm_workspace_bytes(const sclbm_config *cfg, size_t *bytes) {
    std::string why;
    if (!bytes) return fail(SCLBM_EINVAL, "null bytes pointer");
    if (!config_ok(cfg, why)) return fail(SCLBM_EINVAL, "invalid config: %s", why.c_str());
    *bytes = make_layout(cfg).total;
    return SCLBM_OK;
}

sclbm_status sclbm_default_launch(const sclbm_config *cfg, int32_t *tile_rows, int32_t *zchunk, int32_t *tile_waves) {
    std::string why;
    if (!config_ok(cfg, why)) return fail(SCLBM_EINVAL, "invalid config: %s", why.c_str());
    int ty = 0, wx = 0;
    default_tile(*cfg, ty, wx);
    if (tile_rows) *tile_rows = ty;
    if (zchunk) *zchunk = default_zchunk(*cfg, ty, wx);
    if (tile_waves) *tile_waves = wx;
    return SCLBM_OK;
}

sclbm_status sclbm_create(const sclbm_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream,
                          sclbm_ctx **out) {
    std::string why;
    if (!out) return fail(SCLBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!config_ok(cfg, why)) return fail(SCLBM_EINVAL, "invalid config: %s", why.c_str());
    const Layout lay = make_layout(cfg);
    if (!dev_workspace) return fail(SCLBM_EINVAL, "null workspace");
    if (bytes < lay.total) return fail(SCLBM_ESIZE, "workspace %zu bytes < required %zu", bytes, lay.total);
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) return fail(SCLBM_ESIZE, "workspace not 256-byte aligned");
    sclbm_ctx *c = new (std::nothrow) sclbm_ctx();
    if (!c) return fail(SCLBM_EINVAL, "host allocation failed");
    c->cfg = *cfg;
    c->lay = lay;
    {
        // the static scratch's address on this device, resolved here with the device current
        double *unused = nullptr;
        sclbm_status st = SCLBM_OK;
        if (hipGetDevice(&c->device) != hipSuccess) st = fail(SCLBM_EHIP, "hipGetDevice failed");
        if (st == SCLBM_OK) st = scratch_address(c->device, &unused);
        if (st != SCLBM_OK) {
            delete c;
            return st;
        }
    }
    c->ws = static_cast<char *>(dev_workspace);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->n = 0;
    c->par = 0;
    default_tile(*cfg, c->tile_rows, c->tile_waves);
    c->zchunk = default_zchunk(*cfg, c->tile_rows, c->tile_waves);
    c->tab_first.assign(cfg->nbox, 0);
    c->tab_len.assign(cfg->nbox, 0);
    c->N = int64_t(cfg->nx) * cfg->ny * cfg->nz;
    c->geom.nx = cfg->nx;
    c->geom.ny = cfg->ny;
    c->geom.nz = cfg->nz;
    c->geom.nnode = c->N;
    c->geom.xc[0] = 0.5 * (cfg->nx - 1);
    c->geom.xc[1] = 0.5 * (cfg->ny - 1);
    c->geom.xc[2] = 0.5 * (cfg->nz - 1);
    std::vector<int64_t> zeros(std::max(2, cfg->nbox), 0);
    hipError_t e = hipMemcpyAsync(c->ws + lay.first, zeros.data(), size_t(cfg->nbox) * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->clock(), zeros.data(), 16, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(SCLBM_EHIP, "create: %s", hipGetErrorString(e));
    }
    *out = c;
    return SCLBM_OK;
}

sclbm_status sclbm_destroy(sclbm_ctx *ctx) {
    if (ctx) drop_graph(ctx);
    delete ctx;
    return SCLBM_OK;
}

sclbm_status sclbm_init_droplet(sclbm_ctx *c, int32_t box, const double center[3], double radius, double width,
                                double rho_in, double rho_out, const double A0[9]) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, true))) return st;
    if (!center) return fail(SCLBM_EINVAL, "null center");
    if (!(width > 0.0) || !(radius >= 0.0)) return fail(SCLBM_EINVAL, "need width > 0 and radius >= 0");
    if (!(rho_in > 0.0) || !(rho_out > 0.0)) return fail(SCLBM_EINVAL, "densities must be positive");
    DropletInit d{};
    for (int k = 0; k < 3; ++k) d.ctr[k] = center[k];
    d.radius = radius;
    d.width = width;
    d.rho_in = rho_in;
    d.rho_out = rho_out;
    for (int k = 0; k < 9; ++k) d.A0.a[k] = A0 ? A0[k] : 0.0;
    return init_common(c, box, 0, d, nullptr, nullptr, nullptr);
}

sclbm_status sclbm_init_fields(sclbm_ctx *c, int32_t box, const double *rho_a, const double *rho_b, const double *u) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!rho_a || !rho_b) return fail(SCLBM_EINVAL, "null density field");
    DropletInit d{};
    return init_common(c, box, 1, d, rho_a, rho_b, u);
}

sclbm_status sclbm_set_gradient_table(sclbm_ctx *c, int32_t box, const double *A, int64_t first_step, int64_t n) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (c->cfg.bc != SCLBM_BC_GHOST) return fail(SCLBM_ESTATE, "gradient table needs the ghost boundary");
    if (!A) return fail(SCLBM_EINVAL, "null table");
    if (n < 1 || n > c->cfg.table_len) return fail(SCLBM_EINVAL, "n=%lld outside [1, table_len=%lld]", (long long)n,
                                                   (long long)c->cfg.table_len);
    if (first_step < 0) return fail(SCLBM_EINVAL, "first_step must be >= 0");
    for (int64_t t = 0; t < n; ++t)
        for (int k = 0; k < 9; ++k)
            if (!std::isfinite(A[9 * t + k])) return fail(SCLBM_EINVAL, "row %lld has a non-finite entry", (long long)t);
    if (c->cfg.mach_max > 0.0) {
        const double vmax = c->cfg.mach_max / std::sqrt(3.0);
        for (int64_t t = 0; t < n; ++t) {
            const double v = max_ghost_speed(c->cfg, A + 9 * t, c->geom.xc);
            if (v > vmax)
                return fail(SCLBM_EINVAL, "row %lld: ghost speed %.6g exceeds mach_max*c_s = %.6g", (long long)t, v, vmax);
        }
    }
    double *dtab = reinterpret_cast<double *>(c->ws + c->lay.atab) + size_t(box) * size_t(c->cfg.table_len) * 9;
    HIP_TRY(hipMemcpyAsync(dtab, A, size_t(n) * 9 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    int64_t *dfirst = reinterpret_cast<int64_t *>(c->ws + c->lay.first) + box;
    HIP_TRY(hipMemcpyAsync(dfirst, &first_step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));  // host sources may be released on return
    c->tab_first[box] = first_step;
    c->tab_len[box] = n;
    return SCLBM_OK;
}

sclbm_status sclbm_init_uniform(sclbm_ctx *c, int32_t box, double rho_a, double rho_b, const double u0[3]) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, true))) return st;
    if (!(rho_a > 0.0) || !(rho_b > 0.0)) return fail(SCLBM_EINVAL, "densities must be positive");
    DropletInit d{};
    d.rho_in = rho_a;
    d.rho_out = rho_b;
    for (int k = 0; k < 3; ++k) {
        d.u0[k] = u0 ? u0[k] : 0.0;
        if (!std::isfinite(d.u0[k])) return fail(SCLBM_EINVAL, "non-finite velocity");
    }
    return init_common(c, box, 2, d, nullptr, nullptr, nullptr);
}

sclbm_status sclbm_set_gradient(sclbm_ctx *c, int32_t box, const double A[9]) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, true))) return st;
    if (!A) return fail(SCLBM_EINVAL, "null gradient");
    const int64_t n = c->cfg.table_len;
    std::vector<double> rows;
    try {
        rows.resize(size_t(n) * 9);
    } catch (const std::bad_alloc &) {
        return fail(SCLBM_EINVAL, "host allocation of %lld rows failed", (long long)n);
    }
    for (int64_t t = 0; t < n; ++t)
        for (int k = 0; k < 9; ++k) rows[size_t(t) * 9 + k] = A[k];
    const int b0 = box < 0 ? 0 : box, b1 = box < 0 ? c->cfg.nbox : box + 1;
    for (int b = b0; b < b1; ++b)
        if ((st = sclbm_set_gradient_table(c, b, rows.data(), c->n, n))) return st;
    return SCLBM_OK;
}

sclbm_status sclbm_set_health_check(sclbm_ctx *c, int64_t every) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (every < 0) return fail(SCLBM_EINVAL, "every must be >= 0");
    c->health_every = every;
    return SCLBM_OK;
}

namespace {

sclbm_status launch_stats(sclbm_ctx *c, int32_t b0, int32_t nb, double *partial, double *result);

// Every box's FP64 totals and count of nodes with a NaN/Inf or non-positive
// density at the current time (synchronises); EUNSTABLE names the first bad box.
sclbm_status health_check(sclbm_ctx *c) {
    sclbm_status st = launch_stats(c, 0, c->cfg.nbox, nullptr, nullptr);
    if (st) return st;
    std::vector<double> r(size_t(c->cfg.nbox) * NSTAT);
    HIP_TRY(hipMemcpyAsync(r.data(), c->result(), r.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->cfg.nbox; ++b) {
        const double *v = r.data() + size_t(b) * NSTAT;
        if (v[15] != 0.0 || !std::isfinite(v[0]) || !std::isfinite(v[1]))
            return fail(SCLBM_EUNSTABLE, "box %d at step %lld: %.0f nodes with NaN/Inf or non-positive density", b,
                        (long long)c->n, v[15]);
    }
    return SCLBM_OK;
}

sclbm_status check_table(sclbm_ctx *c, int64_t nsteps) {
    if (c->cfg.bc != SCLBM_BC_GHOST) return SCLBM_OK;
    for (int b = 0; b < c->cfg.nbox; ++b)
        if (c->n < c->tab_first[b] || c->n + nsteps > c->tab_first[b] + c->tab_len[b])
            return fail(SCLBM_ESTATE, "box %d: gradient table covers steps [%lld, %lld), need [%lld, %lld)", b,
                        (long long)c->tab_first[b], (long long)(c->tab_first[b] + c->tab_len[b]), (long long)c->n,
                        (long long)(c->n + nsteps));
    return SCLBM_OK;
}

StepArgs base_args(sclbm_ctx *c) {
    StepArgs a{};
    a.atab = reinterpret_cast<const double *>(c->ws + c->lay.atab);
    a.tab_first = reinterpret_cast<const int64_t *>(c->ws + c->lay.first);
    a.table_len = c->cfg.table_len;
    a.nnode = c->N;
    a.nx = c->cfg.nx;
    a.ny = c->cfg.ny;
    a.nz = c->cfg.nz;
    a.zchunk = c->zchunk;
    a.nzc = (c->cfg.nz + c->zchunk - 1) / c->zchunk;
    // tile order: x fastest, then y, then z-chunk (groups of one chunk).  Each XCD
    // then takes a run of neighbouring rows of one chunk, whose ring rows it reads
    // from its own L2.  Groups of up to 4 / (x tiles) chunks had been best or within
    // 0.5 % before the ghost faces were balanced; since, single chunks run the 128^3
    // FP32 box 2.5 % faster (126.4-127.9 against 130.5-130.6 us per launch) and
    // every other box measured within 0.5 % (96^3 - 320^3, all formats at 256^3).
    a.zgroup = 1;
    for (int s = 0; s < 2; ++s) {
        a.tau[s] = c->cfg.tau[s];
        a.omega[s] = 1.0 / c->cfg.tau[s];
        a.rho_b[s] = c->cfg.rho_b[s];
    }
    a.g = c->cfg.g_ab;
    for (int k = 0; k < 3; ++k) a.xc[k] = c->geom.xc[k];
    return a;
}

// Enqueue nsteps launches starting from buffer parity `par` (no host state change).
hipError_t enqueue_steps(sclbm_ctx *c, int64_t nsteps, int par) {
    StepArgs a = base_args(c);
    for (int64_t t = 0; t < nsteps; ++t) {
        a.src = c->fbuf(par);
        a.dst = c->fbuf(1 - par);
        a.ref_src = c->refbuf(par);
        a.ref_dst = c->refbuf(1 - par);
        a.clk_in = c->clock() + par;
        a.clk_out = c->clock() + (1 - par);
        hipError_t e = launch_step_prec(c, a);
        if (e != hipSuccess) return e;
        par ^= 1;
    }
    return hipSuccess;
}

void drop_graph(sclbm_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_steps = 0;
    c->graph_par = -1;
}

}  // namespace

sclbm_status sclbm_step(sclbm_ctx *c, int64_t nsteps) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (nsteps < 0) return fail(SCLBM_EINVAL, "nsteps < 0");
    if (nsteps == 0) return SCLBM_OK;
    if ((st = check_table(c, nsteps))) return st;
    // with the health check on, steps go in segments that end where the time is a
    // multiple of health_every, and each such time is checked
    int64_t left = nsteps;
    while (left > 0) {
        int64_t seg = left;
        if (c->health_every > 0) seg = std::min(left, c->health_every - c->n % c->health_every);
        hipError_t e = enqueue_steps(c, seg, c->par);
        if (e != hipSuccess) return fail(SCLBM_EHIP, "step kernel: %s", hipGetErrorString(e));
        c->par ^= int(seg & 1);
        c->n += seg;
        left -= seg;
        if (c->health_every > 0 && c->n % c->health_every == 0 && (st = health_check(c))) return st;
    }
    return SCLBM_OK;
}

sclbm_status sclbm_step_graph(sclbm_ctx *c, int64_t nsteps) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (nsteps < 2 || (nsteps & 1)) return fail(SCLBM_EINVAL, "nsteps must be even and >= 2");
    if ((st = check_table(c, nsteps))) return st;
    if (!c->graph_exec || c->graph_steps != nsteps || c->graph_par != c->par || c->graph_ty != c->tile_rows ||
        c->graph_wx != c->tile_waves || c->graph_zc != c->zchunk) {
        drop_graph(c);
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_steps(c, nsteps, c->par);
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(SCLBM_EHIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph_exec = nullptr;
            return fail(SCLBM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        c->graph_steps = nsteps;
        c->graph_par = c->par;
        c->graph_ty = c->tile_rows;
        c->graph_wx = c->tile_waves;
        c->graph_zc = c->zchunk;
    }
    HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
    c->n += nsteps;  // even: the parity is unchanged
    if (c->health_every > 0) return health_check(c);  // once, after the replay
    return SCLBM_OK;
}

sclbm_status sclbm_autotune(sclbm_ctx *c, int32_t trial_steps, int32_t *tile_rows, int32_t *zchunk,
                            int32_t *tile_waves, float *best_ms) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (trial_steps < 1 || trial_steps > 100000) return fail(SCLBM_EINVAL, "trial_steps must be in [1, 100000]");
    if ((st = check_table(c, int64_t(trial_steps) + 1))) return st;
    const int ty_keep = c->tile_rows, wx_keep = c->tile_waves, zc_keep = c->zchunk;
    const int64_t n0 = c->n;
    const int par0 = c->par;
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    float best = -1.0f;
    int bty = ty_keep, bwx = wx_keep, bzc = zc_keep;
    // candidates: every valid tile with z-chunks 2 .. 64 (capped at nz), the
    // tile's default z-chunk, so that the default launch is always among them,
    // and the chunk that fills the device in one round
    const int tys[4] = {4, 8, 4, 4}, wxs[4] = {1, 1, 2, 4};
    const int zcs[6] = {2, 4, 8, 16, 32, 64};
    std::vector<std::array<int, 3>> cand;
    for (int ti = 0; ti < 4; ++ti) {
        if (!valid_tile(c->cfg, tys[ti], wxs[ti])) continue;
        if (c->cfg.nx <= 64 * (wxs[ti] / 2)) continue;  // the tile's last column would hold no nodes
        std::vector<int> zl;
        for (int zc : zcs) zl.push_back(std::min(zc, c->cfg.nz));
        zl.push_back(default_zchunk(c->cfg, tys[ti], wxs[ti]));
        if (const int z1 = one_round_zchunk(c->cfg, tys[ti], wxs[ti])) zl.push_back(z1);
        std::sort(zl.begin(), zl.end());
        zl.erase(std::unique(zl.begin(), zl.end()), zl.end());
        for (int zc : zl) cand.push_back({tys[ti], wxs[ti], zc});
    }
    sclbm_status result = SCLBM_OK;
    for (size_t ci = 0; ci < cand.size() && result == SCLBM_OK; ++ci) {
        c->tile_rows = cand[ci][0];
        c->tile_waves = cand[ci][1];
        c->zchunk = cand[ci][2];
        int64_t clk[2] = {n0, n0};
        hipError_t e = hipMemcpyAsync(c->clock(), clk, sizeof clk, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = enqueue_steps(c, 1, par0 ^ 0);  // warm-up (reads row n0)
        if (e == hipSuccess) e = hipMemcpyAsync(c->clock(), clk, sizeof clk, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev0, c->stream);
        if (e == hipSuccess) e = enqueue_steps(c, trial_steps, par0);
        if (e == hipSuccess) e = hipEventRecord(ev1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
        if (e != hipSuccess) {
            result = fail(SCLBM_EHIP, "autotune: %s", hipGetErrorString(e));
            break;
        }
        ms /= float(trial_steps);
        if (best < 0.0f || ms < best) {
            best = ms;
            bty = c->tile_rows;
            bwx = c->tile_waves;
            bzc = c->zchunk;
        }
    }
    (void)hipEventDestroy(ev0);  // teardown: nothing to do on failure
    (void)hipEventDestroy(ev1);
    // restore the time; the populations hold trial results
    int64_t clk[2] = {n0, n0};
    HIP_TRY(hipMemcpyAsync(c->clock(), clk, sizeof clk, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->n = n0;
    c->par = par0;
    if (result != SCLBM_OK) {
        c->tile_rows = ty_keep;
        c->tile_waves = wx_keep;
        c->zchunk = zc_keep;
        return result;
    }
    c->tile_rows = bty;
    c->tile_waves = bwx;
    c->zchunk = bzc;
    drop_graph(c);
    if (tile_rows) *tile_rows = bty;
    if (zchunk) *zchunk = bzc;
    if (tile_waves) *tile_waves = bwx;
    if (best_ms) *best_ms = best;
    return SCLBM_OK;
}

sclbm_status sclbm_get_step(const sclbm_ctx *c, int64_t *step) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!step) return fail(SCLBM_EINVAL, "null step pointer");
    *step = c->n;
    return SCLBM_OK;
}

sclbm_status sclbm_fields(sclbm_ctx *c, int32_t box, double *rho_a, double *rho_b, double *u) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!rho_a || !rho_b) return fail(SCLBM_EINVAL, "rho_a and rho_b must not be NULL");
    return fields_into(c, box, rho_a, rho_b, u);
}

sclbm_status sclbm_totals(sclbm_ctx *c, int32_t box, double mass[2], double momentum[3]) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!mass || !momentum) return fail(SCLBM_EINVAL, "null output");
    if ((st = launch_stats(c, box, 1, nullptr, nullptr))) return st;
    double r[NSTAT];
    HIP_TRY(hipMemcpyAsync(r, c->result(), sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    mass[0] = r[0];
    mass[1] = r[1];
    momentum[0] = r[2];
    momentum[1] = r[3];
    momentum[2] = r[4];
    if (r[15] != 0.0) return fail(SCLBM_EUNSTABLE, "%.0f nodes with NaN/Inf or non-positive density", r[15]);
    return SCLBM_OK;
}

sclbm_status sclbm_droplet_moments(sclbm_ctx *c, int32_t box, double *dev_out10) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!dev_out10) return fail(SCLBM_EINVAL, "null output");
    if ((st = launch_stats(c, box, 1, nullptr, nullptr))) return st;
    HIP_TRY(hipMemcpyAsync(dev_out10, c->result() + 5, 10 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_droplet_moments_all(sclbm_ctx *c, double *dev_out) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!dev_out) return fail(SCLBM_EINVAL, "null output");
    if ((st = launch_stats(c, 0, c->cfg.nbox, nullptr, nullptr))) return st;
    HIP_TRY(hipMemcpy2DAsync(dev_out, 10 * sizeof(double), c->result() + 5, NSTAT * sizeof(double), 10 * sizeof(double),
                             size_t(c->cfg.nbox), hipMemcpyDeviceToDevice, c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_droplet_moments_all_static(sclbm_ctx *c, double *dev_out) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!dev_out) return fail(SCLBM_EINVAL, "null output");
    const size_t nb = size_t(c->cfg.nbox), bpb = stats_blocks(&c->cfg);
    const size_t need = nb * (bpb + 1) * NSTAT;
    if (need > kScratchDoubles)
        return fail(SCLBM_ESIZE, "%zu boxes need %zu doubles of static scratch; it holds %zu (%zu boxes of this size)",
                    nb, need, kScratchDoubles, kScratchDoubles / ((bpb + 1) * NSTAT));
    double *s = nullptr;
    if ((st = scratch_address(c->device, &s))) return st;
    // every partial and result slot read below is written first by this call's kernels
    double *partial = s, *result = s + nb * bpb * NSTAT;
    if ((st = launch_stats(c, 0, c->cfg.nbox, partial, result))) return st;
    HIP_TRY(hipMemcpy2DAsync(dev_out, 10 * sizeof(double), result + 5, NSTAT * sizeof(double), 10 * sizeof(double),
                             nb, hipMemcpyDeviceToDevice, c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_droplet_from_moments(const double mom[10], const double center[3], int64_t step,
                                        sclbm_droplet_stats *out) {
    if (!mom || !center || !out) return fail(SCLBM_EINVAL, "null argument");
    std::memset(out, 0, sizeof *out);
    out->step = step;
    const double S0 = mom[0];
    out->volume = S0;
    if (!(S0 > 0.0)) {
        for (int k = 0; k < 3; ++k) out->com[k] = center[k];
        return SCLBM_OK;
    }
    const double m1[3] = {mom[1] / S0, mom[2] / S0, mom[3] / S0};
    for (int k = 0; k < 3; ++k) out->com[k] = center[k] + m1[k];
    // S2 about the centre -> covariance about the centre of mass
    out->cov[0] = mom[4] / S0 - m1[0] * m1[0];
    out->cov[1] = mom[5] / S0 - m1[0] * m1[1];
    out->cov[2] = mom[6] / S0 - m1[0] * m1[2];
    out->cov[3] = mom[7] / S0 - m1[1] * m1[1];
    out->cov[4] = mom[8] / S0 - m1[1] * m1[2];
    out->cov[5] = mom[9] / S0 - m1[2] * m1[2];
    double lam[3];
    sym3_eigenvalues(out->cov, lam);
    for (int k = 0; k < 3; ++k) out->semi_axes[k] = std::sqrt(5.0 * std::max(0.0, lam[k]));
    const double s = out->semi_axes[0] + out->semi_axes[2];
    out->deformation = s > 0.0 ? (out->semi_axes[0] - out->semi_axes[2]) / s : 0.0;
    out->r_eq = std::cbrt(3.0 * S0 / (4.0 * M_PI));
    return SCLBM_OK;
}

sclbm_status sclbm_mm_semi_axes(const double *M, int64_t n, double *axes) {
    if (!M || !axes) return fail(SCLBM_EINVAL, "null argument");
    if (n < 0) return fail(SCLBM_EINVAL, "n must be >= 0");
    for (int64_t t = 0; t < n; ++t) {
        const double *m = M + 9 * t;
        // symmetric part (the integrator keeps M symmetric up to rounding)
        const double c00 = m[0], c11 = m[4], c22 = m[8];
        const double c01 = 0.5 * (m[1] + m[3]), c02 = 0.5 * (m[2] + m[6]), c12 = 0.5 * (m[5] + m[7]);
        const double sm[6] = {c00, c01, c02, c11, c12, c22};
        double lam[3];
        sym3_eigenvalues(sm, lam);
        for (int k = 0; k < 3; ++k) axes[3 * t + k] = std::sqrt(std::max(0.0, lam[k]));
    }
    return SCLBM_OK;
}

sclbm_status sclbm_droplet(sclbm_ctx *c, int32_t box, sclbm_droplet_stats *out) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!out) return fail(SCLBM_EINVAL, "null output");
    if ((st = launch_stats(c, box, 1, nullptr, nullptr))) return st;
    double r[NSTAT];
    HIP_TRY(hipMemcpyAsync(r, c->result(), sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return sclbm_droplet_from_moments(r + 5, c->geom.xc, c->n, out);
}

sclbm_status sclbm_droplet_surface_all(sclbm_ctx *c, double *dev_out) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!dev_out) return fail(SCLBM_EINVAL, "null output");
    const int ntx = (c->cfg.nx - 1 + SURF_T - 1) / SURF_T, nty = (c->cfg.ny - 1 + SURF_T - 1) / SURF_T;
    const int ntiles = ntx * nty;
    // at most 8 stats blocks' worth of partials per box (2 values each instead of 16)
    const int nblk = std::min<int>(ntiles, int(8 * stats_blocks(&c->cfg)));
    hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using S = typename Prec<P>::S;
        const S *f = reinterpret_cast<const S *>(c->fbuf(c->par));
        hipLaunchKernelGGL((k_surface<P>), dim3(nblk, c->cfg.nbox), dim3(NRED_THREADS), 0, c->stream, f,
                           c->refbuf(c->par), c->geom, 0, ntx, ntiles, c->partial());
        return hipGetLastError();
    });
    if (e != hipSuccess) return fail(SCLBM_EHIP, "surface kernel: %s", hipGetErrorString(e));
    hipLaunchKernelGGL((k_final<2>), dim3(c->cfg.nbox), dim3(NRED_THREADS), 0, c->stream, c->partial(), nblk, dev_out);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

sclbm_status sclbm_deformation_lbm(double area, double volume, double *d_lbm) {
    if (!d_lbm) return fail(SCLBM_EINVAL, "null output");
    if (!(area > 0.0) || !(volume >= 0.0)) return fail(SCLBM_EINVAL, "area must be positive, volume non-negative");
    const double omega0 = std::cbrt(36.0 * M_PI * volume * volume);
    *d_lbm = std::sqrt(std::max(0.0, 1.0 - omega0 / area));
    return SCLBM_OK;
}

sclbm_status sclbm_droplet_mass_all(sclbm_ctx *c, double *dev_out) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!dev_out) return fail(SCLBM_EINVAL, "null output");
    if ((st = launch_drop_mass(c, 0, c->cfg.nbox))) return st;
    HIP_TRY(hipMemcpyAsync(dev_out, c->mass_now(), size_t(c->cfg.nbox) * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_reinject(sclbm_ctx *c, int32_t box, const double *target_mass) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, true))) return st;
    if (!target_mass) return fail(SCLBM_EINVAL, "null target");
    const int32_t b0 = box < 0 ? 0 : box, nb = box < 0 ? c->cfg.nbox : 1;
    for (int32_t i = 0; i < nb; ++i)
        if (!(target_mass[i] > 0.0) || !std::isfinite(target_mass[i]))
            return fail(SCLBM_EINVAL, "target mass %d must be positive and finite", i);
    HIP_TRY(hipMemcpyAsync(c->mass_target() + b0, target_mass, size_t(nb) * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    if ((st = launch_drop_mass(c, b0, nb))) return st;
    hipError_t e = by_prec(c->cfg.prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using S = typename Prec<P>::S;
        S *f = reinterpret_cast<S *>(c->fbuf(c->par));
        const unsigned blocks = std::min<unsigned>(grid1d(c->N, 256), 2048u);
        hipLaunchKernelGGL((k_reinject<P>), dim3(blocks, nb), dim3(256), 0, c->stream, f, c->refbuf(c->par), c->geom,
                           b0, c->mass_now(), c->mass_target());
        return hipGetLastError();
    });
    if (e != hipSuccess) return fail(SCLBM_EHIP, "reinjection kernel: %s", hipGetErrorString(e));
    // the host copy of the target must outlive the transfer
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_velocity_error(sclbm_ctx *c, int32_t box, const double A[9], double *e0) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if ((st = check_box(c, box, false))) return st;
    if (!A || !e0) return fail(SCLBM_EINVAL, "null argument");
    double *d = c->diag();
    if ((st = fields_into(c, box, d, d + c->N, d + 2 * c->N))) return st;
    Mat3 m;
    for (int k = 0; k < 9; ++k) m.a[k] = A[k];
    hipLaunchKernelGGL(k_e0, dim3(NRED_BLOCKS), dim3(NRED_THREADS), 0, c->stream, d + 2 * c->N, c->geom, m,
                       c->partial());
    HIP_LAUNCHED();
    double r[2];
    if ((st = reduce_final<2>(c, NRED_BLOCKS, r))) return st;
    if (!(r[1] > 0.0)) return fail(SCLBM_EINVAL, "the imposed flow is zero on this box");
    *e0 = std::sqrt(r[0]) / std::sqrt(r[1]);
    return SCLBM_OK;
}

sclbm_status sclbm_mm_integrate(const double *dev_A, int64_t ntraj, int64_t nrows, double tau_d, double chi,
                                int32_t substeps, int32_t record_every, const double *dev_M0, double *dev_M,
                                void *hip_stream) {
    if (!dev_A || !dev_M) return fail(SCLBM_EINVAL, "null table or output");
    if (ntraj < 1 || nrows < 1) return fail(SCLBM_EINVAL, "need ntraj >= 1 and nrows >= 1");
    if (!(tau_d > 0.0) || !(chi > 0.0)) return fail(SCLBM_EINVAL, "need tau_d > 0 and chi > 0");
    if (substeps < 1 || record_every < 1) return fail(SCLBM_EINVAL, "need substeps >= 1 and record_every >= 1");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_mm, dim3(unsigned((ntraj + 63) / 64)), dim3(64), 0, s, dev_A, ntraj, nrows, tau_d, chi,
                       int(substeps), int(record_every), dev_M0, dev_M);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

sclbm_status sclbm_state_bytes(const sclbm_ctx *c, size_t *bytes) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!bytes) return fail(SCLBM_EINVAL, "null bytes pointer");
    *bytes = 64 + c->lay.fbytes + c->lay.refbytes;
    return SCLBM_OK;
}

namespace {
struct CkptHeader {
    char magic[8];
    int64_t n;
    int32_t nx, ny, nz, nbox, prec, bc;
    int64_t fbytes;
};
static_assert(sizeof(CkptHeader) <= 64, "header");
}  // namespace

sclbm_status sclbm_save(sclbm_ctx *c, void *host_buf, size_t bytes) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!host_buf) return fail(SCLBM_EINVAL, "null buffer");
    const size_t need = 64 + c->lay.fbytes + c->lay.refbytes;
    if (bytes < need) return fail(SCLBM_ESIZE, "buffer %zu < %zu", bytes, need);
    CkptHeader h{};
    std::memcpy(h.magic, "SCLBMCK1", 8);
    h.n = c->n;
    h.nx = c->cfg.nx;
    h.ny = c->cfg.ny;
    h.nz = c->cfg.nz;
    h.nbox = c->cfg.nbox;
    h.prec = c->cfg.prec;
    h.bc = c->cfg.bc;
    h.fbytes = int64_t(c->lay.fbytes);
    std::memset(host_buf, 0, 64);
    std::memcpy(host_buf, &h, sizeof h);
    HIP_TRY(hipMemcpyAsync(static_cast<char *>(host_buf) + 64, c->fbuf(c->par), c->lay.fbytes, hipMemcpyDeviceToHost,
                           c->stream));
    if (c->lay.refbytes)
        HIP_TRY(hipMemcpyAsync(static_cast<char *>(host_buf) + 64 + c->lay.fbytes, c->refbuf(c->par), c->lay.refbytes,
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

sclbm_status sclbm_load(sclbm_ctx *c, const void *host_buf, size_t bytes) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!host_buf) return fail(SCLBM_EINVAL, "null buffer");
    if (bytes < 64) return fail(SCLBM_ESIZE, "buffer too small");
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof h);
    if (std::memcmp(h.magic, "SCLBMCK1", 8) != 0) return fail(SCLBM_EINVAL, "not a checkpoint");
    if (h.nx != c->cfg.nx || h.ny != c->cfg.ny || h.nz != c->cfg.nz || h.nbox != c->cfg.nbox ||
        h.prec != c->cfg.prec || h.bc != c->cfg.bc || h.fbytes != int64_t(c->lay.fbytes))
        return fail(SCLBM_EINVAL, "checkpoint was written for a different configuration");
    if (bytes < 64 + c->lay.fbytes + c->lay.refbytes) return fail(SCLBM_ESIZE, "buffer truncated");
    HIP_TRY(hipMemcpyAsync(c->fbuf(0), static_cast<const char *>(host_buf) + 64, c->lay.fbytes, hipMemcpyHostToDevice,
                           c->stream));
    if (c->lay.refbytes)
        HIP_TRY(hipMemcpyAsync(c->refbuf(0), static_cast<const char *>(host_buf) + 64 + c->lay.fbytes, c->lay.refbytes,
                               hipMemcpyHostToDevice, c->stream));
    int64_t clk[2] = {h.n, h.n};
    HIP_TRY(hipMemcpyAsync(c->clock(), clk, sizeof clk, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->par = 0;
    c->n = h.n;
    drop_graph(c);
    return SCLBM_OK;
}

sclbm_status sclbm_set_launch(sclbm_ctx *c, int32_t tile_rows, int32_t zchunk, int32_t tile_waves) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (!valid_tile(c->cfg, tile_rows, tile_waves))
        return fail(SCLBM_EINVAL,
                    "tile (rows %d, waves %d) must be (4, 1), (8, 1), (4, 2), or (4, 4) with a 16-bit format",
                    tile_rows, tile_waves);
    if (zchunk < 1) return fail(SCLBM_EINVAL, "zchunk must be >= 1");
    c->tile_rows = tile_rows;
    c->tile_waves = tile_waves;
    c->zchunk = std::min<int32_t>(zchunk, c->cfg.nz);
    drop_graph(c);
    return SCLBM_OK;
}

sclbm_status sclbm_get_launch(const sclbm_ctx *c, int32_t *tile_rows, int32_t *zchunk, int32_t *tile_waves) {
    sclbm_status st = check_ctx(c);
    if (st) return st;
    if (tile_rows) *tile_rows = c->tile_rows;
    if (zchunk) *zchunk = c->zchunk;
    if (tile_waves) *tile_waves = c->tile_waves;
    return SCLBM_OK;
}

}  // extern "C"
