// Kernels of the droplet-shape surrogate: a 576 -> 512 -> 512 -> 512 -> 3 ReLU
// perceptron from a window of the velocity-gradient history (64 samples of A(t),
// Sec. 3) to the droplet's three semi-axes (Sec. 2 Eq. 4 takes D from them).
//
// Arithmetic: BF16 operands, FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16), FP32 biases, FP32 master weights and Adam moments.
// Every product is "NT": C[m][n] = sum_k A[m][k] B[n][k] with both operands
// contiguous in k, so each lane's MFMA fragment is one 16-byte load.  The
// forward pass writes every hidden activation twice, [batch][unit] for the next
// layer's product and [unit][batch] for the weight gradient's product (whose
// contraction runs over the batch); the backward pass does the same for the
// pre-activation gradients, and Adam keeps a transposed BF16 copy of the hidden
// weights for the input-gradient products.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sclmlp {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NIN = 576;    // 64 samples x 9 gradient entries
constexpr int NHID = 512;
constexpr int NOUT = 3;
constexpr int NLAYER = 4;
constexpr int ROW_ALIGN = 128;  // the batch is padded to this many rows inside the library

// flat FP32 parameter vector: W1 [512][576], b1, W2 [512][512], b2, W3, b3, W4 [3][512], b4
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NHID * NIN;
constexpr int OFF_W2 = OFF_B1 + NHID;
constexpr int OFF_B2 = OFF_W2 + NHID * NHID;
constexpr int OFF_W3 = OFF_B2 + NHID;
constexpr int OFF_B3 = OFF_W3 + NHID * NHID;
constexpr int OFF_W4 = OFF_B3 + NHID;
constexpr int OFF_B4 = OFF_W4 + NOUT * NHID;
constexpr int NPARAM = OFF_B4 + NOUT;
static_assert(NPARAM == 822275, "parameter count");

// ---------------------------------------------------------------------------------------------
// GEMM: C = A B^T with an epilogue.  A [M][K] (row stride lda), B [N][K] (ldb), K % 8 == 0.
// K is staged through LDS BK columns at a time (k beyond K reads as zero); deep stages keep
// many loads in flight per workgroup, which the short contractions here need to hide HBM latency.
enum Epi { EPI_RELU = 0, EPI_MASK = 1, EPI_F32 = 2 };

struct GemmArgs {
    const bf16 *A, *B;
    int M, N, K, lda, ldb;
    // AF32 form: A is FP32 (Af, row stride lda), normalised on the fly as (a - ashift[k]) * ascale[k]
    // and rounded to BF16 while staged; rows >= arows read as zero.
    const float *Af, *ashift, *ascale;
    int arows;
    const float *bias;   // EPI_RELU: per column n
    const bf16 *mask;    // EPI_MASK: element (m, n) kept where mask > 0 (row stride ldmask)
    int ldmask;
    void *C;             // bf16 (RELU, MASK; may be null) or float (F32), row stride ldc
    int ldc;
    bf16 *CT;            // optional transposed bf16 copy, CT[n][m], row stride ldct
    int ldct;
};

__device__ __forceinline__ uint4 ld16(const bf16 *p) { return *reinterpret_cast<const uint4 *>(p); }

template <int BM, int BN, int BK, int EPI, bool AF32 = false>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g) {
    constexpr int LDK = BK + 8;            // 16-byte pad per LDS row spreads the fragment reads over banks
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int RC = BK / 8;             // 16-byte chunks per tile row
    constexpr int CA = BM * RC / 256, CB = BN * RC / 256;
    static_assert(BK % 64 == 0 && (BM * RC) % 256 == 0 && (BN * RC) % 256 == 0, "tile");
    static_assert(FM >= 1 && FN >= 1 && CA >= 1 && CB >= 1, "tile");
    // one LDS buffer: the A and B stages during the contraction, then the BF16 output tile
    constexpr int LDC = BN + 8;
    constexpr int SMEM = (BM + BN) * LDK > BM * LDC ? (BM + BN) * LDK : BM * LDC;
    __shared__ __attribute__((aligned(16))) bf16 smem[SMEM];
    bf16 *const As = smem;
    bf16 *const Bs = smem + BM * LDK;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // XCD-aware order: consecutive workgroups go round-robin over the 8 XCDs; renumber so
    // that the column tiles of one row tile share an XCD (and its L2 copy of the A rows).
    const int ntn = gridDim.x, total = gridDim.x * gridDim.y;
    int lin = blockIdx.y * ntn + blockIdx.x;
    if ((total & 7) == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
    const int m0 = (lin / ntn) * BM, n0 = (lin % ntn) * BN;

    uint4 ra[CA], rb[CB];
    float4 fa[CA][2];  // AF32: raw FP32 A chunks, normalised and converted when staged
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i, r = c / RC, kc = (c % RC) * 8;
            if (AF32) {
                const bool live = m0 + r < g.arows && k0 + kc < g.K;
                const float4 *src =
                    reinterpret_cast<const float4 *>(g.Af + (live ? (size_t)(m0 + r) * g.lda + k0 + kc : 0));
                fa[i][0] = live ? src[0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                fa[i][1] = live ? src[1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                ra[i] = (m0 + r < g.M && k0 + kc < g.K) ? ld16(g.A + (size_t)(m0 + r) * g.lda + k0 + kc)
                                                         : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i, r = c / RC, kc = (c % RC) * 8;
            rb[i] = (n0 + r < g.N && k0 + kc < g.K) ? ld16(g.B + (size_t)(n0 + r) * g.ldb + k0 + kc)
                                                     : make_uint4(0, 0, 0, 0);
        }
    };
    auto sstore = [&](int k0) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i, r = c / RC, kc = (c % RC) * 8;
            if (AF32) {
                const int kq = k0 + kc < g.K ? k0 + kc : 0;
                const float4 sa = *reinterpret_cast<const float4 *>(g.ashift + kq);
                const float4 sb = *reinterpret_cast<const float4 *>(g.ashift + kq + 4);
                const float4 ca = *reinterpret_cast<const float4 *>(g.ascale + kq);
                const float4 cb = *reinterpret_cast<const float4 *>(g.ascale + kq + 4);
                bf16x8 h;
                h[0] = (bf16)((fa[i][0].x - sa.x) * ca.x);
                h[1] = (bf16)((fa[i][0].y - sa.y) * ca.y);
                h[2] = (bf16)((fa[i][0].z - sa.z) * ca.z);
                h[3] = (bf16)((fa[i][0].w - sa.w) * ca.w);
                h[4] = (bf16)((fa[i][1].x - sb.x) * cb.x);
                h[5] = (bf16)((fa[i][1].y - sb.y) * cb.y);
                h[6] = (bf16)((fa[i][1].z - sb.z) * cb.z);
                h[7] = (bf16)((fa[i][1].w - sb.w) * cb.w);
                if (m0 + r >= g.arows || k0 + kc >= g.K) h = bf16x8{};
                *reinterpret_cast<bf16x8 *>(As + r * LDK + kc) = h;
            } else {
                *reinterpret_cast<uint4 *>(As + r * LDK + kc) = ra[i];
            }
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i;
            *reinterpret_cast<uint4 *>(Bs + (c / RC) * LDK + (c % RC) * 8) = rb[i];
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
        for (int s = 0; s < BK / 16; ++s) {
            bf16x8 a[FM], b[FN];
            const int kk = s * 16 + (lane >> 5) * 8;
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * WM + i * 32 + (lane & 31)) * LDK + kk);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * WN + j * 32 + (lane & 31)) * LDK + kk);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            __syncthreads();
            sstore((kt + 1) * BK);
            __syncthreads();
        }
    }

    // accumulator element 4q + j of a 32x32 fragment sits at row 8q + 4 (lane / 32) + j, column lane % 32
    if (EPI == EPI_F32) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = n0 + wn * WN + j * 32 + (lane & 31);
                if (col >= g.N) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row0 = m0 + wm * WM + i * 32 + 8 * q + 4 * (lane >> 5);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (row0 + e < g.M)
                            static_cast<float *>(g.C)[(size_t)(row0 + e) * g.ldc + col] = acc[i][j][4 * q + e];
                }
            }
        return;
    }
    // BF16 outputs: bias + ReLU or the ReLU mask, into an LDS tile, then 16-byte rows to memory
    __syncthreads();  // every wave is done with the A and B stages
    bf16 *const Cs = smem;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int cl = wn * WN + j * 32 + (lane & 31), col = n0 + cl;
            const float bias = (EPI == EPI_RELU && col < g.N) ? g.bias[col] : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rl = wm * WM + i * 32 + 8 * q + 4 * (lane >> 5);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[i][j][4 * q + e];
                    if (EPI == EPI_RELU) v = fmaxf(v + bias, 0.0f);
                    if (EPI == EPI_MASK) {
                        const int row = m0 + rl + e;
                        v = (row < g.M && col < g.N && (float)g.mask[(size_t)row * g.ldmask + col] > 0.0f) ? v : 0.0f;
                    }
                    Cs[(rl + e) * LDC + cl] = (bf16)v;
                }
            }
        }
    __syncthreads();
    if (g.C) {
        bf16 *C = static_cast<bf16 *>(g.C);
        for (int c = tid; c < BM * BN / 8; c += 256) {
            const int r = c / (BN / 8), cc = (c % (BN / 8)) * 8;
            const int row = m0 + r, col = n0 + cc;
            if (row >= g.M) continue;
            if (col + 8 <= g.N) {
                *reinterpret_cast<uint4 *>(C + (size_t)row * g.ldc + col) = *reinterpret_cast<const uint4 *>(Cs + r * LDC + cc);
            } else {
                for (int e = 0; e < 8 && col + e < g.N; ++e) C[(size_t)row * g.ldc + col + e] = Cs[r * LDC + cc + e];
            }
        }
    }
    if (g.CT) {
        for (int c = tid; c < BM * BN / 8; c += 256) {
            const int r = c / (BM / 8), mm = (c % (BM / 8)) * 8;  // r: column of the tile, mm: first row
            const int col = n0 + r, row0 = m0 + mm;
            if (col >= g.N) continue;
            bf16x8 h;
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = Cs[(mm + e) * LDC + r];
            bf16 *dst = g.CT + (size_t)col * g.ldct + row0;
            if (row0 + 8 <= g.M) {
                *reinterpret_cast<bf16x8 *>(dst) = h;
            } else {
                for (int e = 0; e < 8 && row0 + e < g.M; ++e) dst[e] = h[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Input preparation: gather (optional index), optional cubic symmetry of the box, normalise,
// round to BF16; rows >= n are zero.  Tiles of 64 rows x 64 features, grid (NIN / 64, Mpad / 64).
// A row whose index (or symmetry id) is out of range is treated as padding and counted in *bad.
//
// Symmetry id s in [0, 48): P = signed permutation with P[i][perm(i)] = sign(i), perm the
// (s / 8)-th permutation of (0, 1, 2) in lexicographic order, sign(i) = -1 where bit i of s % 8
// is set.  Every sample A of the window becomes P A P^T:  A'_ij = sign(i) sign(j) A_{perm(i) perm(j)}.
__device__ __forceinline__ int sym_source(int s, int e, float &sgn) {
    // e = 3 i + j within one 3 x 3 sample
    const int i = e / 3, j = e - 3 * i;
    const int pi = s >> 3;                       // 012 021 102 120 201 210
    const int p0 = pi < 2 ? 0 : (pi < 4 ? 1 : 2);
    const int p1 = (pi == 0 || pi == 5) ? 1 : ((pi == 1 || pi == 3) ? 2 : 0);
    const int p2 = 3 - p0 - p1;
    const int qi = i == 0 ? p0 : (i == 1 ? p1 : p2);
    const int qj = j == 0 ? p0 : (j == 1 ? p1 : p2);
    sgn = (((s >> i) ^ (s >> j)) & 1) ? -1.0f : 1.0f;
    return 3 * qi + qj;
}

template <bool TRANSPOSED>
__global__ __launch_bounds__(256) void k_prep(const float *win, const int32_t *index, const int32_t *sym, int n,
                                              int ndata, const float *shift, const float *scale, bf16 *X, bf16 *XT,
                                              int Mpad, unsigned *bad) {
    __shared__ bf16 tile[64][66];
    const int c0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = c0 + tx;
    const int t9 = c / 9, e = c - 9 * t9;
    const float sh = shift[c], sc = scale[c];
    for (int r = ty; r < 64; r += 4) {
        const int m = m0 + r;
        float v = 0.0f;
        if (m < n) {
            const int64_t src = index ? (int64_t)index[m] : (int64_t)m;
            const int s = sym ? sym[m] : 0;
            if (src >= 0 && src < ndata && s >= 0 && s < 48) {
                float sgn = 1.0f;
                const int f = s ? 9 * t9 + sym_source(s, e, sgn) : c;
                v = (win[src * NIN + f] * sgn - sh) * sc;
            } else if (tx == 0 && blockIdx.x == 0) {
                atomicAdd(bad, 1u);
            }
        }
        const bf16 b = (bf16)v;
        X[(size_t)m * NIN + c] = b;
        if (TRANSPOSED) tile[r][tx] = b;
    }
    if (TRANSPOSED) {
        __syncthreads();
        for (int r = ty; r < 64; r += 4) XT[(size_t)(c0 + r) * Mpad + m0 + tx] = tile[tx][r];
    }
}

// ---------------------------------------------------------------------------------------------
// Output layer (3 units, no activation): one wave per row, each lane 8 of the 512 inputs.
// PREDICT: writes de-normalised semi-axes for rows < n.  Training: writes dY = 2 (y - t) / (3 n)
// (zero on padding rows) and per-block sums of (y - t)^2 and of dY.  OUT_ROWS rows per block
// (two per wave: few dependent loads per wave, many blocks in flight).
constexpr int OUT_ROWS = 8;
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool PREDICT>
__global__ __launch_bounds__(256) void k_out(const bf16 *H, const bf16 *W4, const float *b4, int n, const float *oshift,
                                             const float *oscale, float *out, const float *targets,
                                             const int32_t *index, const int32_t *sym, int ndata, float *dY,
                                             double *partial) {
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float w[NOUT][8];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(W4 + j * NHID + lane * 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) w[j][e] = (float)v[e];
    }
    double loss = 0.0, db[NOUT] = {0.0, 0.0, 0.0};
    const float inv = n > 0 ? 2.0f / (3.0f * (float)n) : 0.0f;
    for (int r = 0; r < OUT_ROWS / 4; ++r) {
        const int m = blockIdx.x * OUT_ROWS + wave * (OUT_ROWS / 4) + r;
        const bf16x8 h = *reinterpret_cast<const bf16x8 *>(H + (size_t)m * NHID + lane * 8);
        float s[NOUT] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float hv = (float)h[e];
#pragma unroll
            for (int j = 0; j < NOUT; ++j) s[j] = fmaf(hv, w[j][e], s[j]);
        }
#pragma unroll
        for (int j = 0; j < NOUT; ++j) s[j] = wave_sum(s[j]) + b4[j];
        if (PREDICT) {
            if (m < n && lane < NOUT) {
                const float y = lane == 0 ? s[0] : (lane == 1 ? s[1] : s[2]);
                out[(size_t)m * NOUT + lane] = y / oscale[lane] + oshift[lane];
            }
        } else {
            bool valid = m < n;
            int64_t src = 0;
            if (valid) {
                src = index ? (int64_t)index[m] : (int64_t)m;
                const int sv = sym ? sym[m] : 0;
                valid = src >= 0 && src < ndata && sv >= 0 && sv < 48;
            }
#pragma unroll
            for (int j = 0; j < NOUT; ++j) {
                const float t = valid ? (targets[src * NOUT + j] - oshift[j]) * oscale[j] : 0.0f;
                const float d = valid ? s[j] - t : 0.0f;
                const float g = d * inv;
                if (lane == j) dY[(size_t)m * NOUT + j] = g;
                loss += (double)d * (double)d;
                db[j] += (double)g;
            }
        }
    }
    if (!PREDICT) {
        if (lane == 0) {
            red[wave][0] = loss;
            for (int j = 0; j < NOUT; ++j) red[wave][1 + j] = db[j];
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double t = 0.0;
            for (int q = 0; q < 4; ++q) t += red[q][threadIdx.x];
            partial[blockIdx.x * 4 + threadIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Inference in one launch: the four layers for FW_M rows per workgroup, the hidden activations
// kept in LDS.  The first layer reads the FP32 windows (16-byte aligned) and normalises them as
// the AF32 GEMM does; every hidden product accumulates its 16-wide k-steps in the GEMM's order
// with the same bias + ReLU epilogue, and the output layer is k_out's, so the predictions equal
// those of the layer-by-layer path bit for bit.  Wavefront w of the 8 computes output units
// 64 w .. 64 w + 63 of all FW_M rows (two 32 x 32 accumulator tiles) from its own weight rows,
// loaded FW_K columns at a time.  Grid Mpad / FW_M.
constexpr int FW_M = 32;
constexpr int FW_K = 32;
constexpr int FW_LDX = NIN + 8;   // 16-byte row pad: fragment reads spread over the banks
constexpr int FW_LDH = NHID + 8;
constexpr int FW_T = 512;         // threads
constexpr int FW_D = 4;           // weight stages in flight per wavefront (register buffers)

struct ForwardArgs {
    const float *win;             // [n][NIN], 16-byte aligned
    int n;
    const float *ashift, *ascale; // input normalisation
    const bf16 *W[3];             // hidden weights in fragment order (frag_index)
    const float *bias[3];
    const bf16 *W4;               // [NOUT][NHID]
    const float *b4, *oshift, *oscale;
    float *out;                   // [n][NOUT]
};

__global__ __launch_bounds__(FW_T) void k_forward(ForwardArgs f) {
    __shared__ __attribute__((aligned(16))) bf16 hx[FW_M * FW_LDX];          // input, then layer 2's output
    __shared__ __attribute__((aligned(16))) bf16 ha[FW_M * FW_LDH];          // layers 1 and 3's outputs
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * FW_M;

    // input rows: (a - shift) * scale rounded to BF16, rows >= n zero
    for (int c = tid; c < FW_M * NIN / 8; c += FW_T) {
        const int r = c / (NIN / 8), kc = (c % (NIN / 8)) * 8;
        const bool live = m0 + r < f.n;
        const float4 *src = reinterpret_cast<const float4 *>(f.win + (live ? (size_t)(m0 + r) * NIN + kc : 0));
        const float4 a0 = live ? src[0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 a1 = live ? src[1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 sa = *reinterpret_cast<const float4 *>(f.ashift + kc);
        const float4 sb = *reinterpret_cast<const float4 *>(f.ashift + kc + 4);
        const float4 ca = *reinterpret_cast<const float4 *>(f.ascale + kc);
        const float4 cb = *reinterpret_cast<const float4 *>(f.ascale + kc + 4);
        bf16x8 h;
        h[0] = (bf16)((a0.x - sa.x) * ca.x);
        h[1] = (bf16)((a0.y - sa.y) * ca.y);
        h[2] = (bf16)((a0.z - sa.z) * ca.z);
        h[3] = (bf16)((a0.w - sa.w) * ca.w);
        h[4] = (bf16)((a1.x - sb.x) * cb.x);
        h[5] = (bf16)((a1.y - sb.y) * cb.y);
        h[6] = (bf16)((a1.z - sb.z) * cb.z);
        h[7] = (bf16)((a1.w - sb.w) * cb.w);
        if (!live) h = bf16x8{};
        *reinterpret_cast<bf16x8 *>(hx + r * FW_LDX + kc) = h;
    }

    // one hidden layer: Hout = relu(Hin W^T + b), K = NIN or NHID.  Every weight fragment is used
    // by one wavefront only (the one owning its output units), so each wavefront loads its own
    // fragments, 1 KB of consecutive bytes each in the fragment-ordered copy, into a ring of FW_D
    // register stages, FW_D - 1 stages of products ahead of their use (the loop is unrolled: buffer
    // indices are constants); only the activations, which all wavefronts read, go through LDS.
    auto layer = [&](auto kconst, const bf16 *Hin, int ldin, const bf16 *W, const float *bias, bf16 *Hout) {
        constexpr int K = decltype(kconst)::value;
        constexpr int nk = K / FW_K;
        uint4 bq[FW_D][FW_K / 16][2];  // [stage][k-step][tile]
        // this wavefront's tiles 2 wave, 2 wave + 1 of K / 16 fragments of 1 KB each
        const bf16 *wtile = W + ((size_t)(2 * wave) * (K / 16) * 64 + lane) * 8;
        auto gload = [&](int st, uint4 (&q)[FW_K / 16][2]) {
#pragma unroll
            for (int s = 0; s < FW_K / 16; ++s)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    q[s][j] = ld16(wtile + ((size_t)j * (K / 16) + st * (FW_K / 16) + s) * 512);
        };
        f32x16 acc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[j][e] = 0.0f;
#pragma unroll
        for (int d = 0; d < FW_D; ++d)
            if (d < nk) gload(d, bq[d]);
#pragma unroll
        for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
            for (int s = 0; s < FW_K / 16; ++s) {
                const int kk = s * 16 + (lane >> 5) * 8;
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Hin + (lane & 31) * ldin + kt * FW_K + kk);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        av, __builtin_bit_cast(bf16x8, bq[kt % FW_D][s][j]), acc[j], 0, 0, 0);
            }
            if (kt + FW_D < nk) gload(kt + FW_D, bq[kt % FW_D]);
        }
        // accumulator element 4q + e of a 32x32 tile sits at row 8q + 4 (lane / 32) + e, column lane % 32
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = wave * 64 + j * 32 + (lane & 31);
            const float bb = bias[col];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    Hout[(8 * q + 4 * (lane >> 5) + e) * FW_LDH + col] = (bf16)fmaxf(acc[j][4 * q + e] + bb, 0.0f);
        }
        __syncthreads();
    };
    __syncthreads();
    layer(std::integral_constant<int, NIN>{}, hx, FW_LDX, f.W[0], f.bias[0], ha);
    layer(std::integral_constant<int, NHID>{}, ha, FW_LDH, f.W[1], f.bias[1], hx);
    layer(std::integral_constant<int, NHID>{}, hx, FW_LDH, f.W[2], f.bias[2], ha);

    // output layer (k_out's arithmetic): each wavefront FW_M / 8 rows, lane l the inputs 8 l .. 8 l + 7
    float w[NOUT][8];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(f.W4 + j * NHID + lane * 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) w[j][e] = (float)v[e];
    }
    for (int r = 0; r < FW_M / 8; ++r) {
        const int rl = wave * (FW_M / 8) + r, m = m0 + rl;
        const bf16x8 h = *reinterpret_cast<const bf16x8 *>(ha + rl * FW_LDH + lane * 8);
        float s[NOUT] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float hv = (float)h[e];
#pragma unroll
            for (int j = 0; j < NOUT; ++j) s[j] = fmaf(hv, w[j][e], s[j]);
        }
#pragma unroll
        for (int j = 0; j < NOUT; ++j) s[j] = wave_sum(s[j]) + f.b4[j];
        if (m < f.n && lane < NOUT) {
            const float y = lane == 0 ? s[0] : (lane == 1 ? s[1] : s[2]);
            f.out[(size_t)m * NOUT + lane] = y / f.oscale[lane] + f.oshift[lane];
        }
    }
}

// Sum of the per-block partials in a fixed order (thread t takes blocks t, t + 256, ...; then a
// fixed tree): loss = sum (y - t)^2 / (3 n), db4 = sum dY.  One block of 256 threads.
__global__ __launch_bounds__(256) void k_loss_final(const double *partial, int nblocks, int n, double *loss,
                                                    float *db4) {
    __shared__ double red[256][4];
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[j] += partial[b * 4 + j];
#pragma unroll
    for (int j = 0; j < 4; ++j) red[threadIdx.x][j] = t[j];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[threadIdx.x][j] += red[threadIdx.x + h][j];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (loss) *loss = n > 0 ? red[0][0] / (3.0 * (double)n) : 0.0;
        for (int j = 0; j < NOUT; ++j) db4[j] = (float)red[0][1 + j];
    }
}

// dZ3[m][k] = (sum_j dY[m][j] W4[j][k]) * (H3[m][k] > 0), written [m][k] and [k][m].
// Tiles 64 x 64, grid (NHID / 64, Mpad / 64).
__global__ __launch_bounds__(256) void k_out_back(const float *dY, const bf16 *W4, const bf16 *H, bf16 *dZ, bf16 *dZT,
                                                  int Mpad) {
    __shared__ bf16 tile[64][66];
    const int k0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int k = k0 + tx;
    const float w0 = (float)W4[k], w1 = (float)W4[NHID + k], w2 = (float)W4[2 * NHID + k];
    for (int r = ty; r < 64; r += 4) {
        const int m = m0 + r;
        const float *d = dY + (size_t)m * NOUT;
        float v = d[0] * w0 + d[1] * w1 + d[2] * w2;
        v = (float)H[(size_t)m * NHID + k] > 0.0f ? v : 0.0f;
        const bf16 b = (bf16)v;
        dZ[(size_t)m * NHID + k] = b;
        tile[r][tx] = b;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) dZT[(size_t)(k0 + r) * Mpad + m0 + tx] = tile[tx][r];
}

// out[r * ors + j * ojs] = sum_m AT[r][m] * V[m][j]  (V == nullptr: ones, J == 1); one block per row.
template <int J>
__global__ __launch_bounds__(256) void k_rowdot(const bf16 *AT, int ld, int len, const float *V, float *out, int ors,
                                                int ojs) {
    __shared__ float red[4][J];
    const int r = blockIdx.x;
    float s[J];
#pragma unroll
    for (int j = 0; j < J; ++j) s[j] = 0.0f;
    for (int m = threadIdx.x; m < len; m += 256) {
        const float a = (float)AT[(size_t)r * ld + m];
#pragma unroll
        for (int j = 0; j < J; ++j) s[j] = V ? fmaf(a, V[(size_t)m * J + j], s[j]) : s[j] + a;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        s[j] = wave_sum(s[j]);
        if (lane == 0) red[wave][j] = s[j];
    }
    __syncthreads();
    if (threadIdx.x < J) {
        const int j = threadIdx.x;
        out[(size_t)r * ors + j * ojs] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
    }
}

// ---------------------------------------------------------------------------------------------
// Adam on the FP32 master parameters, then the BF16 copies the products read.
struct Seg {
    int off, rows, cols;
    bf16 *w;   // [rows][cols] copy, or null
    bf16 *wt;  // [cols][rows] copy, or null
    bf16 *wf;  // copy in MFMA fragment order (frag_index), or null
};

// Position of W[n][k] (K = cols, a multiple of 16) in the fragment-ordered copy the one-launch
// inference reads: [tile n / 32][k-step k / 16][lane][8], lane (n % 32) + 32 ((k % 16) / 8), so
// that one wavefront's B fragment of a 32 x 32 x 16 product is 1 KB of consecutive bytes.
__host__ __device__ __forceinline__ size_t frag_index(int n, int k, int K) {
    const int lane = (n & 31) + 32 * ((k & 15) >> 3);
    return ((size_t)((n >> 5) * (K >> 4) + (k >> 4)) * 64 + lane) * 8 + (k & 7);
}
struct AdamArgs {
    float *p;
    const float *g;
    float *m, *v;
    int n;
    int update;  // 0: only refresh the BF16 copies
    float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^step
    Seg seg[NLAYER];
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n; i += gridDim.x * 256) {
        float p = a.p[i];
        if (a.update) {
            const float g = a.g[i];
            const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
            const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
            a.m[i] = m;
            a.v[i] = v;
            p -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
            a.p[i] = p;
        }
#pragma unroll
        for (int s = 0; s < NLAYER; ++s) {
            const Seg &q = a.seg[s];
            const int o = i - q.off;
            if (o >= 0 && o < q.rows * q.cols) {
                const bf16 b = (bf16)p;
                if (q.w) q.w[o] = b;
                if (q.wt) q.wt[(size_t)(o % q.cols) * q.rows + o / q.cols] = b;
                if (q.wf) q.wf[frag_index(o / q.cols, o % q.cols, q.cols)] = b;
            }
        }
    }
}

}  // namespace sclmlp
