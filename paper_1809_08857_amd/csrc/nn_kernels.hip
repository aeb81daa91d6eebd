// Device kernels of the learned initial guess: a 3D convolutional U-net in
// bfloat16 with FP32 accumulation on the CDNA4 matrix cores
// (v_mfma_f32_16x16x32_bf16), its backward pass and its optimiser.
//
// Convolutions are implicit GEMMs.  One MFMA computes a 16x16 tile
// D[co][v] += W[co][k] X[k][v] over 32 reduction indices k = (tap, input
// channel): the weights are the A operand (16 output channels, k
// contiguous per row), the activations the B operand (16 cells along x,
// eight consecutive channels of one cell per lane = one 16-byte load from
// the channels-last tensor).  The result layout gives each lane four
// consecutive output channels of one cell, so the epilogue stores 8 bytes
// per lane and a row of 16 cells is written contiguously.
//
// The input gradient of a convolution is again a convolution (transposed
// weights; mirrored taps for 3x3x3, DOWN2 <-> UP2 for the strided pair), so
// conv_k serves the forward and the backward data pass.  The weight
// gradient reduces over cells: wgrad_k puts cells on the reduction axis and
// gathers eight cells of one channel per lane from the channels-last
// tensors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "nn_internal.h"

namespace nn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf2f(unsigned b) { return __uint_as_float((b & 0xffffu) << 16); }

// float -> bfloat16, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ unsigned f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// bfloat16 pattern > 0 (NaN excluded)
__device__ __forceinline__ bool bf_pos(unsigned b) { return !(b & 0x8000u) && (b & 0x7fffu) && (b & 0x7fffu) <= 0x7f80u; }

__device__ __forceinline__ u32x4 ld16(const bf16_t *p) { return *reinterpret_cast<const u32x4 *>(p); }

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
}

__device__ __forceinline__ u32x4 pack8(const unsigned (&e)[8]) {
    u32x4 r;
    r.x = e[0] | (e[1] << 16);
    r.y = e[2] | (e[3] << 16);
    r.z = e[4] | (e[5] << 16);
    r.w = e[6] | (e[7] << 16);
    return r;
}

// Epilogue of one lane: output channels co..co+3 of output cell ov, with
// the bias of those channels (zero without one) already in registers.
__device__ __forceinline__ void store4b(const ConvArgs &a, size_t ov, int co, f32x4 acc, f32x4 bias) {
    float v[4] = {acc.x + bias.x, acc.y + bias.y, acc.z + bias.z, acc.w + bias.w};
    if (a.relu) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
    }
    bf16_t *d;
    const bf16_t *mk;
    int cd, cc, ac;
    if (co < a.da) {
        d = a.dstA, cd = a.da, cc = co, mk = a.maskA, ac = a.accA;
    } else {
        d = a.dstB, cd = a.db, cc = co - a.da, mk = a.maskB, ac = a.accB;
    }
    const size_t off = ov * cd + cc;
    if (mk) {
        const u32x2 mm = *reinterpret_cast<const u32x2 *>(mk + off);
        if (!bf_pos(mm.x)) v[0] = 0.f;
        if (!bf_pos(mm.x >> 16)) v[1] = 0.f;
        if (!bf_pos(mm.y)) v[2] = 0.f;
        if (!bf_pos(mm.y >> 16)) v[3] = 0.f;
    }
    if (ac) {
        const u32x2 o = *reinterpret_cast<const u32x2 *>(d + off);
        v[0] += bf2f(o.x);
        v[1] += bf2f(o.x >> 16);
        v[2] += bf2f(o.y);
        v[3] += bf2f(o.y >> 16);
    }
    u32x2 st;
    st.x = f2bf(v[0]) | (f2bf(v[1]) << 16);
    st.y = f2bf(v[2]) | (f2bf(v[3]) << 16);
    *reinterpret_cast<u32x2 *>(d + off) = st;
}

// Two floats -> packed bfloat16 pair (hardware conversion, round to nearest even).
__device__ __forceinline__ unsigned pk_bf16(float lo, float hi) {
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}

__device__ __forceinline__ f32x4 bias4(const ConvArgs &a, int co) {
    return a.bias ? f32x4{a.bias[co], a.bias[co + 1], a.bias[co + 2], a.bias[co + 3]} : f32x4{0.f, 0.f, 0.f, 0.f};
}

// Epilogue of one lane: output channels co..co+3 of output cell ov.
__device__ __forceinline__ void store4(const ConvArgs &a, size_t ov, int co, f32x4 acc) {
    store4b(a, ov, co, acc, bias4(a, co));
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// fences global memory, which makes every wave wait for its outstanding
// global loads and stores; the z-marching convolution shares only LDS
// between its waves and keeps loads of the next plane in flight across the
// barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Hardware block w of n -> logical block, so that each of the 8 XCDs (which
// receive blocks round-robin) works on one contiguous range of tiles and
// the halos its tiles share stay in its own L2.
__device__ __forceinline__ int xcd_order(int w, int n) {
    const int q = n / 8, r = n % 8;
    const int xcd = w % 8, pos = w / 8;
    return xcd * q + min(xcd, r) + pos;
}

// ------------------------------------------------------------------ conv
// Block: 4 waves; wave w owns output row y = 4*blockIdx.y + w and NT rows
// z = NT*blockIdx.z' + 0..NT-1 of a 16-cell x segment, for all COUT output
// channels (MT = COUT/16 tiles).  UP2 tiles the coarse input grid and
// spends blockIdx.z on the 8 output parities as well.
template <int GEOM, int COUT, int NT>
__global__ __launch_bounds__(256) void conv_k(ConvArgs a) {
    constexpr int MT = COUT / 16;
    constexpr int T = GEOM == G_SAME3 ? 27 : (GEOM == G_DOWN2 ? 8 : 1);  // taps summed per output
    constexpr int WT = GEOM == G_SAME3 ? 27 : 8;                          // taps per weight row
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int K = T * cin;
    const int nchunk = (K + 31) >> 5;
    int tnx, tny, tnz;
    if (GEOM == G_UP2) {
        tnx = a.inx, tny = a.iny, tnz = a.inz;
    } else {
        tnx = a.onx, tny = a.ony, tnz = a.onz;
    }
    int bz = blockIdx.z, par = 0;
    if (GEOM == G_UP2) {
        const int nzb = (tnz + NT - 1) / NT;
        par = bz / nzb;
        bz -= par * nzb;
    }
    const int x = blockIdx.x * 16 + col;
    const int y = blockIdx.y * 4 + wave;
    const int z0 = bz * NT;
    const bool colok = x < tnx && y < tny;

    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Operands of chunk c + 1 are loaded before the products of chunk c.
    // Loads are unconditional (from clamped addresses) and the operands
    // outside the reduction range or the grid are zeroed by a mask where
    // they are used, so that no load is waited for under a branch.
    auto fetch = [&](int c, u32x4 (&A)[MT], u32x4 (&B)[NT], unsigned &am, unsigned (&bm)[NT]) {
        const int k0 = c * 32 + grp * 8;
        const bool kok = k0 < K;
        const int tap = kok ? k0 / cin : 0;
        const int ci = kok ? k0 - tap * cin : 0;
        const bf16_t *src;
        int cs, cl;
        if (ci < a.ca) {
            src = a.srcA, cs = a.ca, cl = ci;
        } else {
            src = a.srcB, cs = a.cb, cl = ci - a.ca;
        }
        int dx = 0, dy = 0, dz = 0;
        if (GEOM == G_SAME3) {
            dz = tap / 9 - 1;
            dy = (tap / 3) % 3 - 1;
            dx = tap % 3 - 1;
        } else if (GEOM == G_DOWN2) {
            dz = tap >> 2;
            dy = (tap >> 1) & 1;
            dx = tap & 1;
        }
        const int wt = GEOM == G_UP2 ? par : tap;
        am = kok ? 0xffffffffu : 0u;
#pragma unroll
        for (int m = 0; m < MT; ++m) A[m] = ld16(a.w + ((size_t)(m * 16 + col) * WT + wt) * cin + ci);
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int z = z0 + n;
            bool ok = kok && colok && z < tnz;
            int sx, sy, sz;
            if (GEOM == G_SAME3) {
                sx = x + dx, sy = y + dy, sz = z + dz;
                ok = ok && sx >= 0 && sx < a.inx && sy >= 0 && sy < a.iny && sz >= 0 && sz < a.inz;
            } else if (GEOM == G_DOWN2) {
                sx = 2 * x + dx, sy = 2 * y + dy, sz = 2 * z + dz;
            } else {
                sx = x, sy = y, sz = z;
            }
            sx = min(max(sx, 0), a.inx - 1), sy = min(max(sy, 0), a.iny - 1), sz = min(max(sz, 0), a.inz - 1);
            bm[n] = ok ? 0xffffffffu : 0u;
            B[n] = ld16(src + (((size_t)sz * a.iny + sy) * a.inx + sx) * cs + cl);
        }
    };
    u32x4 An[MT], Bn[NT];
    unsigned amn, bmn[NT];
    fetch(0, An, Bn, amn, bmn);
    for (int c = 0; c < nchunk; ++c) {
        u32x4 A[MT], B[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) A[m] = An[m];
#pragma unroll
        for (int n = 0; n < NT; ++n) B[n] = Bn[n];
        const unsigned am = amn;
        unsigned bm[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) bm[n] = bmn[n];
        if (c + 1 < nchunk) fetch(c + 1, An, Bn, amn, bmn);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[m][n] = mfma(A[m] & am, B[n] & bm[n], acc[m][n]);
    }

    int px = 0, py = 0, pz = 0;
    if (GEOM == G_UP2) {
        pz = par >> 2;
        py = (par >> 1) & 1;
        px = par & 1;
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int z = z0 + n;
        if (!colok || z >= tnz) continue;
        int ox = x, oy = y, oz = z;
        if (GEOM == G_UP2) ox = 2 * x + px, oy = 2 * y + py, oz = 2 * z + pz;
        const size_t ov = ((size_t)oz * a.ony + oy) * a.onx + ox;
#pragma unroll
        for (int m = 0; m < MT; ++m) store4(a, ov, m * 16 + grp * 4, acc[m][n]);
    }
}

// Stride-2 convolution (DOWN2) with 16, 32 or 64 input channels: a block
// computes 16 output cells of one row on NT planes for all MT channel tiles,
// and its 4 waves split the reduction (8 taps x cin = 4 * CPW K-chunks of
// 32): wave w takes chunks w, w + 4, ...  Each wave issues the loads of all
// its chunks before its first product, so a block waits for one memory
// latency, not one per chunk.  The partial sums meet in LDS and each wave
// adds the four (in wave order) for a quarter of the output tiles.
template <int MT, int NT, int CPW>
__global__ __launch_bounds__(256) void down2_k(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int x = blockIdx.x * 16 + col, y = blockIdx.y, z0 = blockIdx.z * NT;
    const int xc = min(x, a.onx - 1);
    u32x4 A[CPW][MT], B[CPW][NT];
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
        const int k0 = (wave + 4 * i) * 32 + grp * 8;
        const int tap = k0 / cin, ci = k0 - tap * cin;
        const int dz = tap >> 2, dy = (tap >> 1) & 1, dx = tap & 1;
        const bf16_t *src = ci < a.ca ? a.srcA + ci : a.srcB + (ci - a.ca);
        const int cs = ci < a.ca ? a.ca : a.cb;
#pragma unroll
        for (int m = 0; m < MT; ++m) A[i][m] = ld16(a.w + ((size_t)(m * 16 + col) * 8 + tap) * cin + ci);
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int zc = min(z0 + n, a.onz - 1);
            B[i][n] = ld16(src + (((size_t)(2 * zc + dz) * a.iny + 2 * y + dy) * a.inx + 2 * xc + dx) * cs);
        }
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < CPW; ++i) acc[m][n] = mfma(A[i][m], B[i][n], acc[m][n]);
        }
    __shared__ __align__(16) f32x4 part[4][MT * NT][64];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) part[wave][m * NT + n][lane] = acc[m][n];
    __syncthreads();
    for (int p = wave; p < MT * NT; p += 4) {
        const int m = p / NT, n = p % NT;
        const f32x4 v = part[0][p][lane] + part[1][p][lane] + part[2][p][lane] + part[3][p][lane];
        const int z = z0 + n;
        if (x < a.onx && z < a.onz) store4(a, ((size_t)z * a.ony + y) * a.onx + x, m * 16 + grp * 4, v);
    }
}

// Transposed stride-2 convolution (UP2) with 32 or 64 input channels (NCH
// K-chunks) and 16, 32 or 64 output channels.  A block owns 16 coarse cells
// of one row on NT coarse planes; wave w forms the output parities
// (px, py, pz) = (0 and 1, w & 1, w >> 1) from them, the weights of its two
// parities in registers.  The two px parities of a lane are adjacent fine
// cells, so the stores of a fine row are contiguous.  Coarse cells outside
// the grid read a clamped cell and store nothing.
template <int MT, int NT, int NCH>
__global__ __launch_bounds__(256) void up2_k(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int x = blockIdx.x * 16 + col, y = blockIdx.y, z0 = blockIdx.z * NT;
    const int py = wave & 1, pz = wave >> 1;
    u32x4 A[2][NCH][MT];
    f32x4 bv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        bv[m] = bias4(a, m * 16 + grp * 4);
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                A[px][c][m] = ld16(a.w + ((size_t)(m * 16 + col) * 8 + pz * 4 + py * 2 + px) * cin + c * 32 + grp * 8);
    }
    const int xc = min(x, a.inx - 1);
    u32x4 B[NT][NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int ch = c * 32 + grp * 8;
        const bf16_t *src = ch < a.ca ? a.srcA + ch : a.srcB + (ch - a.ca);
        const int cs = ch < a.ca ? a.ca : a.cb;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int zc = min(z0 + n, a.inz - 1);
            B[n][c] = ld16(src + (((size_t)zc * a.iny + y) * a.inx + xc) * cs);
        }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int z = z0 + n;
        f32x4 acc[2][MT];
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                acc[px][m] = bv[m];
#pragma unroll
                for (int c = 0; c < NCH; ++c) acc[px][m] = mfma(A[px][c][m], B[n][c], acc[px][m]);
            }
        if (x >= a.inx || z >= a.inz) continue;
#pragma unroll
        for (int px = 0; px < 2; ++px) {
            const size_t ov = ((size_t)(2 * z + pz) * a.ony + 2 * y + py) * a.onx + 2 * x + px;
#pragma unroll
            for (int m = 0; m < MT; ++m) store4b(a, ov, m * 16 + grp * 4, acc[px][m], f32x4{0.f, 0.f, 0.f, 0.f});
        }
    }
}

// 3x3x3 convolution with the input tile staged in LDS.  Block: output tile
// of 16 x RY x RZ cells (x fastest); wave w owns rows r = w, w+4, ... of
// the RY*RZ rows of 16 cells, for all COUT output channels.  The input
// channels are staged CC at a time: the (18) x (RY+2) x (RZ+2) halo tile,
// zero outside the grid, with a per-cell stride of VS bfloat16 (16-byte
// units odd, so the 16 cells a lane group reads hit distinct banks).  Each
// MFMA takes its B operand (8 channels of one cell per lane) from LDS and
// its A operand (16 output channels x 8 taps/channels) from the weights.
template <int COUT, int CC, int RY, int RZ>
__global__ __launch_bounds__(256) void conv3_lds_k(ConvArgs a) {
    constexpr int MT = COUT / 16;
    constexpr int RPW = RY * RZ / 4;
    constexpr int HX = 18, HY = RY + 2, HZ = RZ + 2;
    constexpr int NV = HX * HY * HZ;
    constexpr int G8 = CC / 8;                      // 8-channel groups per cell
    constexpr int VS = (G8 % 2 == 0) ? CC + 8 : CC; // LDS stride per cell
    constexpr int GPT = G8 < 4 ? G8 : 4;            // lane groups per tap
    constexpr int TPC = 4 / GPT;                    // taps per K-chunk of 32
    constexpr int CPT = G8 / GPT;                   // K-chunks per tap
    __shared__ __align__(16) bf16_t tile[NV * VS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int ntx = (a.onx + 15) / 16, nty = (a.ony + RY - 1) / RY, ntz = (a.onz + RZ - 1) / RZ;
    const int b = xcd_order(blockIdx.x, ntx * nty * ntz);
    const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
    const int x0 = bx * 16, y0 = by * RY, z0 = bz * RZ;

    f32x4 acc[MT][RPW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < RPW; ++r) acc[m][r] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    // this lane's tap offset within a K-chunk and channel offset within a tap
    const int tsub = grp / GPT;
    const int cl = (grp % GPT) * 8;

    for (int cb = 0; cb < cin; cb += CC) {
        __syncthreads();
        for (int i = threadIdx.x; i < NV * G8; i += 256) {
            const int v = i / G8, q = i - v * G8;
            const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            u32x4 val = zero;
            if (gx >= 0 && gx < a.inx && gy >= 0 && gy < a.iny && gz >= 0 && gz < a.inz) {
                const int ci = cb + q * 8;
                const size_t cell = ((size_t)gz * a.iny + gy) * a.inx + gx;
                val = ci < a.ca ? ld16(a.srcA + cell * a.ca + ci) : ld16(a.srcB + cell * a.cb + (ci - a.ca));
            }
            *reinterpret_cast<u32x4 *>(tile + v * VS + q * 8) = val;
        }
        __syncthreads();
#pragma unroll 1
        for (int t0 = 0; t0 < 27; t0 += TPC) {
            const int tap = t0 + tsub;
            const bool tok = tap < 27;
            const int tq = tok ? tap : 0;
            const int dz = tq / 9, dy = (tq / 3) % 3, dx = tq % 3;  // offsets + 1
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int ch = c * 32 + cl;  // channel within the staged block
                u32x4 A[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    A[m] = tok ? ld16(a.w + ((size_t)(m * 16 + col) * 27 + tq) * cin + cb + ch) : zero;
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int row = wave + 4 * r;
                    const int ry = row % RY, rz = row / RY;
                    const int v = ((rz + dz) * HY + (ry + dy)) * HX + col + dx;
                    const u32x4 B = tok ? *reinterpret_cast<const u32x4 *>(tile + v * VS + ch) : zero;
#pragma unroll
                    for (int m = 0; m < MT; ++m) acc[m][r] = mfma(A[m], B, acc[m][r]);
                }
            }
        }
    }
    const int ox = x0 + col;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int row = wave + 4 * r;
        const int oy = y0 + row % RY, oz = z0 + row / RY;
        if (ox >= a.onx || oy >= a.ony || oz >= a.onz) continue;
        const size_t ov = ((size_t)oz * a.ony + oy) * a.onx + ox;
#pragma unroll
        for (int m = 0; m < MT; ++m) store4(a, ov, m * 16 + grp * 4, acc[m][r]);
    }
}

// LDS byte offset (in cells) of tap t in the halo tile, taps (dz,dy,dx)+1.
template <int HX, int HY>
__device__ __forceinline__ constexpr int tap_off(int t) {
    return ((t / 9) * HY + (t / 3) % 3) * HX + t % 3;
}

// 3x3x3 convolution, weights resident in registers.  As conv3_lds_k, but
// the waves split the output channels into WM groups (wave w: channel
// tiles of group w % WM, rows w / WM, w / WM + 4/WM, ...), and each wave
// loads its whole A operand for the staged channel block (NCH K-chunks)
// into registers before the K loop, which is fully unrolled so that every
// LDS address is a per-row base plus a compile-time offset.
template <int COUT, int CC, int RY, int RZ, int WM>
__global__ __launch_bounds__(256) void conv3_reg_k(ConvArgs a) {
    constexpr int MT = COUT / 16;
    constexpr int MTW = MT / WM;                    // channel tiles per wave
    constexpr int WR = 4 / WM;                      // wave groups along rows
    constexpr int RW = RY * RZ / WR;                // rows per wave
    constexpr int HX = 18, HY = RY + 2, HZ = RZ + 2;
    constexpr int NV = HX * HY * HZ;
    constexpr int G8 = CC / 8;
    constexpr int VS = (G8 % 2 == 0) ? CC + 8 : CC;
    constexpr int GPT = G8 < 4 ? G8 : 4;            // lane groups per tap
    constexpr int TPC = 4 / GPT;                    // taps per K-chunk
    constexpr int NCH = (27 + TPC - 1) / TPC;       // K-chunks per staged block
    static_assert(G8 <= 4, "staged channel block must fit one K-chunk per tap");
    __shared__ __align__(16) bf16_t tile[NV * VS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int wm = wave % WM, wr = wave / WM;
    const int cin = a.ca + a.cb;
    const int ntx = (a.onx + 15) / 16, nty = (a.ony + RY - 1) / RY, ntz = (a.onz + RZ - 1) / RZ;
    const int b = xcd_order(blockIdx.x, ntx * nty * ntz);
    const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
    const int x0 = bx * 16, y0 = by * RY, z0 = bz * RZ;
    const int tsub = grp / GPT;
    const int cl = (grp % GPT) * 8;

    f32x4 acc[MTW][RW];
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[m][r] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    int rbase[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int row = wr + WR * r;
        rbase[r] = ((row / RY) * HY + row % RY) * HX + col;
    }

    for (int cb = 0; cb < cin; cb += CC) {
        u32x4 A[NCH][MTW];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int tap = c * TPC + tsub;
#pragma unroll
            for (int m = 0; m < MTW; ++m) {
                const int co = (wm * MTW + m) * 16 + col;
                A[c][m] = tap < 27 ? ld16(a.w + ((size_t)co * 27 + tap) * cin + cb + cl) : zero;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < NV * G8; i += 256) {
            const int v = i / G8, q = i - v * G8;
            const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            u32x4 val = zero;
            if (gx >= 0 && gx < a.inx && gy >= 0 && gy < a.iny && gz >= 0 && gz < a.inz) {
                const int ci = cb + q * 8;
                const size_t cell = ((size_t)gz * a.iny + gy) * a.inx + gx;
                val = ci < a.ca ? ld16(a.srcA + cell * a.ca + ci) : ld16(a.srcB + cell * a.cb + (ci - a.ca));
            }
            *reinterpret_cast<u32x4 *>(tile + v * VS + q * 8) = val;
        }
        __syncthreads();
        // B operands of chunk c + 1 are read before the products of chunk c
        auto fetchB = [&](int c, u32x4 (&B)[RW]) {
            // this lane's tap in chunk c (past the last tap: any cell, A is 0)
            int off = tap_off<HX, HY>(c * TPC < 27 ? c * TPC : 26);
#pragma unroll
            for (int k = 1; k < TPC; ++k)
                if (tsub == k) off = tap_off<HX, HY>(c * TPC + k < 27 ? c * TPC + k : 26);
#pragma unroll
            for (int r = 0; r < RW; ++r) B[r] = *reinterpret_cast<const u32x4 *>(tile + (rbase[r] + off) * VS + cl);
        };
        u32x4 Bn[RW];
        fetchB(0, Bn);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            u32x4 Bc[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) Bc[r] = Bn[r];
            if (c + 1 < NCH) fetchB(c + 1, Bn);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int m = 0; m < MTW; ++m) acc[m][r] = mfma(A[c][m], Bc[r], acc[m][r]);
            // keep the order: next chunk's LDS reads, then this chunk's MFMAs
            if (c + 1 < NCH) __builtin_amdgcn_sched_group_barrier(0x100, RW, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, RW * MTW, 0);
        }
    }
    const int ox = x0 + col;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int row = wr + WR * r;
        const int oy = y0 + row % RY, oz = z0 + row / RY;
        if (ox >= a.onx || oy >= a.ony || oz >= a.onz) continue;
        const size_t ov = ((size_t)oz * a.ony + oy) * a.onx + ox;
#pragma unroll
        for (int m = 0; m < MTW; ++m) store4(a, ov, (wm * MTW + m) * 16 + grp * 4, acc[m][r]);
    }
}

// 3x3x3 convolution marching along z: 8, 16 or 32 input channels with 16
// or 32 output channels, 64 input channels with 32 or 64 output channels
// (the other shapes take the staged-tile kernels).  Block: NWV waves on an xy tile of
// 16 x BY output cells and a chunk of zc output planes.  A wave owns one
// 16-channel output tile (wm), one share of the input channels (kh of KS,
// CK channels each) and RW rows of the tile (row group wr); its weights
// stay in registers for the whole block.
//
// The block streams the input planes zb-1 .. zb+zc through LDS (two
// slots: the plane being read and the next one, loaded into registers
// during the products of the current one).  Input plane z' contributes to
// output planes z'+1, z', z'-1 (taps tz = 0, 1, 2), so each wave keeps
// three planes of accumulators in a ring; after plane z' the output plane
// z'-1 is complete and is stored.  Every B operand read from LDS (16 cells
// of one input row at one x offset) serves the 3 output rows and the 3
// output planes it reaches: up to 9 MFMAs per LDS read.
//
// K-chunks of 32 reduction indices per (ty, tz), over the wave's CK
// channels: with 8, one chunk of the taps tx = 0, 1, 2 (last quarter of the
// weights zero); with 16, chunk 0 = taps tx = 0, 1 and chunk 1 = tap tx = 2
// (upper half of the weights zero); with 32, chunk c = tap tx = c.
//
// With the input channels split over two waves (KS = 2, 64 input
// channels), the wave with kh = 0 stores the even rows and the other the
// odd rows: before the plane's barrier each wave writes to LDS its partial
// sums of the rows the other one stores, and adds the other's partial sums
// of its own rows after it (two LDS slots of partial sums, by plane parity).
// With four (KS = 4, 128 input channels) wave kh stores row kh and adds the
// three other waves' partial sums of it in wave order.  A block covers
// 16 * MT output channels; where the layer has more, the channel group g is
// part of the block index.
//
// The bias enters as the accumulator operand of each output plane's first
// MFMA (in the wave with kh = 0), which also starts the plane's
// accumulators afresh.
//
// PLAIN: the epilogue is ReLU (if RELU) into dstA only (no mask, no
// accumulation, no second destination, dstA under 2 GiB), converted by the
// hardware's packed bfloat16 conversion.  Its stores are buffer stores
// issued by every lane in every step, with an offset past the end of the
// buffer where there is nothing to write (the hardware drops those), so the
// number of memory operations per step does not depend on a branch and the
// waits for the next plane's loads do not also wait for the completion of
// the stores issued after them.
template <int MT, int KS>
constexpr int zm_waves() {
    return MT * KS <= 4 ? 4 : MT * KS;
}

template <int CIN, int MT, int KS, bool PLAIN, bool RELU>
__global__ __launch_bounds__((64 * zm_waves<MT, KS>()), (8 / zm_waves<MT, KS>())) void conv3_zm_k(ConvArgs a, int zc) {
    constexpr int NWV = zm_waves<MT, KS>();            // waves per block
    constexpr int NTH = 64 * NWV;
    constexpr int CK = CIN / KS;                       // input channels per wave
    constexpr int RW = 4;                              // output rows per wave
    constexpr int WR = NWV / (MT * KS);                // wave groups along y
    constexpr int BY = RW * WR;                        // output rows per block
    constexpr int HX = 18, HY = BY + 2;
    constexpr int NV = HX * HY;                        // cells per staged plane
    constexpr int G8 = CIN / 8;                        // 16-byte groups per cell
    constexpr int VS = (G8 % 2 == 0) ? CIN + 8 : CIN;  // LDS stride per cell (odd 16-byte count)
    constexpr int NCK = CK == 32 ? 3 : (CK == 16 ? 2 : 1);  // K-chunks per (ty, tz)
    constexpr int CPW = NTH / G8;                      // cells staged per pass of the block
    constexpr int NLD = (NV + CPW - 1) / CPW;          // staging loads per thread and plane
    constexpr int NVS = NLD * CPW;                     // cells per LDS slot (the last pass whole)
    constexpr int RS = RW / KS;                        // rows a wave stores
    static_assert(CK == 8 || CK == 16 || CK == 32, "8, 16 or 32 input channels per wave");
    static_assert(KS == 1 || KS == 2 || KS == 4, "input channels split over 1, 2 or 4 waves");
    static_assert(NWV % (MT * KS) == 0, "whole wave groups");
    static_assert(KS == 1 || WR == 1, "the partial sums are indexed by output tile and row only");
    __shared__ __align__(16) bf16_t tile[2 * NVS * VS];
    __shared__ __align__(16) f32x4 part[KS == 1 ? 1 : 2 * MT * RW * (KS == 4 ? 4 : 1) * 64];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int wm = wave % MT, kh = (wave / MT) % KS, wr = wave / (MT * KS);
    const int kc = kh * CK;  // first input channel of this wave
    const int cin = a.ca + a.cb;
    const int ng = (a.da + a.db) / (16 * MT);  // output channel groups
    const int ntx = (a.onx + 15) / 16, nty = (a.ony + BY - 1) / BY, ntz = (a.onz + zc - 1) / zc;
    const int bg = xcd_order(blockIdx.x, ntx * nty * ntz * ng);
    const int g = bg % ng, b = bg / ng;
    const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
    const int x0 = bx * 16, y0 = by * BY, zb = bz * zc;
    const int mo = (g * MT + wm) * 16;     // first output channel of this wave
    const int nout = min(zc, a.onz - zb);  // output planes of this block
    const int nsteps = nout + 2;           // input planes zb-1 .. zb+nout
    const u32x4 zero = {0u, 0u, 0u, 0u};

    // this lane's x tap and channel offset in each K-chunk
    int ctx[NCK], cci[NCK];
    bool cok[NCK];
#pragma unroll
    for (int c = 0; c < NCK; ++c) {
        if constexpr (CK == 8) {
            ctx[c] = grp < 3 ? grp : 2;
            cci[c] = 0;
            cok[c] = grp < 3;
        } else if constexpr (CK == 16) {
            ctx[c] = c == 0 ? grp / 2 : 2;
            cci[c] = (grp % 2) * 8;
            cok[c] = c == 0 || grp < 2;
        } else {
            ctx[c] = c;
            cci[c] = grp * 8;
            cok[c] = true;
        }
        cci[c] += kc;
    }
    // weights A[ty][tz][c]: output channel wm*16 + col, reduction lanes of grp
    u32x4 A[3][3][NCK];
    {
        const bf16_t *wr0 = a.w + (size_t)(mo + col) * 27 * cin;
#pragma unroll
        for (int ty = 0; ty < 3; ++ty)
#pragma unroll
            for (int tz = 0; tz < 3; ++tz)
#pragma unroll
                for (int c = 0; c < NCK; ++c) {
                    const u32x4 w = ld16(wr0 + (tz * 9 + ty * 3 + ctx[c]) * cin + cci[c]);
                    A[ty][tz][c] = cok[c] ? w : zero;
                }
    }

    // staging: thread t loads 8 channels (group t % G8) of cells t / G8 + k * CPW.
    // Loads are unconditional (cells outside the grid read cell 0 of the
    // plane, planes outside read plane 0) and the zeros are put in where
    // the values are written to LDS, so no load waits under a branch.
    const int q = threadIdx.x % G8, v0 = threadIdx.x / G8;
    const int ch = q * 8;
    const bool fromA = ch < a.ca;
    const bf16_t *sbase = fromA ? a.srcA + ch : a.srcB + (ch - a.ca);
    const int cs = fromA ? a.ca : a.cb;
    const size_t plane = (size_t)a.inx * a.iny;
    int soff[NLD];   // cell offset within a plane
    bool sok[NLD];   // inside the grid and the tile
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int v = v0 + k * CPW;
        const int hx = v % HX, hy = v / HX;
        const int gx = x0 + hx - 1, gy = y0 + hy - 1;
        sok[k] = v < NV && gx >= 0 && gx < a.inx && gy >= 0 && gy < a.iny;
        soff[k] = sok[k] ? gy * a.inx + gx : 0;
    }
    auto load_plane = [&](int z, u32x4 (&R)[NLD]) {
        const bf16_t *p = sbase + (size_t)(z >= 0 && z < a.inz ? z : 0) * plane * cs;
#pragma unroll
        for (int k = 0; k < NLD; ++k) R[k] = ld16(p + (size_t)soff[k] * cs);
    };
    auto store_plane = [&](int slot, int z, const u32x4 (&R)[NLD]) {
        bf16_t *t = tile + slot * (NVS * VS);
        const bool zok = z >= 0 && z < a.inz;
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const unsigned m = (zok && sok[k]) ? 0xffffffffu : 0u;
            *reinterpret_cast<u32x4 *>(t + (v0 + k * CPW) * VS + ch) = R[k] & m;
        }
    };

    f32x4 acc[3][RW];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[p][r] = f32x4{0.f, 0.f, 0.f, 0.f};
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    // B operand addresses: row j of the wave's RW + 2 input rows, chunk c
    int boff[NCK];
#pragma unroll
    for (int c = 0; c < NCK; ++c) boff[c] = ((wr * RW) * HX + col + ctx[c]) * VS + cci[c];

    const f32x4 bv = bias4(a, mo + grp * 4);
    const f32x4 bstart = kh == 0 ? bv : zero4;  // the bias enters once
    // destination as a buffer resource (plain epilogue only)
    const __amdgpu_buffer_rsrc_t dst = __builtin_amdgcn_make_buffer_rsrc(
        a.dstA, (short)0, PLAIN ? (int)((size_t)a.onx * a.ony * a.onz * a.da * sizeof(bf16_t)) : 0, 0x00020000);
    // R holds the next input plane from the LDS write of one plane to that
    // of the next, so its loads are in flight across a barrier, an epilogue
    // and a plane of products.
    u32x4 R[NLD];
    load_plane(zb - 1, R);
    store_plane(0, zb - 1, R);
    // weights, bias and the first plane are in registers: nothing is left
    // outstanding that the loop would have to wait for
    __builtin_amdgcn_s_waitcnt(0);
    if (nsteps > 1) load_plane(zb, R);
    lds_barrier();

    const int ox = x0 + col;
    // rows this wave stores: r = KS * i + kh; plain epilogue: their byte
    // offsets in plane zb and the bytes per plane
    bool rok[RS];
    unsigned roff[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        const int oy = y0 + wr * RW + KS * i + kh;
        rok[i] = ox < a.onx && oy < a.ony;
        roff[i] = (unsigned)(((((size_t)zb * a.ony + oy) * a.onx + ox) * a.da + mo + grp * 4) * sizeof(bf16_t));
    }
    const unsigned pbytes = (unsigned)((size_t)a.onx * a.ony * a.da * sizeof(bf16_t));
    // input plane zb - 1 + s; S3 = s % 3 fixes the accumulator ring at compile time
    auto step = [&](auto s3c, int s) {
        constexpr int S3 = decltype(s3c)::value;
        const bf16_t *t = tile + (s & 1) * (NVS * VS);
#pragma unroll
        for (int j = 0; j < RW + 2; ++j) {
            u32x4 B[NCK];
#pragma unroll
            for (int c = 0; c < NCK; ++c) B[c] = *reinterpret_cast<const u32x4 *>(t + boff[c] + j * HX * VS);
#pragma unroll
            for (int c = 0; c < NCK; ++c)
#pragma unroll
                for (int r = j - 2; r <= j; ++r)
                    if (r >= 0 && r < RW)
#pragma unroll
                        for (int tz = 0; tz < 3; ++tz) {
                            // the first product into output plane zb + s (tap tz = 0) starts from the bias
                            f32x4 &d = acc[(S3 + 3 - tz) % 3][r];
                            d = mfma(A[j - r][tz][c], B[c], (tz == 0 && j == r && c == 0) ? bstart : d);
                        }
        }
        // output plane zb + s - 2 is complete (in acc[P]); the rows this wave stores
        constexpr int P = (S3 + 1) % 3;
        f32x4 out[RS];
        if constexpr (KS == 2) {
            // partial sums of the other wave's rows to LDS
            f32x4 *pw = part + ((s & 1) * MT + wm) * RW * 64 + lane;
#pragma unroll
            for (int i = 0; i < RS; ++i) {
                pw[(2 * i + 1 - kh) * 64] = kh ? acc[P][2 * i] : acc[P][2 * i + 1];
                out[i] = kh ? acc[P][2 * i + 1] : acc[P][2 * i];
            }
        } else if constexpr (KS == 4) {
            // partial sums of the other waves' rows to LDS, by row and writer
            f32x4 *pw = part + ((s & 1) * MT + wm) * RW * 4 * 64 + kh * 64 + lane;
#pragma unroll
            for (int r = 0; r < RW; ++r)
                if (r != kh) pw[r * 4 * 64] = acc[P][r];
            out[0] = kh == 0 ? acc[P][0] : kh == 1 ? acc[P][1] : kh == 2 ? acc[P][2] : acc[P][3];
        } else {
#pragma unroll
            for (int i = 0; i < RS; ++i) out[i] = acc[P][i];
        }
        if (s + 1 < nsteps) store_plane((s + 1) & 1, zb + s, R);
        if (s + 2 < nsteps) load_plane(zb + s + 1, R);
        lds_barrier();
        if constexpr (KS == 2) {
            const f32x4 *pr = part + ((s & 1) * MT + wm) * RW * 64 + lane;
#pragma unroll
            for (int i = 0; i < RS; ++i) out[i] += pr[(2 * i + kh) * 64];
        } else if constexpr (KS == 4) {
            const f32x4 *pr = part + (((s & 1) * MT + wm) * RW + kh) * 4 * 64 + lane;
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (w != kh) out[0] += pr[w * 64];
        }
        const int oz = zb + s - 2;
        if constexpr (PLAIN) {
            const unsigned pofs = (unsigned)(s - 2) * pbytes;
#pragma unroll
            for (int i = 0; i < RS; ++i) {
                f32x4 v = out[i];
                if constexpr (RELU) {
                    v.x = fmaxf(v.x, 0.f), v.y = fmaxf(v.y, 0.f);
                    v.z = fmaxf(v.z, 0.f), v.w = fmaxf(v.w, 0.f);
                }
                u32x2 st;
                st.x = pk_bf16(v.x, v.y);
                st.y = pk_bf16(v.z, v.w);
                __builtin_amdgcn_raw_buffer_store_b64(st, dst, (s >= 2 && rok[i]) ? roff[i] + pofs : 0x80000000u, 0, 0);
            }
        } else if (s >= 2) {
#pragma unroll
            for (int i = 0; i < RS; ++i) {
                const int oy = y0 + wr * RW + KS * i + kh;
                if (ox < a.onx && oy < a.ony)
                    store4b(a, ((size_t)oz * a.ony + oy) * a.onx + ox, mo + grp * 4, out[i], zero4);
            }
        }
    };
    for (int s = 0; s < nsteps; s += 3) {
        step(std::integral_constant<int, 0>{}, s);
        if (s + 1 < nsteps) step(std::integral_constant<int, 1>{}, s + 1);
        if (s + 2 < nsteps) step(std::integral_constant<int, 2>{}, s + 2);
    }
}

// ----------------------------------------------------------------- wgrad
// dW[co][t][ci] = sum_q G(q, t)[co] X(q, t)[ci] with
//   SAME3: q over the output grid, G = g[q],      X = x[q + o_t]
//   DOWN2: q over the coarse output, G = g[q],    X = x[2q + t]
//   UP2  : q over the coarse input,  G = g[2q+t], X = x[q]
// as D[co][ci] += A[co][q] B[q][ci] with 32 cells q per MFMA.  Block:
// input-channel tile blockIdx.x (16 channels) x cell slice blockIdx.y;
// wave w owns taps w, w+4, ...  Each block writes its partial sums.
template <int GEOM, int MT>
__global__ __launch_bounds__(256) void wgrad_k(WgradArgs a, int steps_per_slice) {
    constexpr int T = GEOM == G_SAME3 ? 27 : 8;
    constexpr int TW = (T + 3) / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int cout = MT * 16;
    const int ci = blockIdx.x * 16 + col;
    const bool ciok = ci < cin;
    const bf16_t *xs;
    int cs, cl;
    if (ci < a.ca) {
        xs = a.xA, cs = a.ca, cl = ci;
    } else {
        xs = a.xB, cs = a.cb, cl = ci - a.ca;
    }
    unsigned qnx, qny, qnz;
    if (GEOM == G_UP2) {
        qnx = a.xnx, qny = a.xny, qnz = a.xnz;
    } else {
        qnx = a.gnx, qny = a.gny, qnz = a.gnz;
    }
    const unsigned qplane = qnx * qny;
    const unsigned nq = qplane * qnz;
    const unsigned nsteps = (nq + 31) / 32;
    const unsigned st0 = blockIdx.y * (unsigned)steps_per_slice;
    const unsigned st1 = min(st0 + (unsigned)steps_per_slice, nsteps);

    f32x4 acc[MT][TW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < TW; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (unsigned step = st0; step < st1; ++step) {
        int qx[8], qy[8], qz[8];
        bool qok[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned q = step * 32 + grp * 8 + j;
            qok[j] = q < nq;
            const unsigned qq = qok[j] ? q : 0;
            const unsigned z = qq / qplane, r = qq - z * qplane;
            const unsigned yy = r / qnx;
            qz[j] = z, qy[j] = yy, qx[j] = r - yy * qnx;
        }
        u32x4 A[MT], B;
        if (GEOM != G_UP2) {
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                unsigned e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const size_t q = ((size_t)qz[j] * qny + qy[j]) * qnx + qx[j];
                    e[j] = qok[j] ? a.g[q * cout + m * 16 + col] : 0u;
                }
                A[m] = pack8(e);
            }
        } else {
            unsigned e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const size_t q = ((size_t)qz[j] * qny + qy[j]) * qnx + qx[j];
                e[j] = (qok[j] && ciok) ? xs[q * cs + cl] : 0u;
            }
            B = pack8(e);
        }
#pragma unroll
        for (int tw = 0; tw < TW; ++tw) {
            const int t = wave + 4 * tw;
            if (t >= T) break;
            if (GEOM == G_SAME3) {
                const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                unsigned e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int sx = qx[j] + dx, sy = qy[j] + dy, sz = qz[j] + dz;
                    const bool ok = qok[j] && ciok && sx >= 0 && sx < a.xnx && sy >= 0 && sy < a.xny && sz >= 0 &&
                                    sz < a.xnz;
                    e[j] = ok ? xs[(((size_t)sz * a.xny + sy) * a.xnx + sx) * cs + cl] : 0u;
                }
                B = pack8(e);
            } else if (GEOM == G_DOWN2) {
                const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
                unsigned e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const size_t s = (((size_t)(2 * qz[j] + tz) * a.xny + 2 * qy[j] + ty) * a.xnx + 2 * qx[j] + tx);
                    e[j] = (qok[j] && ciok) ? xs[s * cs + cl] : 0u;
                }
                B = pack8(e);
            } else {
                const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    unsigned e[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const size_t s = (((size_t)(2 * qz[j] + tz) * a.gny + 2 * qy[j] + ty) * a.gnx + 2 * qx[j] + tx);
                        e[j] = qok[j] ? a.g[s * cout + m * 16 + col] : 0u;
                    }
                    A[m] = pack8(e);
                }
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m][tw] = mfma(A[m], B, acc[m][tw]);
        }
    }
    if (!ciok) return;
    float *P = a.partials + (size_t)blockIdx.y * cout * T * cin;
#pragma unroll
    for (int tw = 0; tw < TW; ++tw) {
        const int t = wave + 4 * tw;
        if (t >= T) break;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const float v[4] = {acc[m][tw].x, acc[m][tw].y, acc[m][tw].z, acc[m][tw].w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = m * 16 + grp * 4 + r;
                P[((size_t)co * T + t) * cin + ci] = v[r];
            }
        }
    }
}

// Weight gradient of a 3x3x3 convolution with both operands staged in LDS.
// Block: input-channel tile blockIdx.x (16 channels) x a contiguous range
// of 16x4x4 output tiles (blockIdx.y).  Per tile the input halo (18x6x6
// cells x 16 channels, zero outside the grid) and the output gradient
// (256 cells x COUT channels) are staged with 16-byte loads; each MFMA then
// reduces 32 cells of the tile, whose values the lanes gather from LDS
// (8 cells of one channel per lane).  Wave w owns taps w, w+4, ...
template <int MT>
__global__ __launch_bounds__(256) void wgrad3_lds_k(WgradArgs a, int tiles_per_block) {
    constexpr int COUT = MT * 16;
    constexpr int TW = 7;
    constexpr int HX = 18, HY = 6, HZ = 6, NV = HX * HY * HZ;
    constexpr int XS = 24;         // bf16 per staged input cell (16 channels + pad)
    constexpr int GS = COUT + 8;   // bf16 per staged gradient cell
    __shared__ __align__(16) bf16_t xt[NV * XS];
    __shared__ __align__(16) bf16_t gt[256 * GS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int cin = a.ca + a.cb;
    const int c0 = blockIdx.x * 16;
    const int ntx = (a.gnx + 15) / 16, nty = (a.gny + 3) / 4, ntz = (a.gnz + 3) / 4;
    const int ntiles = ntx * nty * ntz;
    const int tb0 = blockIdx.y * tiles_per_block, tb1 = min(tb0 + tiles_per_block, ntiles);
    const u32x4 zero = {0u, 0u, 0u, 0u};

    f32x4 acc[MT][TW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < TW; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int tb = tb0; tb < tb1; ++tb) {
        const int bx = tb % ntx, by = (tb / ntx) % nty, bz = tb / (ntx * nty);
        const int x0 = bx * 16, y0 = by * 4, z0 = bz * 4;
        __syncthreads();
        for (int i = threadIdx.x; i < NV * 2; i += 256) {
            const int v = i >> 1, q = i & 1;
            const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            const int c = c0 + q * 8;
            u32x4 val = zero;
            if (c < cin && gx >= 0 && gx < a.xnx && gy >= 0 && gy < a.xny && gz >= 0 && gz < a.xnz) {
                const size_t cell = ((size_t)gz * a.xny + gy) * a.xnx + gx;
                val = c < a.ca ? ld16(a.xA + cell * a.ca + c) : ld16(a.xB + cell * a.cb + (c - a.ca));
            }
            *reinterpret_cast<u32x4 *>(xt + v * XS + q * 8) = val;
        }
        for (int i = threadIdx.x; i < 256 * (COUT / 8); i += 256) {
            const int v = i / (COUT / 8), q = i % (COUT / 8);
            const int gx = x0 + (v & 15), gy = y0 + ((v >> 4) & 3), gz = z0 + (v >> 6);
            u32x4 val = zero;
            if (gx < a.gnx && gy < a.gny && gz < a.gnz)
                val = ld16(a.g + (((size_t)gz * a.gny + gy) * a.gnx + gx) * COUT + q * 8);
            *reinterpret_cast<u32x4 *>(gt + v * GS + q * 8) = val;
        }
        __syncthreads();
#pragma unroll 1
        for (int step = 0; step < 8; ++step) {
            const int row = step * 2 + (grp >> 1);   // 0..15 = (ly, lz)
            const int ly = row & 3, lz = row >> 2;
            const int lx0 = (grp & 1) * 8;
            u32x4 A[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                unsigned e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) e[j] = gt[(row * 16 + lx0 + j) * GS + m * 16 + col];
                A[m] = pack8(e);
            }
#pragma unroll
            for (int tw = 0; tw < TW; ++tw) {
                const int t = wave + 4 * tw;
                if (t >= 27) break;
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                const int base = ((lz + dz) * HY + (ly + dy)) * HX + lx0 + dx;
                unsigned e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) e[j] = xt[(base + j) * XS + col];
                const u32x4 B = pack8(e);
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[m][tw] = mfma(A[m], B, acc[m][tw]);
            }
        }
    }
    const int ci = c0 + col;
    if (ci >= cin) return;
    float *P = a.partials + (size_t)blockIdx.y * COUT * 27 * cin;
#pragma unroll
    for (int tw = 0; tw < TW; ++tw) {
        const int t = wave + 4 * tw;
        if (t >= 27) break;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const float v[4] = {acc[m][tw].x, acc[m][tw].y, acc[m][tw].z, acc[m][tw].w};
#pragma unroll
            for (int r = 0; r < 4; ++r) P[((size_t)(m * 16 + grp * 4 + r) * 27 + t) * cin + ci] = v[r];
        }
    }
}

// ------------------------------------------------------------ reductions
// Bias gradient: each thread keeps one 8-channel group (256 is a multiple
// of C/8) and reads 16 bytes per cell, so a block sweeps its cells with
// coalesced loads; the groups are then summed through LDS.
template <int C>
__global__ __launch_bounds__(256) void bias_grad_k(const bf16_t *g, unsigned cells, float *partials,
                                                   unsigned cells_per_slice) {
    constexpr int G8 = C / 8;
    __shared__ float red[256][9];
    const int tid = threadIdx.x;
    const unsigned v0 = blockIdx.x * cells_per_slice;
    const unsigned v1 = min(v0 + cells_per_slice, cells);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (v1 > v0) {
        const size_t k0 = (size_t)v0 * G8, k1 = (size_t)v1 * G8;
        for (size_t k = k0 + tid; k < k1; k += 256) {
            const u32x4 w = ld16(g + k * 8);
            s[0] += bf2f(w.x), s[1] += bf2f(w.x >> 16), s[2] += bf2f(w.y), s[3] += bf2f(w.y >> 16);
            s[4] += bf2f(w.z), s[5] += bf2f(w.z >> 16), s[6] += bf2f(w.w), s[7] += bf2f(w.w >> 16);
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[tid][e] = s[e];
    __syncthreads();
    if (tid < C) {
        const int grp = tid / 8, e = tid % 8;
        float t = 0.f;
        for (int k = grp; k < 256; k += G8) t += red[k][e];
        partials[(size_t)blockIdx.x * C + tid] = t;
    }
}

// First level of the partial-sum reduction: group blockIdx.y of `groups`
// sums its share of the slices (in slice order).
__global__ __launch_bounds__(256) void reduce1_k(const float *P, int nslice, int n, int stride, int groups,
                                                 float *out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int per = (nslice + groups - 1) / groups;
    const int j0 = blockIdx.y * per, j1 = min(j0 + per, nslice);
    float s = 0.f;
    for (int j = j0; j < j1; ++j) s += P[(size_t)j * stride + i];
    out[(size_t)blockIdx.y * n + i] = s;
}

__global__ __launch_bounds__(256) void reduce_k(const float *P, int nslice, int n, int stride, int cinp,
                                                int cin_real, float *out, int accumulate) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int ci = i % cinp;
    if (ci >= cin_real) return;
    float s = 0.f;
    for (int j = 0; j < nslice; ++j) s += P[(size_t)j * stride + i];
    const size_t o = (size_t)(i / cinp) * cin_real + ci;
    out[o] = accumulate ? out[o] + s : s;
}

// Blocks take chunks of 4096 values, 16 per thread, whose loads are all
// issued before the first comparison (an index past the end reads the last
// value again, which leaves the maximum unchanged).  At most 256 blocks, so
// that at most 256 atomics meet at the result.
__global__ __launch_bounds__(256) void maxabs_k(const double *x, size_t n, unsigned long long *out) {
    __shared__ double red[256];
    double m = 0.0;
    for (size_t b = (size_t)blockIdx.x * 4096; b < n; b += (size_t)gridDim.x * 4096) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const size_t i = b + k * 256 + threadIdx.x;
            v[k] = x[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) m = fmax(m, fabs(v[k]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    // non-negative doubles order like their bit patterns
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ __launch_bounds__(256) void prep_input_k(const double *s, size_t n, const double *sigma, bf16_t *x8) {
    const size_t i = blockIdx.x * 256ull + threadIdx.x;
    if (i >= n) return;
    const double sg = *sigma;
    const double v = sg > 0.0 ? s[i] / sg : s[i];
    u32x4 w = {f2bf((float)v), 0u, 0u, 0u};
    *reinterpret_cast<u32x4 *>(x8 + i * 8) = w;
}

__device__ __forceinline__ void load16ch(const bf16_t *a, size_t v, float (&x)[16]) {
    const u32x4 p0 = ld16(a + v * 16), p1 = ld16(a + v * 16 + 8);
    const unsigned w[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[2 * k] = bf2f(w[k]);
        x[2 * k + 1] = bf2f(w[k] >> 16);
    }
}

struct Coef3 {
    double c[3];
};

struct Grid3 {
    int nx, ny, nz;
};

// Blocks of the input-side kernels (first layer, head): 256 threads on a
// 64 x 4 tile of one z plane.  The scaled input x = s / sigma of the tile
// and its one-cell halo on planes z-1, z, z+1 is staged in LDS (0 outside
// the grid), optionally rounded to bfloat16.
constexpr int kInTX = 64, kInTY = 4;
struct InTile {
    float v[3][kInTY + 2][kInTX + 2];
};

// All of a thread's loads are issued (from clamped addresses) before the
// first value is scaled, so their latencies overlap.
__device__ __forceinline__ void stage_input(const double *s, Grid3 g, double sg, bool round_bf16, InTile &t) {
    const int x0 = blockIdx.x * kInTX, y0 = blockIdx.y * kInTY, z = blockIdx.z;
    constexpr int N = 3 * (kInTY + 2) * (kInTX + 2);
    constexpr int NI = (N + 255) / 256;
    double sv[NI];
    bool ok[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int hx = i % (kInTX + 2), r = i / (kInTX + 2);
        const int hy = r % (kInTY + 2), hz = r / (kInTY + 2);
        const int qx = x0 + hx - 1, qy = y0 + hy - 1, qz = z + hz - 1;
        ok[k] = i < N && qx >= 0 && qx < g.nx && qy >= 0 && qy < g.ny && qz >= 0 && qz < g.nz;
        const int cx = min(max(qx, 0), g.nx - 1), cy = min(max(qy, 0), g.ny - 1), cz = min(max(qz, 0), g.nz - 1);
        sv[k] = s[((size_t)cz * g.ny + cy) * g.nx + cx];
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= N) break;
        float v = (float)(sg > 0.0 ? sv[k] / sg : sv[k]);
        if (round_bf16) v = bf2f(f2bf(v));
        (&t.v[0][0][0])[i] = ok[k] ? v : 0.f;
    }
    __syncthreads();
}

// Features of the head at this thread's cell: c0b's 16 channels, then x at
// the 27 taps (from the staged tile).
__device__ __forceinline__ void head_features(const bf16_t *a, size_t v, const InTile &t, int lx, int ly,
                                              float (&f)[kHeadIn]) {
    float x16[16];
    load16ch(a, v, x16);
#pragma unroll
    for (int c = 0; c < 16; ++c) f[c] = x16[c];
#pragma unroll
    for (int q = 0; q < 27; ++q) f[16 + q] = t.v[q / 9][ly + (q / 3) % 3][lx + q % 3];
}

// Prediction head, marching along z: a block owns a 64 x 4 tile of kHeadZ
// planes.  x = s / sigma (FP32) of the tile and its one-cell halo sits in a
// ring of four LDS planes, each staged once: while plane z is predicted
// (taps on planes z-1, z, z+1), plane z+2 is written to the fourth slot,
// which the previous plane's barrier has freed.
constexpr int kHeadZ = 8;
__global__ __launch_bounds__(256) void head_predict_k(const bf16_t *a, const double *s, Grid3 g, const float *wh,
                                                      const float *bh, const double *sigma, Coef3 coef, double *g0,
                                                      double *g1, double *g2) {
    constexpr int PX = kInTX + 2, PY = kInTY + 2, NP = PX * PY;
    constexpr int NI = (NP + 255) / 256;
    __shared__ float ring[4][NP];
    const double sg = *sigma > 0.0 ? *sigma : 1.0;
    const int x0 = blockIdx.x * kInTX, y0 = blockIdx.y * kInTY, zb = blockIdx.z * kHeadZ;
    const int nzb = min(kHeadZ, g.nz - zb);
    // staging of a plane: cells i = threadIdx.x + 256 k of the halo tile,
    // loaded from clamped addresses (zero outside the grid)
    size_t soff[NI];
    bool sok[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int qx = x0 + i % PX - 1, qy = y0 + i / PX - 1;
        sok[k] = i < NP && qx >= 0 && qx < g.nx && qy >= 0 && qy < g.ny;
        soff[k] = (size_t)min(max(qy, 0), g.ny - 1) * g.nx + min(max(qx, 0), g.nx - 1);
    }
    const size_t plane = (size_t)g.nx * g.ny;
    auto load = [&](int z, double (&v)[NI]) {
        const double *p = s + (size_t)min(max(z, 0), g.nz - 1) * plane;
#pragma unroll
        for (int k = 0; k < NI; ++k) v[k] = p[soff[k]];
    };
    auto put = [&](int z, const double (&v)[NI]) {
        float *r = ring[(z - zb + 1) & 3];
        const bool zok = z >= 0 && z < g.nz;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int i = threadIdx.x + 256 * k;
            if (i < NP) r[i] = (zok && sok[k]) ? (float)(v[k] / sg) : 0.f;
        }
    };
    double v[NI];
    load(zb - 1, v);
    put(zb - 1, v);
    load(zb, v);
    put(zb, v);
    load(zb + 1, v);
    put(zb + 1, v);
    __syncthreads();

    const int lx = threadIdx.x % kInTX, ly = threadIdx.x / kInTX;
    const int px = x0 + lx, py = y0 + ly;
    const bool ok = px < g.nx && py < g.ny;
    const size_t c0 = (size_t)min(py, g.ny - 1) * g.nx + min(px, g.nx - 1);
    // the 16 channels of c0b at this thread's cell, loaded one plane ahead
    u32x4 q0 = ld16(a + ((size_t)zb * plane + c0) * 16), q1 = ld16(a + ((size_t)zb * plane + c0) * 16 + 8);
    for (int t = 0; t < nzb; ++t) {
        const int z = zb + t;
        if (t + 1 < nzb) load(z + 2, v);
        const size_t cell = (size_t)z * plane + c0;
        const size_t nxt = (size_t)min(z + 1, g.nz - 1) * plane + c0;
        const u32x4 n0 = ld16(a + nxt * 16), n1 = ld16(a + nxt * 16 + 8);
        float f[kHeadIn];
        {
            const unsigned w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                f[2 * k] = bf2f(w[k]);
                f[2 * k + 1] = bf2f(w[k] >> 16);
            }
        }
        q0 = n0, q1 = n1;
#pragma unroll
        for (int q = 0; q < 27; ++q)
            f[16 + q] = ring[(t + q / 9) & 3][(ly + (q / 3) % 3) * PX + lx + q % 3];
        float y[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float acc = bh[i];
#pragma unroll
            for (int c = 0; c < kHeadIn; ++c) acc = fmaf(wh[i * kHeadIn + c], f[c], acc);
            y[i] = acc;
        }
        if (ok) {
            g0[cell] = sg * coef.c[0] * (double)y[0];
            g1[cell] = sg * coef.c[1] * (double)y[1];
            g2[cell] = sg * coef.c[2] * (double)y[2];
        }
        if (t + 1 < nzb) put(z + 2, v);
        __syncthreads();
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(256) void head_train_k(const bf16_t *a, const double *s, Grid3 g, const float *wh,
                                                    const float *bh, const double *sigma, const float *t, bf16_t *ga,
                                                    float *partials) {
    __shared__ float red[4][kHeadRed];
    __shared__ InTile tile;
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    const double sg0 = *sigma > 0.0 ? *sigma : 1.0;
    stage_input(s, g, sg0, false, tile);
    const int lx = threadIdx.x % kInTX, ly = threadIdx.x / kInTX;
    const int px = blockIdx.x * kInTX + lx, py = blockIdx.y * kInTY + ly, pz = blockIdx.z;
    const bool ok = px < g.nx && py < g.ny;
    const size_t v = ok ? ((size_t)pz * g.ny + py) * g.nx + px : 0;
    float f[kHeadIn], gy[3], sse = 0.f;
    if (ok) {
        head_features(a, v, tile, lx, ly, f);
        const float k = 2.f / (3.f * (float)n);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float acc = bh[i];
#pragma unroll
            for (int c = 0; c < kHeadIn; ++c) acc = fmaf(wh[i * kHeadIn + c], f[c], acc);
            const float d = acc - t[v * 3 + i];
            sse = fmaf(d, d, sse);
            gy[i] = k * d;
        }
        unsigned w[8];
#pragma unroll
        for (int c = 0; c < 16; c += 2) {
            float q0 = wh[c] * gy[0] + wh[kHeadIn + c] * gy[1] + wh[2 * kHeadIn + c] * gy[2];
            float q1 = wh[c + 1] * gy[0] + wh[kHeadIn + c + 1] * gy[1] + wh[2 * kHeadIn + c + 1] * gy[2];
            if (!(f[c] > 0.f)) q0 = 0.f;
            if (!(f[c + 1] > 0.f)) q1 = 0.f;
            w[c / 2] = f2bf(q0) | (f2bf(q1) << 16);
        }
        *reinterpret_cast<u32x4 *>(ga + v * 16) = u32x4{w[0], w[1], w[2], w[3]};
        *reinterpret_cast<u32x4 *>(ga + v * 16 + 8) = u32x4{w[4], w[5], w[6], w[7]};
    } else {
#pragma unroll
        for (int c = 0; c < kHeadIn; ++c) f[c] = 0.f;
        gy[0] = gy[1] = gy[2] = 0.f;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int c = 0; c < kHeadIn; ++c) {
            const float r = wave_sum(gy[i] * f[c]);
            if (lane == 0) red[wave][i * kHeadIn + c] = r;
        }
        const float r = wave_sum(gy[i]);
        if (lane == 0) red[wave][3 * kHeadIn + i] = r;
    }
    const float r = wave_sum(sse);
    if (lane == 0) red[wave][kHeadRed - 1] = r;
    __syncthreads();
    const size_t bid = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
    for (int k = threadIdx.x; k < kHeadRed; k += 256)
        partials[bid * kHeadRed + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
}

__global__ __launch_bounds__(256) void make_target_k(const double *p0, const double *p1, const double *p2, size_t n,
                                                     Coef3 k2, Coef3 scale, const double *sigma, float *t,
                                                     unsigned *maxbits) {
    const size_t v = blockIdx.x * 256ull + threadIdx.x;
    const double sg = *sigma > 0.0 ? *sigma : 1.0;
    float m[3] = {0.f, 0.f, 0.f};
    if (v < n) {
        const double ps[3] = {p0[v], p1[v], p2[v]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float tv = (float)(k2.c[i] * ps[i] / (sg * scale.c[i]));
            t[v * 3 + i] = tv;
            m[i] = fabsf(tv);
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float r = m[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r = fmaxf(r, __shfl_xor(r, o, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(maxbits + i, __float_as_uint(r));
    }
}

__global__ __launch_bounds__(256) void adam_k(float *theta, float *m, float *v, const float *g, size_t n, float gscale,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
    const size_t i = blockIdx.x * 256ull + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void pack_fwd_k(const float *W, int cout, int T, int cin, int cinp, bf16_t *wf) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= cout * T * cinp) return;
    const int ci = i % cinp, ct = i / cinp;
    wf[i] = ci < cin ? (bf16_t)f2bf(W[(size_t)ct * cin + ci]) : (bf16_t)0;
}

__global__ __launch_bounds__(256) void pack_bwd_k(const float *W, int cout, int T, int cin, int mirror, bf16_t *wd) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= cout * T * cin) return;
    // wd[ci][t'][co]
    const int co = i % cout, r = i / cout, tp = r % T, ci = r / T;
    const int t = mirror ? T - 1 - tp : tp;
    wd[i] = (bf16_t)f2bf(W[((size_t)co * T + t) * cin + ci]);
}

__global__ __launch_bounds__(256) void fill_zero_k(unsigned *p, size_t nw) {
    for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < nw; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

__global__ __launch_bounds__(256) void bf16_to_f32_k(const bf16_t *s, float *d, size_t n) {
    const size_t i = blockIdx.x * 256ull + threadIdx.x;
    if (i < n) d[i] = bf2f(s[i]);
}

inline unsigned nblk(size_t n) { return (unsigned)((n + 255) / 256); }

template <int GEOM, int COUT>
hipError_t conv_launch(hipStream_t s, const ConvArgs &a) {
    constexpr int NT = COUT >= 128 ? 2 : 4;
    int tnx = a.onx, tny = a.ony, tnz = a.onz;
    if (GEOM == G_UP2) tnx = a.inx, tny = a.iny, tnz = a.inz;
    dim3 grid((tnx + 15) / 16, (tny + 3) / 4, ((tnz + NT - 1) / NT) * (GEOM == G_UP2 ? 8 : 1));
    conv_k<GEOM, COUT, NT><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int COUT, int CC, int RY, int RZ>
hipError_t lds_launch(hipStream_t s, const ConvArgs &a) {
    const int nb = ((a.onx + 15) / 16) * ((a.ony + RY - 1) / RY) * ((a.onz + RZ - 1) / RZ);
    conv3_lds_k<COUT, CC, RY, RZ><<<nb, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int COUT, int CC, int RY, int RZ>
hipError_t reg_launch(hipStream_t s, const ConvArgs &a) {
    constexpr int WM = COUT >= 64 ? 4 : COUT / 16;
    const int nb = ((a.onx + 15) / 16) * ((a.ony + RY - 1) / RY) * ((a.onz + RZ - 1) / RZ);
    conv3_reg_k<COUT, CC, RY, RZ, WM><<<nb, 256, 0, s>>>(a);
    return hipGetLastError();
}

// Staged-tile kernels, for the channel counts the z-marching kernel does
// not take (128 input or output channels, 64 -> 16).  Tile: 16 x 4 x 4
// cells on grids with enough tiles to fill the chip, 16 x 2 x 2 on small
// grids.  With 32 or 64 output channels the weights of a wave stay in
// registers (conv3_reg_k); with 16 and 128 conv3_lds_k keeps more waves in
// flight.
template <int COUT, int CC>
hipError_t lds_tile(hipStream_t s, const ConvArgs &a) {
    const long tiles44 = (long)((a.onx + 15) / 16) * ((a.ony + 3) / 4) * ((a.onz + 3) / 4);
    if constexpr (COUT == 32 || COUT == 64) {
        if (tiles44 >= 1024) return reg_launch<COUT, CC, 4, 4>(s, a);
        return reg_launch<COUT, CC, 2, 2>(s, a);
    } else {
        if (tiles44 >= 1024) return lds_launch<COUT, CC, 4, 4>(s, a);
        return lds_launch<COUT, CC, 2, 2>(s, a);
    }
}

// z-marching kernel: the block count is raised towards the number of
// blocks the chip holds at once (two per CU for 4 waves, one for 8) by
// splitting z into chunks.  Every chunk re-reads two halo planes; chunks of
// 4-wave blocks keep at least 8 output planes (shorter ones measured slower
// at 64^3 and 128^3), those of 8-wave blocks at least 2.  On grids of at
// most 32 planes 4-wave blocks aim at one block per CU with chunks of any
// length (64 -> 64 channels: 15.2 us at 32^3 with 4-plane chunks against
// 18.5 with 2 and 20.3 with 8; 9.5 us at 16^3 with 1-plane chunks).
template <int CIN, int MT, int KS>
hipError_t zm_launch(hipStream_t s, const ConvArgs &a) {
    constexpr int NWV = zm_waves<MT, KS>();
    constexpr int BY = 4 * (NWV / (MT * KS));
    const long ng = (a.da + a.db) / (16 * MT);  // output channel groups (blocks per tile)
    const long txy = (long)((a.onx + 15) / 16) * ((a.ony + BY - 1) / BY) * ng;
    const bool small = NWV == 4 && a.onz <= 32;
    const long want = ((small ? 256 : 512 * 4 / NWV) + txy - 1) / txy;
    int zc = (int)((a.onz + want - 1) / want);
    zc = std::max(zc, std::min(small ? 1 : NWV == 4 ? 8 : 2, a.onz));
    const long nb = txy * ((a.onz + zc - 1) / zc);
    const bool plain = !a.maskA && !a.maskB && !a.accA && !a.accB && a.db == 0 &&
                       (size_t)a.onx * a.ony * a.onz * a.da * sizeof(bf16_t) < (1ull << 31);
    if (plain && a.relu)
        conv3_zm_k<CIN, MT, KS, true, true><<<(unsigned)nb, 64 * NWV, 0, s>>>(a, zc);
    else if (plain)
        conv3_zm_k<CIN, MT, KS, true, false><<<(unsigned)nb, 64 * NWV, 0, s>>>(a, zc);
    else
        conv3_zm_k<CIN, MT, KS, false, false><<<(unsigned)nb, 64 * NWV, 0, s>>>(a, zc);
    return hipGetLastError();
}

template <int COUT>
hipError_t lds_cc(hipStream_t s, const ConvArgs &a) {
    const int cin = a.ca + a.cb;
    if constexpr (COUT == 16 || COUT == 32) {
        if (cin == 8) return zm_launch<8, COUT / 16, 1>(s, a);
        if (cin == 16) return zm_launch<16, COUT / 16, 1>(s, a);
        if (cin == 32) return zm_launch<32, COUT / 16, 1>(s, a);
    }
    if constexpr (COUT == 32 || COUT == 64) {
        // 64 -> 64: two blocks of 32 output channels per tile (4 waves each)
        // fill the small grids better than one 8-wave block
        if (cin == 64) return zm_launch<64, 2, 2>(s, a);
    }
    if constexpr (COUT == 64) {
        if (cin == 128) return zm_launch<128, 2, 4>(s, a);
    }
    if (cin == 8) return lds_tile<COUT, 8>(s, a);
    if (cin == 16) return lds_tile<COUT, 16>(s, a);
    if (cin % 32 == 0 && a.ca % 8 == 0) return lds_tile<COUT, 32>(s, a);
    return hipErrorInvalidValue;
}

hipError_t conv_same3(hipStream_t s, const ConvArgs &a) {
    if (a.inx != a.onx || a.iny != a.ony || a.inz != a.onz) return hipErrorInvalidValue;
    switch (a.da + a.db) {
        case 16: return lds_cc<16>(s, a);
        case 32: return lds_cc<32>(s, a);
        case 64: return lds_cc<64>(s, a);
        case 128: return lds_cc<128>(s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int GEOM>
hipError_t conv_geom(hipStream_t s, const ConvArgs &a) {
    switch (a.da + a.db) {
        case 16: return conv_launch<GEOM, 16>(s, a);
        case 32: return conv_launch<GEOM, 32>(s, a);
        case 64: return conv_launch<GEOM, 64>(s, a);
        case 128: return conv_launch<GEOM, 128>(s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t wgrad_same3(hipStream_t s, const WgradArgs &a) {
    const int cin = a.ca + a.cb;
    const int ntiles = ((a.gnx + 15) / 16) * ((a.gny + 3) / 4) * ((a.gnz + 3) / 4);
    const int tpb = (ntiles + a.nslice - 1) / a.nslice;
    dim3 grid((cin + 15) / 16, a.nslice);
    switch (a.cout) {
        case 16: wgrad3_lds_k<1><<<grid, 256, 0, s>>>(a, tpb); break;
        case 32: wgrad3_lds_k<2><<<grid, 256, 0, s>>>(a, tpb); break;
        case 64: wgrad3_lds_k<4><<<grid, 256, 0, s>>>(a, tpb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int GEOM>
hipError_t wgrad_geom(hipStream_t s, const WgradArgs &a) {
    const int cin = a.ca + a.cb;
    size_t q = GEOM == G_UP2 ? (size_t)a.xnx * a.xny * a.xnz : (size_t)a.gnx * a.gny * a.gnz;
    const unsigned nsteps = (unsigned)((q + 31) / 32);
    const int sps = (int)((nsteps + a.nslice - 1) / a.nslice);
    dim3 grid((cin + 15) / 16, a.nslice);
    switch (a.cout) {
        case 16: wgrad_k<GEOM, 1><<<grid, 256, 0, s>>>(a, sps); break;
        case 32: wgrad_k<GEOM, 2><<<grid, 256, 0, s>>>(a, sps); break;
        case 64: wgrad_k<GEOM, 4><<<grid, 256, 0, s>>>(a, sps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t conv(hipStream_t s, int geom, const ConvArgs &a) {
    if ((a.ca & 7) || (a.cb & 7) || (a.da & 3) || (a.db & 3)) return hipErrorInvalidValue;
    switch (geom) {
        case G_SAME3: return conv_same3(s, a);
        case G_DOWN2: {
            const int cin = a.ca + a.cb, cout = a.da + a.db;
            if ((cin == 16 || cin == 32 || cin == 64) && (cout == 32 || cout == 64) && a.inx == 2 * a.onx &&
                a.iny == 2 * a.ony && a.inz == 2 * a.onz) {
                constexpr int NT = 2;
                const dim3 grid((a.onx + 15) / 16, a.ony, (a.onz + NT - 1) / NT);
                const int key = cin * 1000 + cout;
                switch (key) {
                    case 16032: down2_k<2, NT, 1><<<grid, 256, 0, s>>>(a); break;
                    case 16064: down2_k<4, NT, 1><<<grid, 256, 0, s>>>(a); break;
                    case 32032: down2_k<2, NT, 2><<<grid, 256, 0, s>>>(a); break;
                    case 32064: down2_k<4, NT, 2><<<grid, 256, 0, s>>>(a); break;
                    case 64032: down2_k<2, NT, 4><<<grid, 256, 0, s>>>(a); break;
                    default: down2_k<4, NT, 4><<<grid, 256, 0, s>>>(a); break;
                }
                return hipGetLastError();
            }
            return conv_geom<G_DOWN2>(s, a);
        }
        case G_UP2: {
            const int cin = a.ca + a.cb, cout = a.da + a.db;
            if ((cin == 32 || cin == 64) && (cout == 16 || cout == 32 || cout == 64) && a.onx == 2 * a.inx &&
                a.ony == 2 * a.iny && a.onz == 2 * a.inz) {
                // 4 coarse planes per block where that still leaves 512 blocks (32 -> 16 to
                // 128^3: 20.2 us against 22.4 for 2), 2 on smaller grids (64 -> 64 from 16^3:
                // 10.1 us against 15.6 for 4)
                auto go = [&](auto ntc) {
                    constexpr int NT = decltype(ntc)::value;
                    const dim3 grid((a.inx + 15) / 16, a.iny, (a.inz + NT - 1) / NT);
                    switch (cin * 1000 + cout) {
                        case 32016: up2_k<1, NT, 1><<<grid, 256, 0, s>>>(a); break;
                        case 32032: up2_k<2, NT, 1><<<grid, 256, 0, s>>>(a); break;
                        case 32064: up2_k<4, NT, 1><<<grid, 256, 0, s>>>(a); break;
                        case 64016: up2_k<1, NT, 2><<<grid, 256, 0, s>>>(a); break;
                        case 64032: up2_k<2, NT, 2><<<grid, 256, 0, s>>>(a); break;
                        default: up2_k<4, NT, 2><<<grid, 256, 0, s>>>(a); break;
                    }
                };
                if ((long)((a.inx + 15) / 16) * a.iny * ((a.inz + 3) / 4) >= 512)
                    go(std::integral_constant<int, 4>{});
                else
                    go(std::integral_constant<int, 2>{});
                return hipGetLastError();
            }
            return conv_geom<G_UP2>(s, a);
        }
        default: return hipErrorInvalidValue;
    }
}

int wgrad_slices(int geom, int qx, int qy, int qz, int cin, int cout, size_t max_floats) {
    // work units: 16x4x4 tiles (SAME3) or steps of 32 cells
    const int nsteps = geom == G_SAME3 ? ((qx + 15) / 16) * ((qy + 3) / 4) * ((qz + 3) / 4)
                                       : (int)(((size_t)qx * qy * qz + 31) / 32);
    const int ctiles = (cin + 15) / 16;
    int ns = 1024 / ctiles;
    if (ns < 1) ns = 1;
    if (ns > nsteps) ns = nsteps;
    const size_t per = (size_t)cout * geom_taps(geom) * cin;
    while (ns > 1 && (size_t)ns * per > max_floats) ns /= 2;
    // every slice must own at least one step
    const int sps = (nsteps + ns - 1) / ns;
    return (nsteps + sps - 1) / sps;
}

hipError_t wgrad(hipStream_t s, int geom, const WgradArgs &a) {
    if ((a.ca & 7) || (a.cb & 7) || a.nslice < 1) return hipErrorInvalidValue;
    switch (geom) {
        case G_SAME3: return wgrad_same3(s, a);
        case G_DOWN2: return wgrad_geom<G_DOWN2>(s, a);
        case G_UP2: return wgrad_geom<G_UP2>(s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t bias_grad(hipStream_t s, const bf16_t *g, size_t cells, int c, float *partials, int nslice) {
    const unsigned cps = (unsigned)((cells + nslice - 1) / nslice);
    switch (c) {
        case 16: bias_grad_k<16><<<nslice, 256, 0, s>>>(g, (unsigned)cells, partials, cps); break;
        case 32: bias_grad_k<32><<<nslice, 256, 0, s>>>(g, (unsigned)cells, partials, cps); break;
        case 64: bias_grad_k<64><<<nslice, 256, 0, s>>>(g, (unsigned)cells, partials, cps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t reduce_partials(hipStream_t s, const float *partials, int nslice, int n, int stride, int cinp,
                           int cin_real, float *out, int accumulate, float *work) {
    if (nslice > kReduceGroups && work) {
        reduce1_k<<<dim3(nblk(n), kReduceGroups), 256, 0, s>>>(partials, nslice, n, stride, kReduceGroups, work);
        reduce_k<<<nblk(n), 256, 0, s>>>(work, kReduceGroups, n, n, cinp, cin_real, out, accumulate);
    } else {
        reduce_k<<<nblk(n), 256, 0, s>>>(partials, nslice, n, stride, cinp, cin_real, out, accumulate);
    }
    return hipGetLastError();
}

hipError_t maxabs(hipStream_t s, const double *x, size_t n, double *out) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>((n + 4095) / 4096, 256);
    maxabs_k<<<g, 256, 0, s>>>(x, n, reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t prep_input(hipStream_t s, const double *src, size_t n, const double *sigma, bf16_t *x8) {
    prep_input_k<<<nblk(n), 256, 0, s>>>(src, n, sigma, x8);
    return hipGetLastError();
}

inline dim3 in_grid(int nx, int ny, int nz) { return dim3((nx + kInTX - 1) / kInTX, (ny + kInTY - 1) / kInTY, nz); }

hipError_t head_predict(hipStream_t s, const bf16_t *a, const double *src, int nx, int ny, int nz, const float *wh,
                        const float *bh, const double *sigma, const double coef[3], double *g0, double *g1,
                        double *g2) {
    Coef3 c{{coef[0], coef[1], coef[2]}};
    const dim3 grid((nx + kInTX - 1) / kInTX, (ny + kInTY - 1) / kInTY, (nz + kHeadZ - 1) / kHeadZ);
    head_predict_k<<<grid, 256, 0, s>>>(a, src, Grid3{nx, ny, nz}, wh, bh, sigma, c, g0, g1, g2);
    return hipGetLastError();
}

int head_train_blocks(int nx, int ny, int nz) {
    const dim3 g = in_grid(nx, ny, nz);
    return (int)(g.x * g.y * g.z);
}

hipError_t head_train(hipStream_t s, const bf16_t *a, const double *src, int nx, int ny, int nz, const float *wh,
                      const float *bh, const double *sigma, const float *t, bf16_t *ga, float *partials) {
    head_train_k<<<in_grid(nx, ny, nz), 256, 0, s>>>(a, src, Grid3{nx, ny, nz}, wh, bh, sigma, t, ga, partials);
    return hipGetLastError();
}

hipError_t make_target(hipStream_t s, const double *psi0, const double *psi1, const double *psi2, size_t n,
                       const double kappa2[3], const double scale[3], const double *sigma, float *t,
                       unsigned *maxbits) {
    Coef3 k{{kappa2[0], kappa2[1], kappa2[2]}}, c{{scale[0], scale[1], scale[2]}};
    make_target_k<<<nblk(n), 256, 0, s>>>(psi0, psi1, psi2, n, k, c, sigma, t, maxbits);
    return hipGetLastError();
}

hipError_t adam(hipStream_t s, float *theta, float *m, float *v, const float *g, size_t n, float gscale, float lr,
                float beta1, float beta2, float eps, int step) {
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    adam_k<<<nblk(n), 256, 0, s>>>(theta, m, v, g, n, gscale, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t pack_weights(hipStream_t s, int geom, const float *W, int cout, int cin, int cinp, bf16_t *wf,
                        bf16_t *wd) {
    const int T = geom_taps(geom);
    pack_fwd_k<<<nblk((size_t)cout * T * cinp), 256, 0, s>>>(W, cout, T, cin, cinp, wf);
    if (wd) pack_bwd_k<<<nblk((size_t)cout * T * cin), 256, 0, s>>>(W, cout, T, cin, geom == G_SAME3, wd);
    return hipGetLastError();
}

hipError_t fill_zero(hipStream_t s, void *p, size_t bytes) {
    if (bytes & 3) return hipErrorInvalidValue;
    const size_t nw = bytes / 4;
    unsigned g = nblk(nw);
    if (g > 4096) g = 4096;
    if (g == 0) return hipSuccess;
    fill_zero_k<<<g, 256, 0, s>>>(static_cast<unsigned *>(p), nw);
    return hipGetLastError();
}

hipError_t bf16_to_f32(hipStream_t s, const bf16_t *src, float *dst, size_t n) {
    bf16_to_f32_k<<<nblk(n), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

}  // namespace nn
