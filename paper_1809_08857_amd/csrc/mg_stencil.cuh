// Device templates of the cell-centred stencil kernels (smoother, residual,
// restriction, prolongation, norms).  Included by one translation unit per
// storage type.
//
// Operator of every level (second-order cell-centred finite volumes):
//   (A u)_P = a u_P + h^-2 [ sum_interior beta_f (u_P - u_N)
//                            + sum_Dirichlet 2 beta_b (u_P - g) ]
// with beta_f the harmonic mean of the cell coefficients (finest level),
// a stored face array (coarser levels) or 1, and beta_b the boundary
// cell's own coefficient (or the stored boundary face).  A Neumann face
// contributes nothing.  In terms of the per-cell sums
//   off = sum_interior beta_f u_N + sum_Dirichlet 2 beta_b g
//   dg  = sum_interior beta_f     + sum_Dirichlet 2 beta_b
// a Gauss-Seidel update is u_P = (h^2 b_P + off) / (a h^2 + dg) and the
// residual is b_P - a u_P - h^-2 (dg u_P - off).
#pragma once

#include <type_traits>

#include "mg_internal.h"

namespace mg {

// Prefetch depth of the column-pair kernels (planes in flight per array):
// two planes for FP64; five for the 4- and 2-byte storage types, whose
// planes carry half or a quarter of the bytes.  An odd depth makes the
// plane ring (PD + 3 slots) even, which fixes the red/black parity of each
// unrolled step (FP64 measured no faster with three planes and the fixed
// parity than with two).  The batched engine's kernels keep two.
constexpr int kSmoothPD = 2;
template <class T> constexpr int kSmoothPDOf = sizeof(T) == 8 ? 2 : 5;

template <class T> struct Num;
template <> struct Num<double> {
    using C = double;
    __device__ static __forceinline__ C ld(double v) { return v; }
    __device__ static __forceinline__ double cv(C v) { return v; }
};
template <> struct Num<float> {
    using C = float;
    __device__ static __forceinline__ C ld(float v) { return v; }
    __device__ static __forceinline__ float cv(C v) { return v; }
};
template <> struct Num<bf16> {
    using C = float;
    __device__ static __forceinline__ C ld(bf16 v) { return __bfloat162float(v); }
    __device__ static __forceinline__ bf16 cv(C v) { return __float2bfloat16(v); }
};

// Storage type of the coefficients (cell eps, stored faces) that go with
// fields stored in T: BF16 fields keep FP32 coefficients, whose rounding
// would otherwise perturb the inner operator enough to cost outer steps.
template <class T> struct CoefStore { using type = T; };
template <> struct CoefStore<bf16> { using type = float; };
template <class T> using coef_t = typename CoefStore<T>::type;

template <class T> struct alignas(2 * sizeof(T)) Pair {
    T v[2];
};

// Load two adjacent elements with one memory instruction.  The access goes
// through an integer (vector) of the pair's width: a load of the struct
// itself is split into its two elements early in compilation, and where a
// branch beside it loads the same first element, the two no longer combine.
template <class T> __device__ __forceinline__ Pair<T> ld_wide(const void *p) {
    if constexpr (sizeof(T) == 8) {
        typedef unsigned long long w_t __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(Pair<T>, *reinterpret_cast<const w_t *>(p));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(Pair<T>, *reinterpret_cast<const unsigned long long *>(p));
    } else {
        static_assert(sizeof(T) == 2, "element of 2, 4 or 8 bytes");
        return __builtin_bit_cast(Pair<T>, *reinterpret_cast<const unsigned int *>(p));
    }
}

// A lane's byte offset within plane k, opaque to loop-invariant code
// motion.  Each access is then formed as a uniform plane base (scalar
// registers) plus a 32-bit lane offset, the saddr form of the global memory
// instructions; otherwise the array base is folded into a 64-bit per-lane
// address that is advanced with a 64-bit multiply-add at every plane.  The
// statement emits no instruction.
__device__ __forceinline__ uint32_t lane_at(uint32_t off, int k) {
    asm("" : "+v"(off) : "s"(k));
    return off;
}

// Store a pair with the non-temporal hint: the sweep's output is not read
// again by the same launch, so it should not displace the halo planes that
// neighbouring workgroups are still reading from L2.
template <class T> __device__ __forceinline__ void store_pair_nt(T *p, T a, T b) {
    if constexpr (std::is_same<T, double>::value) {
        typedef double v2 __attribute__((ext_vector_type(2)));
        v2 w;
        w.x = a;
        w.y = b;
        __builtin_nontemporal_store(w, reinterpret_cast<v2 *>(p));
    } else if constexpr (std::is_same<T, float>::value) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        v2 w;
        w.x = a;
        w.y = b;
        __builtin_nontemporal_store(w, reinterpret_cast<v2 *>(p));
    } else {
        static_assert(sizeof(T) == 2, "16-bit storage type");
        uint16_t ua, ub;
        __builtin_memcpy(&ua, &a, 2);
        __builtin_memcpy(&ub, &b, 2);
        __builtin_nontemporal_store((uint32_t)ua | ((uint32_t)ub << 16), reinterpret_cast<uint32_t *>(p));
    }
}

// Hardware hands workgroup w to XCD (w mod 8).  Give every XCD one
// contiguous range of tiles so that tiles sharing halo planes share an L2.
__device__ __forceinline__ int xcd_remap(int w, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X;
    const int xcd = w % X, pos = w / X;
    return xcd * q + min(xcd, r) + pos;
}

// Quotients of the stencil kernels: the hardware reciprocal refined by one
// Newton step, then one multiply.  The divisors here are sums of positive
// coefficients (never zero, infinite or denormal), so the special cases a
// full IEEE division handles cannot occur.  v_rcp_f64 is within about 2^-24
// of 1/s (2.6e8 ulp over 4M random divisors of exponents -300..300); one
// step squares that relative error, leaving the reciprocal within 11 ulp
// (a second step rounds it exactly, at two more FMAs); FP32's v_rcp_f32 is
// within about an ulp before its step.
__device__ __forceinline__ double rcp_nr(double s) {
    const double r = __builtin_amdgcn_rcp(s);
    return fma(r, fma(-s, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float s) {
    float r = __builtin_amdgcn_rcpf(s);
    return fmaf(r, fmaf(-s, r, 1.0f), r);
}
template <class C> __device__ __forceinline__ C qdiv(C n, C d) { return n * rcp_nr(d); }

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// fences global memory, which makes every wave wait for all of its
// outstanding global loads (the register prefetch) at each barrier; the
// stencil kernels never exchange data through global memory inside a
// workgroup, so an LDS-scoped fence is sufficient.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------
// Element-wise kernels run on "bricks": blockDim (BX, BY) covers BX cells
// (or coarse cells / pairs) along x and BY rows along y, blockIdx.z a run
// of kz planes.  No integer division by grid sizes is needed.
struct Brick {
    int kz;  // planes per block along z
};

__device__ __forceinline__ int brick_id() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ int brick_count() { return gridDim.x * gridDim.y * gridDim.z; }

// ---------------------------------------------------------------------
// Prolongation + correction: one thread per pair of fine cells (2I, 2I+1)
// sharing a coarse x index.
// ---------------------------------------------------------------------
// Deterministic reduction of two FP64 sums in two launches.  Each workgroup
// of the reducing kernel stores its partial pair (reduce2_finish); a
// one-workgroup kernel launched next on the same stream (reduce2_final_k)
// sums the partials in a fixed order, writes ws.result[slot] (and
// ws.result[bslot]) and, if done != nullptr, sets *done = 1 when the first
// sum is <= rtol2 * result[ref_slot] (squared residual against squared
// right-hand side), else 0.  The kernel boundary orders the partial stores
// before the final sum: a last-workgroup-finishes scheme would need a
// device-scope fence in every workgroup, which writes back and invalidates
// the L2 of its XCD.
template <int NT>
__device__ __forceinline__ void reduce2_finish(double s0, double s1, const RedWs &ws, int slot, int bid) {
    __shared__ double sh[2][NT / 64];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_down(s0, o, 64);
        s1 += __shfl_down(s1, o, 64);
    }
    if (lane == 0) {
        sh[0][w] = s0;
        sh[1][w] = s1;
    }
    __syncthreads();
    if (tid == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int q = 0; q < NT / 64; ++q) {
            a0 += sh[0][q];
            a1 += sh[1][q];
        }
        double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
        part[2 * bid] = a0;
        part[2 * bid + 1] = a1;
    }
}

constexpr int kFinalThreads = 256;

// The final sum of reduce2_finish's partials (one workgroup of kFinalThreads).
__device__ __forceinline__ void reduce2_final_body(const RedWs &ws, int slot, int bslot, int nb, int ref_slot,
                                                   double rtol2, int *done) {
    constexpr int NT = kFinalThreads;
    __shared__ double sh[2][NT / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
    double a0 = 0.0, a1 = 0.0;
    for (int q = tid; q < nb; q += NT) {
        a0 += part[2 * q];
        a1 += part[2 * q + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_down(a0, o, 64);
        a1 += __shfl_down(a1, o, 64);
    }
    if (lane == 0) {
        sh[0][w] = a0;
        sh[1][w] = a1;
    }
    __syncthreads();
    if (tid == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int q = 0; q < NT / 64; ++q) {
            t0 += sh[0][q];
            t1 += sh[1][q];
        }
        ws.result[slot] = t0;
        if (bslot >= 0) ws.result[bslot] = t1;
        if (done) {
            // the reference may be the right-hand side norm reduced in this same pass
            const double ref = (bslot >= 0 && ref_slot == bslot) ? t1 : ws.result[ref_slot];
            *done = (t0 <= rtol2 * ref) ? 1 : 0;
        }
    }
}

// Face coefficient arrays (FACE mode), see mg_internal.h for the layout.
template <class T>
__device__ __forceinline__ typename Num<T>::C face_x(const T *bx, const Geo &G, int i, int j, int k) {
    return Num<T>::ld(bx[((size_t)k * G.ny + j) * (G.nx + 1) + i]);
}
template <class T>
__device__ __forceinline__ typename Num<T>::C face_y(const T *by, const Geo &G, int i, int j, int k) {
    return Num<T>::ld(by[((size_t)k * (G.ny + 1) + j) * G.nx + i]);
}
template <class T>
__device__ __forceinline__ typename Num<T>::C face_z(const T *bz, const Geo &G, int i, int j, int k) {
    return Num<T>::ld(bz[((size_t)k * G.ny + j) * G.nx + i]);
}

// Six-face sums (off, dg) of cell (i,j,k).  un(d), en(d), fb(d) give the
// neighbour value, neighbour cell coefficient and stored face coefficient
// in direction d = x-, x+, y-, y+, z-, z+; only the accessor matching MODE
// is used.  SAFE: the accessors may be evaluated for every d, also across
// the box boundary (LDS planes with a filled halo), so no branches are
// needed; otherwise they are only evaluated for faces inside the box.
// The sums live in locals (reference out-parameters that may alias would
// otherwise be kept in scratch memory).
template <class C, int MODE, bool SAFE = false, class UN, class EN, class FB>
__device__ __forceinline__ void six_faces(const Geo &G, int i, int j, int k, C eP, UN un, EN en,
                                          FB fb, C &off_out, C &dg_out) {
    C off = C(0), dg = C(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const bool in = d == 0   ? i > 0
                        : d == 1 ? i < G.nx - 1
                        : d == 2 ? j > 0
                        : d == 3 ? j < G.ny - 1
                        : d == 4 ? k > 0
                                 : k < G.nz - 1;
        const bool dir = ((G.bcmask >> d) & 1) != 0;
        C be_in, be_bd;
        if constexpr (MODE == COEF_CONST) {
            be_in = C(1);
            be_bd = C(1);
        } else if constexpr (MODE == COEF_CELL) {
            C eN = eP;
            if (SAFE || in) eN = en(d);
            be_in = qdiv(C(2) * eP * eN, eP + eN);
            be_bd = eP;
        } else {
            be_in = fb(d);
            be_bd = be_in;
        }
        C uN = C(0);
        if (SAFE || in) uN = un(d);
        const C bnd = dir ? C(2) * be_bd : C(0);
        off += in ? be_in * uN : bnd * C(G.g[d]);
        dg += in ? be_in : bnd;
    }
    off_out = off;
    dg_out = dg;
}

// Residual b - A u at cell (i,j,k), all operands read from global memory.
template <class T, int MODE>
__device__ __forceinline__ typename Num<T>::C resid_global(const T *__restrict__ u,
                                                           const T *__restrict__ b,
                                                           const coef_t<T> *__restrict__ eps,
                                                           const coef_t<T> *__restrict__ bx,
                                                           const coef_t<T> *__restrict__ by,
                                                           const coef_t<T> *__restrict__ bz, const Geo &G,
                                                           int i, int j, int k,
                                                           const double *__restrict__ dd = nullptr) {
    using N = Num<T>;
    using C = typename N::C;
    const size_t sy = (size_t)G.nx, sz = (size_t)G.nx * G.ny;
    const size_t p = (size_t)k * sz + (size_t)j * sy + i;
    auto nb = [&](int d) -> size_t {
        return d == 0 ? p - 1 : d == 1 ? p + 1 : d == 2 ? p - sy : d == 3 ? p + sy : d == 4 ? p - sz : p + sz;
    };
    C eP = C(1);
    if constexpr (MODE == COEF_CELL) eP = Num<coef_t<T>>::ld(eps[p]);
    C off, dg;
    six_faces<C, MODE>(
        G, i, j, k, eP, [&](int d) { return N::ld(u[nb(d)]); },
        [&](int d) { return Num<coef_t<T>>::ld(eps[nb(d)]); },
        [&](int d) {
            switch (d) {
                case 0: return face_x(bx, G, i, j, k);
                case 1: return face_x(bx, G, i + 1, j, k);
                case 2: return face_y(by, G, i, j, k);
                case 3: return face_y(by, G, i, j + 1, k);
                case 4: return face_z(bz, G, i, j, k);
                default: return face_z(bz, G, i, j, k + 1);
            }
        },
        off, dg);
    const C uP = N::ld(u[p]);
    C r = N::ld(b[p]) - C(G.a) * uP - C(G.ih2) * (dg * uP - off);
    if constexpr (MODE == COEF_FACED) r -= C(dd[p]) * uP;
    return r;
}

// ---------------------------------------------------------------------
// Fused red-black Gauss-Seidel sweep, column-pair form (out of place).
//
// A workgroup owns a TX x TY tile and marches up a chunk of z planes; each
// thread owns one pair of adjacent x-columns (x, x+1) of the tile grown by a
// 2-cell halo, so on every plane the pair holds exactly one red and one
// black cell.  At step k the pair's red cell on plane k is updated (tile +
// 1-cell ring) from old black values, and the black cell on plane k-1
// (tile only) from new red values.  Vertical neighbours never leave the
// thread's registers; in-plane neighbours are exchanged through LDS (a
// plane of old u and two planes of new red values; for cell coefficients
// also eps and the face planes).  u, b and the coefficients stream in PD
// planes ahead of use, so a wait only ever covers the oldest plane in
// flight.  Ring cells are recomputed by every tile that needs them, from
// the same old values, so tiles never wait for each other and the result
// equals a red sweep followed by a black sweep.  One body per coefficient
// kind: rbgs_const_body (beta = 1), rbgs_cell_body (cell eps, harmonic
// faces), rbgs_face_body (stored faces); rbgs_pair_body is the general
// stored-face form kept for the batched engine.
template <class T> struct SmoothArgs {
    const T *uin;
    T *uout;
    const T *b;
    const coef_t<T> *eps;
    const coef_t<T> *fbx, *fby, *fbz;
    Geo G;
    int cz, tiles_x, tiles_y, nblk;
    const int *done;
    const double *dd;  // COEF_FACED: per-cell extra diagonal
};

// LDS elements (of the compute type) used by one smoother workgroup:
// region planes of old u and of new red values (two), and for cell
// coefficients one plane of eps and three planes each of x and y faces.
template <int MODE, int TX, int TY> constexpr int smooth_lds() {
    return (MODE == COEF_CELL ? 10 : 3) * (TY + 4) * (TX + 4);
}

// Harmonic-mean face coefficient 2 a b / (a + b) of two cell coefficients.
// With a zero coefficient beyond a Neumann face it gives 0; with kBigCoef
// beyond a Dirichlet face it gives 2 eP to rounding (the ghost-cell term of
// that face) for every eP <= kMaxCellCoef, and never overflows.
template <class C> __device__ __forceinline__ C fma_c(C a, C b, C c) {
    if constexpr (sizeof(C) == 8) return fma(a, b, c);
    else return fmaf(a, b, c);
}
// Select between two values.  (A conditional over two lvalues selects an
// address, which keeps the variables in private memory.)
template <class C> __device__ __forceinline__ C csel(bool c, C a, C b) { return c ? a : b; }

template <class C> __device__ __forceinline__ C harm_face(C a, C b) {
    return qdiv<C>((a + a) * b, a + b);
}
// 2^400 (FP64) and 2^60 (FP32 compute of the low-precision copies, where
// the coefficients stay below 2^36 for a rounding-exact boundary term).
template <class C> constexpr C kBigCoef = sizeof(C) == 8 ? C(0x1p400) : C(0x1p60f);

// ---------------------------------------------------------------------
// The same sweep for cell coefficients (harmonic-mean faces).  Every face
// joins a red and a black cell, so each face coefficient is formed once per
// sweep and read by both of its cells: at step k the pair forms the x and
// y faces of plane k+1 (from its own eps and an LDS plane of eps) into one
// of three LDS face planes (plane k+1 being formed, plane k for the red
// cells, plane k-1 for the black cells) and the two vertical faces between
// planes k and k+1 in registers.  Box faces take no branches: an outside
// cell carries u = the boundary value of the box face it lies beyond and a
// coefficient (0 beyond a Neumann face, kBigCoef beyond a Dirichlet face)
// for which harm_face yields that face's term.
template <class T, int TX, int TY, bool ZIN, int PD, bool EVEN>
__device__ __forceinline__ void rbgs_cell_body(const SmoothArgs<T> &A, const int blk,
                                               typename Num<T>::C *smem) {
    using N = Num<T>;
    using C = typename N::C;
    constexpr int PXW = (TX + 4) / 2;  // pairs per region row
    constexpr int RX = TX + 4, RY = TY + 4, PL = RX * RY;
    C(*s_u)[RX] = reinterpret_cast<C(*)[RX]>(smem);                  // old u, plane k
    C(*s_e)[RX] = reinterpret_cast<C(*)[RX]>(smem + PL);             // eps, plane k+1
    C(*s_r)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + 2 * PL);  // new red u, by plane parity
    // s_fx[q][y][c]: face between cells c and c+1 of row y; s_fy[q][y][c]:
    // face between rows y and y+1 of column c; q = plane mod 3
    C(*s_fx)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + 4 * PL);
    C(*s_fy)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + 7 * PL);
    const T *__restrict__ uin = A.uin;
    T *__restrict__ uout = A.uout;
    const T *__restrict__ b = A.b;
    const coef_t<T> *__restrict__ eps = A.eps;
    const Geo &G = A.G;
    const int cz = A.cz, tiles_x = A.tiles_x, tiles_y = A.tiles_y;

    const int tid = threadIdx.x;
    const int tx = blk % tiles_x;
    const int rest = blk / tiles_x;
    const int ty = rest % tiles_y;
    const int tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const C h2 = C(G.h2), ah2 = C(G.ah2);

    const int ry = tid / PXW, pc = tid - ry * PXW;
    const int lx = 2 * pc;                  // LDS column of the pair's first cell
    const int x = lx - 2, y = ry - 2;       // tile coordinates of the pair
    const int gx = x0 + x, gy = y0 + y;     // global coordinates of its first cell
    const bool row_in = gy >= 0 && gy < ny;
    const bool c0_in = row_in && gx >= 0 && gx < nx;
    const bool c1_in = row_in && gx + 1 >= 0 && gx + 1 < nx;
    constexpr bool even_nx = EVEN;  // rows of even length: pairs never straddle a row
    const bool core = x >= 0 && x < TX && y >= 0 && y < TY;
    const size_t rowoff = (size_t)(row_in ? gy : 0) * nx;
    const int lx2 = min(lx + 2, RX - 2);    // next pair (clamped: its face is never read)
    const int ry1 = min(ry + 1, RY - 1);    // next row (clamped likewise)

    // values carried by cells outside the box: u = boundary value and the
    // face-encoding coefficient of the box face beyond which the cell lies
    // (x faces first; a cell outside in x and y is never read)
    const C big = kBigCoef<C>;
    auto side = [&](int c) -> int {
        const int g = gx + c;
        return g < 0 ? 0 : g >= nx ? 1 : gy < 0 ? 2 : gy >= ny ? 3 : 4;
    };
    auto bval = [&](int d) -> C {
        return d == 0 ? C(G.g[0]) : d == 1 ? C(G.g[1]) : d == 2 ? C(G.g[2]) : d == 3 ? C(G.g[3]) : C(0);
    };
    auto bcoef = [&](int d) -> C { return d < 4 && ((G.bcmask >> d) & 1) ? big : C(0); };
    const int sd0 = side(0), sd1 = side(1);
    const C gout0 = bval(sd0), gout1 = bval(sd1), eout0 = bcoef(sd0), eout1 = bcoef(sd1);
    const C gz_lo = C(G.g[4]), gz_hi = C(G.g[5]);
    const C ez_lo = ((G.bcmask >> 4) & 1) ? big : C(0), ez_hi = ((G.bcmask >> 5) & 1) ? big : C(0);

    // offsets (elements) of the pair's cells within a plane (0 outside the
    // box) and of plane k: loads and stores take a uniform plane base plus
    // a 32-bit lane offset, both scaled by the element size of the array
    // (the coefficients may be wider than the fields)
    const uint32_t le0 = (uint32_t)(c0_in ? rowoff + gx : 0);
    const uint32_t le1 = (uint32_t)(c1_in ? rowoff + gx + 1 : 0);
    auto plane_el = [&](int k) -> size_t { return (size_t)min(max(k, 0), nz - 1) * plane; };
    const uint32_t lb0 = le0 * (uint32_t)sizeof(T), lb1 = le1 * (uint32_t)sizeof(T);
    auto plane_at = [&](int k) -> size_t { return plane_el(k) * sizeof(T); };

    struct P2 { C v[2]; };
    P2 zero;
    zero.v[0] = zero.v[1] = C(0);
    // one pair of plane k (a plane outside the box reads the nearest one;
    // the caller masks what it uses)
    auto ld_pair = [&](const auto *__restrict__ a, int k) -> P2 {
        using A_ = std::remove_cv_t<std::remove_reference_t<decltype(*a)>>;
        constexpr uint32_t es = sizeof(A_);
        const char *pk = reinterpret_cast<const char *>(a) + plane_el(k) * es;
        P2 r;
        if (even_nx) {
            const Pair<A_> w = ld_wide<A_>(pk + lane_at(le0 * es, k));
            r.v[0] = Num<A_>::ld(w.v[0]);
            r.v[1] = Num<A_>::ld(w.v[1]);
        } else {
            r.v[0] = Num<A_>::ld(*reinterpret_cast<const A_ *>(pk + lane_at(le0 * es, k)));
            r.v[1] = Num<A_>::ld(*reinterpret_cast<const A_ *>(pk + lane_at(le1 * es, k)));
        }
        return r;
    };
    auto pick = [](const P2 &p, int c) -> C { return csel<C>(c, p.v[1], p.v[0]); };
    // cells outside the box take their boundary values; plane k outside the
    // box: the z face values (cells also outside in x or y are never read)
    auto mask = [&](P2 v, int k, C out0, C out1, C zlo, C zhi) -> P2 {
        const bool kin = k >= 0 && k < nz;
        const C zv = csel<C>(k < 0, zlo, zhi);
        P2 r;
        r.v[0] = csel<C>(kin && c0_in, v.v[0], csel<C>(kin, out0, zv));
        r.v[1] = csel<C>(kin && c1_in, v.v[1], csel<C>(kin, out1, zv));
        return r;
    };
    auto masku = [&](P2 v, int k) { return mask(v, k, gout0, gout1, gz_lo, gz_hi); };
    auto maske = [&](P2 v, int k) { return mask(v, k, eout0, eout1, ez_lo, ez_hi); };

    // A ring of R = PD + 3 plane slots for u, b and eps: plane p occupies
    // slot (p - z0 + 2) mod R from its load, PD steps before the step that
    // first reads it, until the step after its own.  The steps are unrolled
    // R at a time, so every slot index is a constant and no loaded value
    // moves between registers (such a move would wait for its load at
    // once).  u and eps are masked in place when their plane first becomes
    // the upper neighbour.  zA, zB, zC: the vertical faces of the pair
    // between planes k-2|k-1, k-1|k and k|k+1.
    static_assert(PD >= 1 && PD <= 5, "prefetch depth 1..5");
    constexpr int R = PD + 3;
    // parity of gy + k (which cell of the pair is red on plane k): with R
    // even it is the same for step J of every unrolled group, a per-lane
    // constant that needs no per-plane arithmetic
    const int pz = (gy + z0) & 1;
    auto par = [&](auto J, int k) -> int {
        if constexpr (R % 2 == 0) return pz ^ (decltype(J)::value & 1);
        else return (gy + k) & 1;
    };
    P2 su0, su1, su2, su3, su4, su5, su6, su7, sb0, sb1, sb2, sb3, sb4, sb5, sb6, sb7;
    P2 se0, se1, se2, se3, se4, se5, se6, se7;
    auto SU = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return su0; else if constexpr (v == 1) return su1;
        else if constexpr (v == 2) return su2; else if constexpr (v == 3) return su3;
        else if constexpr (v == 4) return su4; else if constexpr (v == 5) return su5;
        else if constexpr (v == 6) return su6; else return su7;
    };
    auto SB = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return sb0; else if constexpr (v == 1) return sb1;
        else if constexpr (v == 2) return sb2; else if constexpr (v == 3) return sb3;
        else if constexpr (v == 4) return sb4; else if constexpr (v == 5) return sb5;
        else if constexpr (v == 6) return sb6; else return sb7;
    };
    auto SE = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return se0; else if constexpr (v == 1) return se1;
        else if constexpr (v == 2) return se2; else if constexpr (v == 3) return se3;
        else if constexpr (v == 4) return se4; else if constexpr (v == 5) return se5;
        else if constexpr (v == 6) return se6; else return se7;
    };
    P2 zA, zB, zC;
    // every lane loads every plane (b outside the tile's ring and planes
    // past the chunk are not used): loads under a condition would make the
    // compiler wait for all outstanding loads where one of them is used
    auto issue = [&](int k, P2 &du, P2 &db, P2 &de) {
        if constexpr (!ZIN) du = ld_pair(uin, k);
        db = ld_pair(b, k);
        de = ld_pair(eps, k);
    };
    auto issue_at = [&](auto I) {
        constexpr int q = decltype(I)::value;
        if constexpr (q < R) issue(z0 - 2 + q, SU(I), SB(I), SE(I));
    };
    auto mask_at = [&](auto I, int p) {
        if constexpr (ZIN) SU(I) = masku(zero, p);
        else SU(I) = masku(SU(I), p);
        SE(I) = maske(SE(I), p);
    };
    auto vface = [&](const P2 &lo, const P2 &hi) {
        P2 r;
        r.v[0] = harm_face(lo.v[0], hi.v[0]);
        r.v[1] = harm_face(lo.v[1], hi.v[1]);
        return r;
    };
    // x and y faces of plane kp from the pair's eps e and the LDS plane s_e
    auto form_faces = [&](int kp, const P2 &e) __attribute__((always_inline)) {
        const int q = (kp + 3) % 3;
        const Pair<C> en = *reinterpret_cast<const Pair<C> *>(&s_e[ry1][lx]);
        Pair<C> w;
        w.v[0] = harm_face(e.v[0], e.v[1]);
        w.v[1] = harm_face(e.v[1], s_e[ry][lx2]);
        *reinterpret_cast<Pair<C> *>(&s_fx[q][ry][lx]) = w;
        w.v[0] = harm_face(e.v[0], en.v[0]);
        w.v[1] = harm_face(e.v[1], en.v[1]);
        *reinterpret_cast<Pair<C> *>(&s_fy[q][ry][lx]) = w;
    };
    auto put_e = [&](const P2 &e) {
        Pair<C> w;
        w.v[0] = e.v[0];
        w.v[1] = e.v[1];
        *reinterpret_cast<Pair<C> *>(&s_e[ry][lx]) = w;
    };
    issue_at(std::integral_constant<int, 0>{});
    issue_at(std::integral_constant<int, 1>{});
    issue_at(std::integral_constant<int, 2>{});
    issue_at(std::integral_constant<int, 3>{});
    issue_at(std::integral_constant<int, 4>{});
    issue_at(std::integral_constant<int, 5>{});
    issue_at(std::integral_constant<int, 6>{});
    issue_at(std::integral_constant<int, 7>{});
    mask_at(std::integral_constant<int, 0>{}, z0 - 2);
    mask_at(std::integral_constant<int, 1>{}, z0 - 1);
    mask_at(std::integral_constant<int, 2>{}, z0);
    // faces of plane z0-1 and the vertical faces below it
    put_e(se1);
    lds_barrier();
    form_faces(z0 - 1, se1);
    zB = vface(se0, se1);
    lds_barrier();
    C rn_cur = C(0), rn_prev = C(0), rn_prev2 = C(0);  // new red values of planes k, k-1, k-2

    auto step = [&](const P2 &um, const P2 &u0, const P2 &up, const P2 &bm, const P2 &b0, const P2 &e0,
                    const P2 &ep, int k, int pk) __attribute__((always_inline)) {
        zC = vface(e0, ep);
        {
            Pair<C> w;
            w.v[0] = u0.v[0];
            w.v[1] = u0.v[1];
            *reinterpret_cast<Pair<C> *>(&s_u[ry][lx]) = w;
        }
        put_e(ep);
        lds_barrier();
        form_faces(k + 1, ep);
        // ---- red cell of plane k (tile + 1-cell ring)
        rn_prev2 = rn_prev;
        rn_prev = rn_cur;
        {
            const int ro = pk;  // red cell of the pair: x + ro
            const int xr = x + ro;
            const int lr = lx + ro;
            const bool kin = k >= 0 && k < nz;
            const bool ring = xr >= -1 && xr <= TX && y >= -1 && y <= TY;
            C rv = csel<C>(kin, csel<C>(ro, gout1, gout0), csel<C>(k < 0, gz_lo, gz_hi));
            if (kin && ring && (ro ? c1_in : c0_in)) {
                const int q = (k + 3) % 3;
                const C fL = s_fx[q][ry][lr - 1], fR = s_fx[q][ry][lr];
                const C fD = s_fy[q][ry - 1][lr], fU = s_fy[q][ry][lr];
                const C fzm = pick(zB, ro), fzp = pick(zC, ro);
                C off = fL * s_u[ry][lr - 1];
                off = fma_c<C>(fR, s_u[ry][lr + 1], off);
                off = fma_c<C>(fD, s_u[ry - 1][lr], off);
                off = fma_c<C>(fU, s_u[ry + 1][lr], off);
                off = fma_c<C>(fzm, pick(um, ro), off);
                off = fma_c<C>(fzp, pick(up, ro), off);
                const C dg = ((fL + fR) + (fD + fU)) + (fzm + fzp);
                rv = qdiv<C>(fma_c<C>(h2, pick(b0, ro), off), ah2 + dg);
            }
            if (ring) s_r[k & 1][ry][lr] = rv;
            rn_cur = rv;
        }
        // ---- black cell of plane k-1 (tile only); write the pair
        {
            const int kb = k - 1;
            const int ro = pk ^ 1;  // red cell of the pair on plane kb
            const int bo = 1 - ro;         // black cell
            if (core && kb >= z0 && kb < z1 && (bo ? c1_in : c0_in)) {
                const int lb = lx + bo;
                const int q = (kb + 3) % 3;
                const C fL = s_fx[q][ry][lb - 1], fR = s_fx[q][ry][lb];
                const C fD = s_fy[q][ry - 1][lb], fU = s_fy[q][ry][lb];
                const C fzm = pick(zA, bo), fzp = pick(zB, bo);
                C off = fL * s_r[kb & 1][ry][lb - 1];
                off = fma_c<C>(fR, s_r[kb & 1][ry][lb + 1], off);
                off = fma_c<C>(fD, s_r[kb & 1][ry - 1][lb], off);
                off = fma_c<C>(fU, s_r[kb & 1][ry + 1][lb], off);
                off = fma_c<C>(fzm, rn_prev2, off);
                off = fma_c<C>(fzp, rn_cur, off);
                const C dg = ((fL + fR) + (fD + fU)) + (fzm + fzp);
                const C vb = qdiv<C>(fma_c<C>(h2, pick(bm, bo), off), ah2 + dg);
                char *pk = reinterpret_cast<char *>(uout) + plane_at(kb);
                if (even_nx) {
                    const T tb = N::cv(vb), tr = N::cv(rn_prev);
                    store_pair_nt(reinterpret_cast<T *>(pk + lane_at(lb0, kb)), bo ? tr : tb, bo ? tb : tr);
                } else {
                    *reinterpret_cast<T *>(pk + (bo ? lb1 : lb0)) = N::cv(vb);
                    if (ro ? c1_in : c0_in) *reinterpret_cast<T *>(pk + (ro ? lb1 : lb0)) = N::cv(rn_prev);
                }
            } else if (!even_nx && core && kb >= z0 && kb < z1 && (ro ? c1_in : c0_in)) {
                // odd nx: the pair's black cell lies outside the box
                char *pk = reinterpret_cast<char *>(uout) + plane_at(kb);
                *reinterpret_cast<T *>(pk + (ro ? lb1 : lb0)) = N::cv(rn_prev);
            }
        }
        lds_barrier();
    };

    // step k = kk + J of an unrolled group: refill slot J (plane k-2, read
    // last by step k-1) with plane k+1+PD (the last plane of the chunk once
    // past it), mask plane k+1, step
    auto iter = [&](auto J, int k) __attribute__((always_inline)) {
        constexpr int q = decltype(J)::value;
        using I1 = std::integral_constant<int, q + 1>;
        using I2 = std::integral_constant<int, q + 2>;
        using I3 = std::integral_constant<int, q + 3>;
        zA = zB;
        zB = zC;
        issue(min(k + 1 + PD, z1 + 1), SU(J), SB(J), SE(J));
        mask_at(I3{}, k + 1);
        step(SU(I1{}), SU(I2{}), SU(I3{}), SB(I1{}), SB(I2{}), SE(I2{}), SE(I3{}), k, par(J, k));
    };
    step(su0, su1, su2, sb0, sb1, se1, se2, z0 - 1, pz ^ 1);
    for (int kk = z0; kk <= z1; kk += R) {
        iter(std::integral_constant<int, 0>{}, kk);
        if (kk + 1 > z1) break;
        iter(std::integral_constant<int, 1>{}, kk + 1);
        if (kk + 2 > z1) break;
        iter(std::integral_constant<int, 2>{}, kk + 2);
        if (kk + 3 > z1) break;
        iter(std::integral_constant<int, 3>{}, kk + 3);
        if constexpr (R > 4) { if (kk + 4 > z1) break; iter(std::integral_constant<int, 4>{}, kk + 4); }
        if constexpr (R > 5) { if (kk + 5 > z1) break; iter(std::integral_constant<int, 5>{}, kk + 5); }
        if constexpr (R > 6) { if (kk + 6 > z1) break; iter(std::integral_constant<int, 6>{}, kk + 6); }
        if constexpr (R > 7) { if (kk + 7 > z1) break; iter(std::integral_constant<int, 7>{}, kk + 7); }
    }
}

// ---------------------------------------------------------------------
// The same sweep for beta = 1.  Every interior face has weight 1, so a cell
// outside the box carries the boundary term of the box face it lies beyond
// (2 g for Dirichlet, 0 for Neumann) and each cell's diagonal sum is fixed
// by its position: no per-face branches or selects remain.
template <class T, int TX, int TY, bool ZIN, int PD, bool EVEN>
__device__ __forceinline__ void rbgs_const_body(const SmoothArgs<T> &A, const int blk,
                                                typename Num<T>::C *smem) {
    using N = Num<T>;
    using C = typename N::C;
    constexpr int PXW = (TX + 4) / 2;  // pairs per region row
    constexpr int RX = TX + 4, RY = TY + 4, PL = RX * RY;
    C(*s_u)[RX] = reinterpret_cast<C(*)[RX]>(smem);                  // old u, plane k
    C(*s_r)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + PL);      // new red u, by plane parity
    const T *__restrict__ uin = A.uin;
    T *__restrict__ uout = A.uout;
    const T *__restrict__ b = A.b;
    const Geo &G = A.G;
    const int cz = A.cz, tiles_x = A.tiles_x, tiles_y = A.tiles_y;

    const int tid = threadIdx.x;
    const int tx = blk % tiles_x;
    const int rest = blk / tiles_x;
    const int ty = rest % tiles_y;
    const int tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const C h2 = C(G.h2), ah2 = C(G.ah2);

    const int ry = tid / PXW, pc = tid - ry * PXW;
    const int lx = 2 * pc;                  // LDS column of the pair's first cell
    const int x = lx - 2, y = ry - 2;       // tile coordinates of the pair
    const int gx = x0 + x, gy = y0 + y;     // global coordinates of its first cell
    const bool row_in = gy >= 0 && gy < ny;
    const bool c0_in = row_in && gx >= 0 && gx < nx;
    const bool c1_in = row_in && gx + 1 >= 0 && gx + 1 < nx;
    constexpr bool even_nx = EVEN;  // rows of even length: pairs never straddle a row
    const bool core = x >= 0 && x < TX && y >= 0 && y < TY;
    const size_t rowoff = (size_t)(row_in ? gy : 0) * nx;

    // box faces: weight in the diagonal (2 Dirichlet, 0 Neumann) and the
    // value carried by the cells beyond them
    auto fw = [&](int d) -> C { return ((G.bcmask >> d) & 1) ? C(2) : C(0); };
    auto hv = [&](int d) -> C { return ((G.bcmask >> d) & 1) ? C(2) * C(G.g[d]) : C(0); };
    auto halo = [&](int c) -> C {
        const int g = gx + c;
        return g < 0 ? hv(0) : g >= nx ? hv(1) : gy < 0 ? hv(2) : gy >= ny ? hv(3) : C(0);
    };
    auto dg_xy = [&](int c) -> C {
        const int g = gx + c;
        return (g > 0 ? C(1) : fw(0)) + (g < nx - 1 ? C(1) : fw(1)) + (gy > 0 ? C(1) : fw(2)) +
               (gy < ny - 1 ? C(1) : fw(3));
    };
    const C hout0 = halo(0), hout1 = halo(1), dxy0 = dg_xy(0), dxy1 = dg_xy(1);
    const C hz_lo = hv(4), hz_hi = hv(5), wz_lo = fw(4), wz_hi = fw(5);
    auto dg_z = [&](int k) -> C { return csel<C>(k > 0, C(1), wz_lo) + csel<C>(k < nz - 1, C(1), wz_hi); };
    // reciprocal diagonal of cell c of the pair on plane k: fixed for the
    // planes between the z box faces, formed there once
    const C rd0 = rcp_nr(ah2 + (dxy0 + C(2))), rd1 = rcp_nr(ah2 + (dxy1 + C(2)));
    auto rdiag = [&](int c, int k) -> C {
        if (k > 0 && k < nz - 1) return csel<C>(c, rd1, rd0);
        return rcp_nr(ah2 + (csel<C>(c, dxy1, dxy0) + dg_z(k)));
    };

    // offsets (elements) of the pair's cells within a plane (0 outside the
    // box) and of plane k: loads and stores take a uniform plane base plus
    // a 32-bit lane offset, both scaled by the element size of the array
    // (the coefficients may be wider than the fields)
    const uint32_t le0 = (uint32_t)(c0_in ? rowoff + gx : 0);
    const uint32_t le1 = (uint32_t)(c1_in ? rowoff + gx + 1 : 0);
    auto plane_el = [&](int k) -> size_t { return (size_t)min(max(k, 0), nz - 1) * plane; };
    const uint32_t lb0 = le0 * (uint32_t)sizeof(T), lb1 = le1 * (uint32_t)sizeof(T);
    auto plane_at = [&](int k) -> size_t { return plane_el(k) * sizeof(T); };

    struct P2 { C v[2]; };
    P2 zero;
    zero.v[0] = zero.v[1] = C(0);
    auto ld_pair = [&](const auto *__restrict__ a, int k) -> P2 {
        using A_ = std::remove_cv_t<std::remove_reference_t<decltype(*a)>>;
        constexpr uint32_t es = sizeof(A_);
        const char *pk = reinterpret_cast<const char *>(a) + plane_el(k) * es;
        P2 r;
        if (even_nx) {
            const Pair<A_> w = ld_wide<A_>(pk + lane_at(le0 * es, k));
            r.v[0] = Num<A_>::ld(w.v[0]);
            r.v[1] = Num<A_>::ld(w.v[1]);
        } else {
            r.v[0] = Num<A_>::ld(*reinterpret_cast<const A_ *>(pk + lane_at(le0 * es, k)));
            r.v[1] = Num<A_>::ld(*reinterpret_cast<const A_ *>(pk + lane_at(le1 * es, k)));
        }
        return r;
    };
    auto pick = [](const P2 &p, int c) -> C { return csel<C>(c, p.v[1], p.v[0]); };
    // (the plane test is uniform: a branch, leaving one select per cell)
    auto masku = [&](P2 v, int k) -> P2 {
        P2 r;
        if (k >= 0 && k < nz) {
            r.v[0] = csel<C>(c0_in, v.v[0], hout0);
            r.v[1] = csel<C>(c1_in, v.v[1], hout1);
        } else {
            r.v[0] = r.v[1] = k < 0 ? hz_lo : hz_hi;
        }
        return r;
    };

    // A ring of R = PD + 3 plane slots for u and for b: plane p occupies
    // slot (p - z0 + 2) mod R from its load, PD steps before the step that
    // first reads it, until the step after its own.  The steps are unrolled
    // R at a time, so every slot index is a constant: each load lands in the
    // registers its readers use and no value moves between registers (a
    // move of a loaded register would wait for that load at once).  u is
    // masked in place when its plane first becomes the upper neighbour
    // (cells outside the box carry their boundary term).
    static_assert(PD >= 1 && PD <= 5, "prefetch depth 1..5");
    constexpr int R = PD + 3;
    // parity of gy + k (which cell of the pair is red on plane k): with R
    // even it is the same for step J of every unrolled group, a per-lane
    // constant that needs no per-plane arithmetic
    const int pz = (gy + z0) & 1;
    auto par = [&](auto J, int k) -> int {
        if constexpr (R % 2 == 0) return pz ^ (decltype(J)::value & 1);
        else return (gy + k) & 1;
    };
    P2 su0, su1, su2, su3, su4, su5, su6, su7, sb0, sb1, sb2, sb3, sb4, sb5, sb6, sb7;
    auto SU = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return su0; else if constexpr (v == 1) return su1;
        else if constexpr (v == 2) return su2; else if constexpr (v == 3) return su3;
        else if constexpr (v == 4) return su4; else if constexpr (v == 5) return su5;
        else if constexpr (v == 6) return su6; else return su7;
    };
    auto SB = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return sb0; else if constexpr (v == 1) return sb1;
        else if constexpr (v == 2) return sb2; else if constexpr (v == 3) return sb3;
        else if constexpr (v == 4) return sb4; else if constexpr (v == 5) return sb5;
        else if constexpr (v == 6) return sb6; else return sb7;
    };
    // every lane loads every plane (b outside the tile's ring and planes
    // past the chunk are not used): loads under a condition would make the
    // compiler wait for all outstanding loads where one of them is used
    auto issue = [&](int k, P2 &du, P2 &db) {
        if constexpr (!ZIN) du = ld_pair(uin, k);
        db = ld_pair(b, k);
    };
    auto issue_at = [&](auto I) {
        constexpr int q = decltype(I)::value;
        if constexpr (q < R) issue(z0 - 2 + q, SU(I), SB(I));
    };
    issue_at(std::integral_constant<int, 0>{});
    issue_at(std::integral_constant<int, 1>{});
    issue_at(std::integral_constant<int, 2>{});
    issue_at(std::integral_constant<int, 3>{});
    issue_at(std::integral_constant<int, 4>{});
    issue_at(std::integral_constant<int, 5>{});
    issue_at(std::integral_constant<int, 6>{});
    issue_at(std::integral_constant<int, 7>{});
    auto mask_at = [&](auto I, int p) {
        if constexpr (ZIN) SU(I) = masku(zero, p);
        else SU(I) = masku(SU(I), p);
    };
    mask_at(std::integral_constant<int, 0>{}, z0 - 2);
    mask_at(std::integral_constant<int, 1>{}, z0 - 1);
    mask_at(std::integral_constant<int, 2>{}, z0);
    C rn_cur = C(0), rn_prev = C(0), rn_prev2 = C(0);  // new red values of planes k, k-1, k-2

    auto step = [&](const P2 &um, const P2 &u0, const P2 &up, const P2 &bm, const P2 &b0, int k, int pk)
                    __attribute__((always_inline)) {
        {
            Pair<C> w;
            w.v[0] = u0.v[0];
            w.v[1] = u0.v[1];
            *reinterpret_cast<Pair<C> *>(&s_u[ry][lx]) = w;
        }
        lds_barrier();
        // ---- red cell of plane k (tile + 1-cell ring)
        rn_prev2 = rn_prev;
        rn_prev = rn_cur;
        {
            const int ro = pk;  // red cell of the pair: x + ro
            const int xr = x + ro;
            const int lr = lx + ro;
            const bool kin = k >= 0 && k < nz;
            const bool ring = xr >= -1 && xr <= TX && y >= -1 && y <= TY;
            C rv;
            if (kin) rv = csel<C>(ro, hout1, hout0);
            else rv = k < 0 ? hz_lo : hz_hi;
            if (kin && ring && (ro ? c1_in : c0_in)) {
                const C off = ((s_u[ry][lr - 1] + s_u[ry][lr + 1]) + (s_u[ry - 1][lr] + s_u[ry + 1][lr])) +
                              (pick(um, ro) + pick(up, ro));
                rv = fma_c<C>(h2, pick(b0, ro), off) * rdiag(ro, k);
            }
            if (ring) s_r[k & 1][ry][lr] = rv;
            rn_cur = rv;
        }
        // ---- black cell of plane k-1 (tile only); write the pair
        {
            const int kb = k - 1;
            const int ro = pk ^ 1;  // red cell of the pair on plane kb
            const int bo = 1 - ro;         // black cell
            if (core && kb >= z0 && kb < z1 && (bo ? c1_in : c0_in)) {
                const int lb = lx + bo;
                const C off = ((s_r[kb & 1][ry][lb - 1] + s_r[kb & 1][ry][lb + 1]) +
                               (s_r[kb & 1][ry - 1][lb] + s_r[kb & 1][ry + 1][lb])) +
                              (rn_prev2 + rn_cur);
                const C vb = fma_c<C>(h2, pick(bm, bo), off) * rdiag(bo, kb);
                char *pk = reinterpret_cast<char *>(uout) + plane_at(kb);
                if (even_nx) {
                    const T tb = N::cv(vb), tr = N::cv(rn_prev);
                    store_pair_nt(reinterpret_cast<T *>(pk + lane_at(lb0, kb)), bo ? tr : tb, bo ? tb : tr);
                } else {
                    *reinterpret_cast<T *>(pk + (bo ? lb1 : lb0)) = N::cv(vb);
                    if (ro ? c1_in : c0_in) *reinterpret_cast<T *>(pk + (ro ? lb1 : lb0)) = N::cv(rn_prev);
                }
            } else if (!even_nx && core && kb >= z0 && kb < z1 && (ro ? c1_in : c0_in)) {
                // odd nx: the pair's black cell lies outside the box
                char *pk = reinterpret_cast<char *>(uout) + plane_at(kb);
                *reinterpret_cast<T *>(pk + (ro ? lb1 : lb0)) = N::cv(rn_prev);
            }
        }
        lds_barrier();
    };

    // step k = kk + J of an unrolled group: refill slot J (plane k-2, read
    // last by step k-1) with plane k+1+PD (the last plane of the chunk once
    // past it), mask plane k+1, step
    auto iter = [&](auto J, int k) __attribute__((always_inline)) {
        constexpr int q = decltype(J)::value;
        using I1 = std::integral_constant<int, q + 1>;
        using I2 = std::integral_constant<int, q + 2>;
        using I3 = std::integral_constant<int, q + 3>;
        issue(min(k + 1 + PD, z1 + 1), SU(J), SB(J));
        mask_at(I3{}, k + 1);
        step(SU(I1{}), SU(I2{}), SU(I3{}), SB(I1{}), SB(I2{}), k, par(J, k));
    };
    step(su0, su1, su2, sb0, sb1, z0 - 1, pz ^ 1);
    for (int kk = z0; kk <= z1; kk += R) {
        iter(std::integral_constant<int, 0>{}, kk);
        if (kk + 1 > z1) break;
        iter(std::integral_constant<int, 1>{}, kk + 1);
        if (kk + 2 > z1) break;
        iter(std::integral_constant<int, 2>{}, kk + 2);
        if (kk + 3 > z1) break;
        iter(std::integral_constant<int, 3>{}, kk + 3);
        if constexpr (R > 4) { if (kk + 4 > z1) break; iter(std::integral_constant<int, 4>{}, kk + 4); }
        if constexpr (R > 5) { if (kk + 5 > z1) break; iter(std::integral_constant<int, 5>{}, kk + 5); }
        if constexpr (R > 6) { if (kk + 6 > z1) break; iter(std::integral_constant<int, 6>{}, kk + 6); }
        if constexpr (R > 7) { if (kk + 7 > z1) break; iter(std::integral_constant<int, 7>{}, kk + 7); }
    }
}

// ---------------------------------------------------------------------
// The same sweep with stored face coefficients (coarse levels of a
// variable-coefficient operator).  Each plane's faces stream in through the
// prefetch ring with u and b: per pair, the three x faces of its row, the
// y faces below and above it and the z faces below it.  A face on a box
// face is scaled once on arrival by 2 (Dirichlet) or 0 (Neumann) and the
// cell beyond it carries u = g, so the update is the plain sum over six
// faces with no branches.
template <class T, int TX, int TY, bool ZIN, int PD, bool EVEN, bool DIAG = false>
__device__ __forceinline__ void rbgs_face_body(const SmoothArgs<T> &A, const int blk,
                                               typename Num<T>::C *smem) {
    using N = Num<T>;
    using C = typename N::C;
    using F = coef_t<T>;
    constexpr int PXW = (TX + 4) / 2;  // pairs per region row
    constexpr int RX = TX + 4, RY = TY + 4, PL = RX * RY;
    C(*s_u)[RX] = reinterpret_cast<C(*)[RX]>(smem);                  // old u, plane k
    C(*s_r)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + PL);      // new red u, by plane parity
    const T *__restrict__ uin = A.uin;
    T *__restrict__ uout = A.uout;
    const T *__restrict__ b = A.b;
    const F *__restrict__ fbx = A.fbx;
    const F *__restrict__ fby = A.fby;
    const F *__restrict__ fbz = A.fbz;
    const Geo &G = A.G;
    const int cz = A.cz, tiles_x = A.tiles_x, tiles_y = A.tiles_y;

    const int tid = threadIdx.x;
    const int tx = blk % tiles_x;
    const int rest = blk / tiles_x;
    const int ty = rest % tiles_y;
    const int tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const C h2 = C(G.h2), ah2 = C(G.ah2);

    const int ry = tid / PXW, pc = tid - ry * PXW;
    const int lx = 2 * pc;                  // LDS column of the pair's first cell
    const int x = lx - 2, y = ry - 2;       // tile coordinates of the pair
    const int gx = x0 + x, gy = y0 + y;     // global coordinates of its first cell
    const bool row_in = gy >= 0 && gy < ny;
    const bool c0_in = row_in && gx >= 0 && gx < nx;
    const bool c1_in = row_in && gx + 1 >= 0 && gx + 1 < nx;
    constexpr bool even_nx = EVEN;  // rows of even length: pairs never straddle a row
    const bool core = x >= 0 && x < TX && y >= 0 && y < TY;
    const size_t rowoff = (size_t)(row_in ? gy : 0) * nx;

    auto dir = [&](int d) { return ((G.bcmask >> d) & 1) != 0; };
    auto bmul = [&](int d) -> C { return dir(d) ? C(2) : C(0); };
    auto gval = [&](int d) -> C {
        return d == 0 ? C(G.g[0]) : d == 1 ? C(G.g[1]) : d == 2 ? C(G.g[2]) : d == 3 ? C(G.g[3]) : C(0);
    };
    auto side = [&](int c) -> int {
        const int g = gx + c;
        return g < 0 ? 0 : g >= nx ? 1 : gy < 0 ? 2 : gy >= ny ? 3 : 4;
    };
    const C gout0 = gval(side(0)), gout1 = gval(side(1));
    const C gz_lo = C(G.g[4]), gz_hi = C(G.g[5]);
    // face multipliers of the pair: x faces at gx, gx+1, gx+2; y below and above
    const C mx0 = gx == 0 ? bmul(0) : C(1);
    const C mx1 = gx + 1 == nx ? bmul(1) : C(1);
    const C mx2 = gx + 2 == nx ? bmul(1) : C(1);
    const C myd = gy == 0 ? bmul(2) : C(1);
    const C myu = gy + 1 == ny ? bmul(3) : C(1);
    const C mz_lo = bmul(4), mz_hi = bmul(5);

    // element offsets of the pair (0 for pairs outside the box, whose faces
    // are never used): fields and z faces, x faces, y faces below / above
    const bool pin = c0_in;  // the pair's first cell is in the box
    const uint32_t le0 = (uint32_t)(c0_in ? rowoff + gx : 0);
    const uint32_t le1 = (uint32_t)(c1_in ? rowoff + gx + 1 : 0);
    const uint32_t lfx = (uint32_t)(pin ? (size_t)gy * (nx + 1) + gx : 0);
    const uint32_t lfd = (uint32_t)(pin ? (size_t)gy * nx + gx : 0);
    const uint32_t lfu = (uint32_t)(pin ? (size_t)(gy + 1) * nx + gx : 0);
    const size_t fxpl = (size_t)ny * (nx + 1), fypl = (size_t)(ny + 1) * nx;
    auto cl = [&](int k, int hi) { return min(max(k, 0), hi); };

    struct P2 { C v[2]; };
    struct FS { C x0, x1, x2; P2 yd, yu, zb; };  // faces of one plane (scaled)
    P2 zero;
    zero.v[0] = zero.v[1] = C(0);
    // element e of plane k (plane length pl) of array a: a uniform plane
    // base plus a 32-bit lane offset
    auto at = [&](const auto *__restrict__ a, int k, size_t pl, uint32_t e) {
        using A_ = std::remove_cv_t<std::remove_reference_t<decltype(*a)>>;
        const char *pk = reinterpret_cast<const char *>(a) + (size_t)k * pl * sizeof(A_);
        return reinterpret_cast<const A_ *>(pk + lane_at(e * (uint32_t)sizeof(A_), k));
    };
    auto ld_u = [&](const T *__restrict__ a, int k) -> P2 {
        const int kc = cl(k, nz - 1);
        P2 r;
        if (even_nx) {
            const Pair<T> w = ld_wide<T>(at(a, kc, plane, le0));
            r.v[0] = N::ld(w.v[0]);
            r.v[1] = N::ld(w.v[1]);
        } else {
            r.v[0] = N::ld(*at(a, kc, plane, le0));
            r.v[1] = N::ld(*at(a, kc, plane, le1));
        }
        return r;
    };
    // raw faces of plane k (scaled when the plane is shifted in)
    auto ld_f = [&](int k) -> FS {
        FS f;
        const int kc = cl(k, nz - 1);
        const F *px = at(fbx, kc, fxpl, lfx);
        f.x0 = Num<F>::ld(px[0]);
        f.x1 = Num<F>::ld(px[1]);
        f.x2 = Num<F>::ld(px[c1_in || !pin ? 2 : 1]);  // odd nx: the pair may end at the box face
        const F *py = fby + (size_t)kc * fypl;
        const F *pz = fbz + (size_t)cl(k, nz) * plane + lfd;
        if (even_nx) {
            const Pair<F> d = ld_wide<F>(at(fby, kc, fypl, lfd));
            const Pair<F> u = ld_wide<F>(at(fby, kc, fypl, lfu));
            const Pair<F> z = ld_wide<F>(at(fbz, cl(k, nz), plane, lfd));
            f.yd.v[0] = Num<F>::ld(d.v[0]);
            f.yd.v[1] = Num<F>::ld(d.v[1]);
            f.yu.v[0] = Num<F>::ld(u.v[0]);
            f.yu.v[1] = Num<F>::ld(u.v[1]);
            f.zb.v[0] = Num<F>::ld(z.v[0]);
            f.zb.v[1] = Num<F>::ld(z.v[1]);
        } else {
            const uint32_t o1 = c1_in ? 1u : 0u;
            f.yd.v[0] = Num<F>::ld(py[lfd]);
            f.yd.v[1] = Num<F>::ld(py[lfd + o1]);
            f.yu.v[0] = Num<F>::ld(py[lfu]);
            f.yu.v[1] = Num<F>::ld(py[lfu + o1]);
            f.zb.v[0] = Num<F>::ld(pz[0]);
            f.zb.v[1] = Num<F>::ld(pz[o1]);
        }
        return f;
    };
    auto scale = [&](FS f, int k) -> FS {
        f.x0 *= mx0;
        f.x1 *= mx1;
        f.x2 *= mx2;
        f.yd.v[0] *= myd;
        f.yd.v[1] *= myd;
        f.yu.v[0] *= myu;
        f.yu.v[1] *= myu;
        const C mz = csel<C>(k == 0, mz_lo, csel<C>(k == nz, mz_hi, C(1)));
        f.zb.v[0] *= mz;
        f.zb.v[1] *= mz;
        return f;
    };
    auto pick = [](const P2 &p, int c) -> C { return csel<C>(c, p.v[1], p.v[0]); };
    auto masku = [&](P2 v, int k) -> P2 {
        const bool kin = k >= 0 && k < nz;
        const C zv = csel<C>(k < 0, gz_lo, gz_hi);
        P2 r;
        r.v[0] = csel<C>(kin && c0_in, v.v[0], csel<C>(kin, gout0, zv));
        r.v[1] = csel<C>(kin && c1_in, v.v[1], csel<C>(kin, gout1, zv));
        return r;
    };

    // A ring of R = PD + 3 plane slots for u, b and the faces: plane p
    // occupies slot (p - z0 + 2) mod R from its load, PD steps before the
    // step that first reads it, until the step after its own.  The steps are
    // unrolled R at a time, so every slot index is a constant and no loaded
    // value moves between registers (such a move would wait for its load at
    // once).  u is masked and the faces scaled in place when their plane
    // first becomes the upper neighbour.
    static_assert(PD >= 1 && PD <= 5, "prefetch depth 1..5");
    constexpr int R = PD + 3;
    // parity of gy + k (which cell of the pair is red on plane k): with R
    // even it is the same for step J of every unrolled group, a per-lane
    // constant that needs no per-plane arithmetic
    const int pz = (gy + z0) & 1;
    auto par = [&](auto J, int k) -> int {
        if constexpr (R % 2 == 0) return pz ^ (decltype(J)::value & 1);
        else return (gy + k) & 1;
    };
    P2 su0, su1, su2, su3, su4, su5, su6, su7, sb0, sb1, sb2, sb3, sb4, sb5, sb6, sb7;
    FS sf0, sf1, sf2, sf3, sf4, sf5, sf6, sf7;
    auto SU = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return su0; else if constexpr (v == 1) return su1;
        else if constexpr (v == 2) return su2; else if constexpr (v == 3) return su3;
        else if constexpr (v == 4) return su4; else if constexpr (v == 5) return su5;
        else if constexpr (v == 6) return su6; else return su7;
    };
    auto SB = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return sb0; else if constexpr (v == 1) return sb1;
        else if constexpr (v == 2) return sb2; else if constexpr (v == 3) return sb3;
        else if constexpr (v == 4) return sb4; else if constexpr (v == 5) return sb5;
        else if constexpr (v == 6) return sb6; else return sb7;
    };
    auto SF = [&](auto I) -> FS & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return sf0; else if constexpr (v == 1) return sf1;
        else if constexpr (v == 2) return sf2; else if constexpr (v == 3) return sf3;
        else if constexpr (v == 4) return sf4; else if constexpr (v == 5) return sf5;
        else if constexpr (v == 6) return sf6; else return sf7;
    };
    // every lane loads every plane (b outside the tile's ring and planes
    // past the chunk are not used): loads under a condition would make the
    // compiler wait for all outstanding loads where one of them is used
    auto issue = [&](int k, P2 &du, P2 &db, FS &df) {
        if constexpr (!ZIN) du = ld_u(uin, k);
        db = ld_u(b, k);
        df = ld_f(k);
    };
    auto issue_at = [&](auto I) {
        constexpr int q = decltype(I)::value;
        if constexpr (q < R) issue(z0 - 2 + q, SU(I), SB(I), SF(I));
    };
    auto mask_at = [&](auto I, int p) {
        if constexpr (ZIN) SU(I) = masku(zero, p);
        else SU(I) = masku(SU(I), p);
        SF(I) = scale(SF(I), p);
    };
    issue_at(std::integral_constant<int, 0>{});
    issue_at(std::integral_constant<int, 1>{});
    issue_at(std::integral_constant<int, 2>{});
    issue_at(std::integral_constant<int, 3>{});
    issue_at(std::integral_constant<int, 4>{});
    issue_at(std::integral_constant<int, 5>{});
    issue_at(std::integral_constant<int, 6>{});
    issue_at(std::integral_constant<int, 7>{});
    mask_at(std::integral_constant<int, 0>{}, z0 - 2);
    mask_at(std::integral_constant<int, 1>{}, z0 - 1);
    mask_at(std::integral_constant<int, 2>{}, z0);
    C rn_cur = C(0), rn_prev = C(0), rn_prev2 = C(0);  // new red values of planes k, k-1, k-2

    auto step = [&](const P2 &um, const P2 &u0, const P2 &up, const P2 &bm, const P2 &b0, const FS &fm,
                    const FS &f0, const FS &fp, int k, int pk) __attribute__((always_inline)) {
        {
            Pair<C> w;
            w.v[0] = u0.v[0];
            w.v[1] = u0.v[1];
            *reinterpret_cast<Pair<C> *>(&s_u[ry][lx]) = w;
        }
        lds_barrier();
        // ---- red cell of plane k (tile + 1-cell ring)
        rn_prev2 = rn_prev;
        rn_prev = rn_cur;
        {
            const int ro = pk;  // red cell of the pair: x + ro
            const int xr = x + ro;
            const int lr = lx + ro;
            const bool kin = k >= 0 && k < nz;
            const bool ring = xr >= -1 && xr <= TX && y >= -1 && y <= TY;
            C rv = csel<C>(kin, csel<C>(ro, gout1, gout0), csel<C>(k < 0, gz_lo, gz_hi));
            if (kin && ring && (ro ? c1_in : c0_in)) {
                const C fL = csel<C>(ro, f0.x1, f0.x0), fR = csel<C>(ro, f0.x2, f0.x1);
                const C fD = pick(f0.yd, ro), fU = pick(f0.yu, ro);
                const C fB = pick(f0.zb, ro), fA = pick(fp.zb, ro);
                C off = fL * s_u[ry][lr - 1];
                off = fma_c<C>(fR, s_u[ry][lr + 1], off);
                off = fma_c<C>(fD, s_u[ry - 1][lr], off);
                off = fma_c<C>(fU, s_u[ry + 1][lr], off);
                off = fma_c<C>(fB, pick(um, ro), off);
                off = fma_c<C>(fA, pick(up, ro), off);
                C dg = ((fL + fR) + (fD + fU)) + (fB + fA);
                if constexpr (DIAG) dg = fma_c<C>(h2, C(A.dd[(size_t)k * plane + (ro ? le1 : le0)]), dg);
                rv = qdiv<C>(fma_c<C>(h2, pick(b0, ro), off), ah2 + dg);
            }
            if (ring) s_r[k & 1][ry][lr] = rv;
            rn_cur = rv;
        }
        // ---- black cell of plane k-1 (tile only); write the pair
        {
            const int kb = k - 1;
            const int ro = pk ^ 1;  // red cell of the pair on plane kb
            const int bo = 1 - ro;         // black cell
            if (core && kb >= z0 && kb < z1 && (bo ? c1_in : c0_in)) {
                const int lb = lx + bo;
                const C fL = csel<C>(bo, fm.x1, fm.x0), fR = csel<C>(bo, fm.x2, fm.x1);
                const C fD = pick(fm.yd, bo), fU = pick(fm.yu, bo);
                const C fB = pick(fm.zb, bo), fA = pick(f0.zb, bo);
                C off = fL * s_r[kb & 1][ry][lb - 1];
                off = fma_c<C>(fR, s_r[kb & 1][ry][lb + 1], off);
                off = fma_c<C>(fD, s_r[kb & 1][ry - 1][lb], off);
                off = fma_c<C>(fU, s_r[kb & 1][ry + 1][lb], off);
                off = fma_c<C>(fB, rn_prev2, off);
                off = fma_c<C>(fA, rn_cur, off);
                C dg = ((fL + fR) + (fD + fU)) + (fB + fA);
                if constexpr (DIAG) dg = fma_c<C>(h2, C(A.dd[(size_t)kb * plane + (bo ? le1 : le0)]), dg);
                const C vb = qdiv<C>(fma_c<C>(h2, pick(bm, bo), off), ah2 + dg);
                T *pk = uout + (size_t)kb * plane;
                if (even_nx) {
                    const T tb = N::cv(vb), tr = N::cv(rn_prev);
                    store_pair_nt(const_cast<T *>(at(uout, kb, plane, le0)), bo ? tr : tb, bo ? tb : tr);
                } else {
                    pk[bo ? le1 : le0] = N::cv(vb);
                    if (ro ? c1_in : c0_in) pk[ro ? le1 : le0] = N::cv(rn_prev);
                }
            } else if (!even_nx && core && kb >= z0 && kb < z1 && (ro ? c1_in : c0_in)) {
                // odd nx: the pair's black cell lies outside the box
                uout[(size_t)kb * plane + (ro ? le1 : le0)] = N::cv(rn_prev);
            }
        }
        lds_barrier();
    };

    // step k = kk + J of an unrolled group: refill slot J (plane k-2, read
    // last by step k-1) with plane k+1+PD (the last plane of the chunk once
    // past it), mask and scale plane k+1, step
    auto iter = [&](auto J, int k) __attribute__((always_inline)) {
        constexpr int q = decltype(J)::value;
        using I1 = std::integral_constant<int, q + 1>;
        using I2 = std::integral_constant<int, q + 2>;
        using I3 = std::integral_constant<int, q + 3>;
        issue(min(k + 1 + PD, z1 + 1), SU(J), SB(J), SF(J));
        mask_at(I3{}, k + 1);
        step(SU(I1{}), SU(I2{}), SU(I3{}), SB(I1{}), SB(I2{}), SF(I1{}), SF(I2{}), SF(I3{}), k, par(J, k));
    };
    step(su0, su1, su2, sb0, sb1, sf0, sf1, sf2, z0 - 1, pz ^ 1);
    for (int kk = z0; kk <= z1; kk += R) {
        iter(std::integral_constant<int, 0>{}, kk);
        if (kk + 1 > z1) break;
        iter(std::integral_constant<int, 1>{}, kk + 1);
        if (kk + 2 > z1) break;
        iter(std::integral_constant<int, 2>{}, kk + 2);
        if (kk + 3 > z1) break;
        iter(std::integral_constant<int, 3>{}, kk + 3);
        if constexpr (R > 4) { if (kk + 4 > z1) break; iter(std::integral_constant<int, 4>{}, kk + 4); }
        if constexpr (R > 5) { if (kk + 5 > z1) break; iter(std::integral_constant<int, 5>{}, kk + 5); }
        if constexpr (R > 6) { if (kk + 6 > z1) break; iter(std::integral_constant<int, 6>{}, kk + 6); }
        if constexpr (R > 7) { if (kk + 7 > z1) break; iter(std::integral_constant<int, 7>{}, kk + 7); }
    }
}

// The stored-face sweep in the general form (per-face sums with box-face
// selects, faces read where they are used): the batched engine's, whose
// one smoother kernel serves every coefficient kind and so must keep a
// modest register footprint.
template <class T, int MODE, int TX, int TY, bool ZIN, int PD>
__device__ __forceinline__ void rbgs_pair_body(const SmoothArgs<T> &A, const int blk,
                                               typename Num<T>::C *smem) {
    static_assert(MODE == COEF_FACE, "stored face coefficients only");
    using N = Num<T>;
    using C = typename N::C;
    constexpr int PXW = (TX + 4) / 2;  // pairs per region row
    constexpr int RX = TX + 4, RY = TY + 4;
    C(*s_u)[RX] = reinterpret_cast<C(*)[RX]>(smem);
    C(*s_r)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + RY * RX);
    const T *__restrict__ uin = A.uin;
    T *__restrict__ uout = A.uout;
    const T *__restrict__ b = A.b;
    const coef_t<T> *__restrict__ fbx = A.fbx;
    const coef_t<T> *__restrict__ fby = A.fby;
    const coef_t<T> *__restrict__ fbz = A.fbz;
    const Geo &G = A.G;
    const int cz = A.cz, tiles_x = A.tiles_x, tiles_y = A.tiles_y;

    const int tid = threadIdx.x;
    const int tx = blk % tiles_x;
    const int rest = blk / tiles_x;
    const int ty = rest % tiles_y;
    const int tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const C h2 = C(G.h2), ah2 = C(G.ah2);

    const int ry = tid / PXW, pc = tid - ry * PXW;
    const int lx = 2 * pc;                  // LDS column of the pair's first cell
    const int x = lx - 2, y = ry - 2;       // tile coordinates of the pair
    const int gx = x0 + x, gy = y0 + y;     // global coordinates of its first cell
    const bool row_in = gy >= 0 && gy < ny;
    const bool c0_in = row_in && gx >= 0 && gx < nx;
    const bool c1_in = row_in && gx + 1 >= 0 && gx + 1 < nx;
    const bool even_nx = (nx & 1) == 0;
    const bool core = x >= 0 && x < TX && y >= 0 && y < TY;
    const size_t rowoff = (size_t)(row_in ? gy : 0) * nx;

    struct P2 { C v[2]; };
    // load one pair of plane k (values outside the box are masked by the caller)
    auto ld_pair = [&](const auto *__restrict__ a, int k) -> P2 {
        using A_ = std::remove_cv_t<std::remove_reference_t<decltype(*a)>>;
        P2 r;
        const bool kin = k >= 0 && k < nz;
        if (even_nx) {
            const size_t g = (kin && c0_in) ? (size_t)k * plane + rowoff + gx : 0;
            const Pair<A_> w = ld_wide<A_>(a + g);
            r.v[0] = Num<A_>::ld(w.v[0]);
            r.v[1] = Num<A_>::ld(w.v[1]);
        } else {
            const size_t base = (size_t)(kin ? k : 0) * plane + rowoff;
            r.v[0] = Num<A_>::ld(a[(kin && c0_in) ? base + gx : 0]);
            r.v[1] = Num<A_>::ld(a[(kin && c1_in) ? base + gx + 1 : 0]);
        }
        return r;
    };
    auto valid = [&](int k, int c) { return k >= 0 && k < nz && (c ? c1_in : c0_in); };
    // select, not an index: a runtime index would force the pair into memory
    auto pick = [](const P2 &p, int c) -> C { return c ? p.v[1] : p.v[0]; };

    // current planes: u at k-1, k, k+1; b at k-1, k, k+1
    P2 um, u0, up, bm, b0, bp;
    // prefetch ring (plane p in slot (p - z0 - 1) mod PD); one named
    // variable per slot so that the ring stays in registers
    static_assert(PD >= 1 && PD <= 4, "prefetch depth 1..4");
    P2 qu0, qu1, qu2, qu3, qb0, qb1, qb2, qb3;
    auto QU = [&](auto S) -> P2 & {
        constexpr int v = decltype(S)::value;
        if constexpr (v == 0) return qu0; else if constexpr (v == 1) return qu1;
        else if constexpr (v == 2) return qu2; else return qu3;
    };
    auto QB = [&](auto S) -> P2 & {
        constexpr int v = decltype(S)::value;
        if constexpr (v == 0) return qb0; else if constexpr (v == 1) return qb1;
        else if constexpr (v == 2) return qb2; else return qb3;
    };
    auto masku = [&](P2 v, int k) { P2 r; r.v[0] = valid(k, 0) ? v.v[0] : C(0); r.v[1] = valid(k, 1) ? v.v[1] : C(0); return r; };
    auto issue = [&](int k, P2 &du, P2 &db) {
        if constexpr (!ZIN) du = ld_pair(uin, k);
        db = ld_pair(b, k);
    };
    {
        P2 t0u, t0b, t1u, t1b, t2u, t2b;
        issue(z0 - 2, t0u, t0b);
        issue(z0 - 1, t1u, t1b);
        issue(z0, t2u, t2b);
        issue(z0 + 1, qu0, qb0);
        if constexpr (PD > 1) issue(z0 + 2, qu1, qb1);
        if constexpr (PD > 2) issue(z0 + 3, qu2, qb2);
        if constexpr (PD > 3) issue(z0 + 4, qu3, qb3);
        P2 zero; zero.v[0] = zero.v[1] = C(0);
        um = ZIN ? zero : masku(t0u, z0 - 2);
        u0 = ZIN ? zero : masku(t1u, z0 - 1);
        up = ZIN ? zero : masku(t2u, z0);
        bm = masku(t0b, z0 - 2);
        b0 = masku(t1b, z0 - 1);
        bp = masku(t2b, z0);
    }
    C rn_cur = C(0), rn_prev = C(0), rn_prev2 = C(0);  // new red values of planes k, k-1, k-2

    auto step = [&](int k) {
        // ---- publish plane k (old u) for the in-plane neighbours
        {
            Pair<C> w;
            w.v[0] = u0.v[0];
            w.v[1] = u0.v[1];
            *reinterpret_cast<Pair<C> *>(&s_u[ry][lx]) = w;
        }
        lds_barrier();
        // ---- red cell of plane k (tile + 1-cell ring)
        rn_prev2 = rn_prev;
        rn_prev = rn_cur;
        {
            const int ro = (gy + k) & 1;  // red cell of the pair: x + ro
            const int xr = x + ro;
            const int lr = lx + ro;
            const bool doit = k >= 0 && k < nz && xr >= -1 && xr <= TX && y >= -1 && y <= TY &&
                              (ro ? c1_in : c0_in);
            if (doit) {
                const int gxr = gx + ro;
                C off, dg;
                six_faces<C, MODE, true>(
                    G, gxr, gy, k, C(1),
                    [&](int d) -> C {
                        if constexpr (ZIN) return C(0);
                        else return d == 0   ? (ro ? u0.v[0] : s_u[ry][lr - 1])
                                    : d == 1 ? (ro ? s_u[ry][lr + 1] : u0.v[1])
                                    : d == 2 ? s_u[ry - 1][lr]
                                    : d == 3 ? s_u[ry + 1][lr]
                                    : d == 4 ? pick(um, ro)
                                             : pick(up, ro);
                    },
                    [&](int) -> C { return C(1); },
                    [&](int d) -> C {
                        return d == 0   ? face_x(fbx, G, gxr, gy, k)
                               : d == 1 ? face_x(fbx, G, gxr + 1, gy, k)
                               : d == 2 ? face_y(fby, G, gxr, gy, k)
                               : d == 3 ? face_y(fby, G, gxr, gy + 1, k)
                               : d == 4 ? face_z(fbz, G, gxr, gy, k)
                                        : face_z(fbz, G, gxr, gy, k + 1);
                    },
                    off, dg);
                rn_cur = qdiv(h2 * pick(b0, ro) + off, ah2 + dg);
                s_r[k & 1][ry][lr] = rn_cur;
            }
        }
        // ---- black cell of plane k-1 (tile only); write the pair
        {
            const int kb = k - 1;
            const int ro = (gy + kb) & 1;  // red cell of the pair on plane kb
            const int bo = 1 - ro;         // black cell
            if (core && kb >= z0 && kb < z1 && (bo ? c1_in : c0_in)) {
                const int gxb = gx + bo;
                const int lb = lx + bo;
                C off, dg;
                six_faces<C, MODE, true>(
                    G, gxb, gy, kb, C(1),
                    [&](int d) -> C {
                        return d == 0   ? (bo ? rn_prev : s_r[kb & 1][ry][lb - 1])
                               : d == 1 ? (bo ? s_r[kb & 1][ry][lb + 1] : rn_prev)
                               : d == 2 ? s_r[kb & 1][ry - 1][lb]
                               : d == 3 ? s_r[kb & 1][ry + 1][lb]
                               : d == 4 ? rn_prev2
                                        : rn_cur;
                    },
                    [&](int) -> C { return C(1); },
                    [&](int d) -> C {
                        return d == 0   ? face_x(fbx, G, gxb, gy, kb)
                               : d == 1 ? face_x(fbx, G, gxb + 1, gy, kb)
                               : d == 2 ? face_y(fby, G, gxb, gy, kb)
                               : d == 3 ? face_y(fby, G, gxb, gy + 1, kb)
                               : d == 4 ? face_z(fbz, G, gxb, gy, kb)
                                        : face_z(fbz, G, gxb, gy, kb + 1);
                    },
                    off, dg);
                const C vb = qdiv(h2 * pick(bm, bo) + off, ah2 + dg);
                const size_t gp = (size_t)kb * plane + rowoff + gx;
                if (even_nx) {
                    Pair<T> o;
                    const T tb = N::cv(vb), tr = N::cv(rn_prev);
                    o.v[0] = bo ? tr : tb;
                    o.v[1] = bo ? tb : tr;
                    *reinterpret_cast<Pair<T> *>(uout + gp) = o;
                } else {
                    uout[gp + bo] = N::cv(vb);
                    if (ro ? c1_in : c0_in) uout[gp + ro] = N::cv(rn_prev);
                }
            } else if (!even_nx && core && kb >= z0 && kb < z1 && (ro ? c1_in : c0_in)) {
                // odd nx: the pair's black cell lies outside the box
                uout[(size_t)kb * plane + rowoff + gx + ro] = N::cv(rn_prev);
            }
        }
        lds_barrier();
    };

    // shift in plane k+1 from ring slot S, refill the slot with k+1+PD, step k
    auto iter = [&](auto S, int k) {
        um = u0; u0 = up;
        bm = b0; b0 = bp;
        if constexpr (!ZIN) up = masku(QU(S), k + 1);
        bp = masku(QB(S), k + 1);
        if (k + 1 + PD <= z1 + 1) issue(k + 1 + PD, QU(S), QB(S));
        step(k);
    };
    step(z0 - 1);
    for (int kk = z0; kk <= z1; kk += PD) {
        iter(std::integral_constant<int, 0>{}, kk);
        if constexpr (PD > 1) { if (kk + 1 > z1) break; iter(std::integral_constant<int, 1>{}, kk + 1); }
        if constexpr (PD > 2) { if (kk + 2 > z1) break; iter(std::integral_constant<int, 2>{}, kk + 2); }
        if constexpr (PD > 3) { if (kk + 3 > z1) break; iter(std::integral_constant<int, 3>{}, kk + 3); }
    }
}

template <class T, int MODE, int TX, int TY, bool ZIN, int PD, bool EVEN>
__device__ __forceinline__ void rbgs_col_body(const SmoothArgs<T> &A, const int blk,
                                              typename Num<T>::C *smem) {
    if constexpr (MODE == COEF_CELL) rbgs_cell_body<T, TX, TY, ZIN, PD, EVEN>(A, blk, smem);
    else if constexpr (MODE == COEF_CONST) rbgs_const_body<T, TX, TY, ZIN, PD, EVEN>(A, blk, smem);
    else rbgs_face_body<T, TX, TY, ZIN, PD, EVEN, MODE == COEF_FACED>(A, blk, smem);
}

// EVEN: the level's rows have even length, so a pair is two adjacent
// elements of one row and moves with one wide access; odd rows take the
// per-element form.  The host picks the variant from nx.
template <class T, int MODE, int TX, int TY, bool ZIN, int PD, bool EVEN>
__global__ __launch_bounds__((TX + 4) / 2 * (TY + 4)) void rbgs_col_k(SmoothArgs<T> A) {
    if (A.done && *A.done) return;  // the solve has converged: nothing left to do
    if (EVEN != ((A.G.nx & 1) == 0)) return;  // not launched this way by the host
    __shared__ typename Num<T>::C smem[smooth_lds<MODE, TX, TY>()];
    rbgs_col_body<T, MODE, TX, TY, ZIN, PD, EVEN>(A, xcd_remap(blockIdx.x, A.nblk), smem);
}

// ---------------------------------------------------------------------
// Residual + restriction (+ squared norm), column-pair streaming form.
//
// bc[K][J][I] = mean of the residuals b - A u of the 8 fine children.  A
// thread owns the fine pair (2I, 2I+1) of one row of the tile grown by one
// cell, marches up the planes of its chunk with u (and eps) streamed PD
// planes ahead, exchanges in-plane neighbours through LDS, keeps vertical
// ones in registers, and sums the pair's residuals over two planes; two
// adjacent rows are then combined into the coarse value.  If slot >= 0 the
// squared residual is also reduced (FP64, deterministic) into ws.result[slot]
// and, with done_out, the convergence flag is set against
// rtol2 * ws.result[ref_slot].
template <class T> struct RrArgs {
    const T *u;
    const T *b;
    const coef_t<T> *eps;
    const coef_t<T> *fbx, *fby, *fbz;
    Geo G;
    T *bc;
    int cz, tiles_x, tiles_y, nblk;
    RedWs ws;
    int slot, ref_slot;
    double rtol2;
    int *done_out;
    const int *done_in;
    const double *dd;  // COEF_FACED: per-cell extra diagonal
};

template <int MODE, int TX, int TY> constexpr int rr_lds() {
    // u plane, accumulators; cell coefficients add an eps plane and two
    // planes (by parity) of x faces (one per pair) and of y faces
    return (MODE == COEF_CELL ? 4 : 1) * (TY + 2) * (TX + 4) + (MODE == COEF_CELL ? 3 : 1) * (TY + 2) * ((TX + 4) / 2);
}
template <int TX, int TY> constexpr int rr_threads() { return (((TX + 4) / 2 * (TY + 2)) + 63) / 64 * 64; }

template <class T, int MODE, int TX, int TY, int PD>
__device__ __forceinline__ double rr_col_body(const RrArgs<T> &A, const int blk, typename Num<T>::C *smem) {
    using N = Num<T>;
    using C = typename N::C;
    constexpr int PXW = (TX + 4) / 2;  // pairs per region row (1-cell halo, pair aligned)
    constexpr int RX = TX + 4, RY = TY + 2;
    constexpr int NTH = PXW * RY;
    constexpr int NTP = (NTH + 63) / 64 * 64;
    constexpr bool CELL = (MODE == COEF_CELL);
    C(*s_u)[RX] = reinterpret_cast<C(*)[RX]>(smem);
    C(*s_e)[RX] = reinterpret_cast<C(*)[RX]>(smem + RY * RX);  // eps of plane k+1 at step k
    C(*s_acc)[PXW] = reinterpret_cast<C(*)[PXW]>(smem + (CELL ? 2 : 1) * RY * RX);
    // Cell coefficients: every face is formed once, by the pair below or to
    // its left, one plane ahead (from the eps plane k+1 in LDS): s_fx[q][ry][pc]
    // is the face between the pair's second cell and the next pair's first
    // cell, s_fy[q][ry][c] the face between rows ry and ry+1 of column c, for
    // planes of parity q.  The pair's inner face and its two vertical faces
    // stay in registers (the face below plane k is the one above plane k-1).
    // harm_face is symmetric to the last bit, so every face has the value
    // either of its cells would form.
    C(*s_fx)[RY][PXW] = reinterpret_cast<C(*)[RY][PXW]>(smem + 2 * RY * RX + RY * PXW);
    C(*s_fy)[RY][RX] = reinterpret_cast<C(*)[RY][RX]>(smem + 2 * RY * RX + 3 * RY * PXW);
    const T *__restrict__ u = A.u;
    const T *__restrict__ b = A.b;
    const coef_t<T> *__restrict__ eps = A.eps;
    const coef_t<T> *__restrict__ fbx = A.fbx;
    const coef_t<T> *__restrict__ fby = A.fby;
    const coef_t<T> *__restrict__ fbz = A.fbz;
    T *__restrict__ bc = A.bc;
    const Geo &G = A.G;
    const int cz = A.cz, tiles_x = A.tiles_x, tiles_y = A.tiles_y;

    const int tid = threadIdx.x;
    const bool live = tid < NTH;
    const int tx = blk % tiles_x;
    const int rest = blk / tiles_x;
    const int ty = rest % tiles_y;
    const int tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const C ih2 = C(G.ih2), a = C(G.a);

    const int ry = live ? tid / PXW : 0, pc = live ? tid - ry * PXW : 0;
    const int lx = 2 * pc;             // LDS column of the pair's first cell
    const int x = lx - 2, y = ry - 1;  // tile coordinates
    const int gx = x0 + x, gy = y0 + y;
    const bool row_in = live && gy >= 0 && gy < ny;
    const bool c_in = row_in && gx >= 0 && gx < nx;  // nx is even here: pairs are all in or all out
    const bool core = live && x >= 0 && x < TX && y >= 0 && y < TY && c_in;
    const size_t rowoff = (size_t)(row_in ? gy : 0) * nx;

    struct P2 { C v[2]; };
    // uniform plane base plus a 32-bit lane offset, scaled by the element
    // size of the array (a plane outside the box reads the nearest one)
    const uint32_t le = (uint32_t)(c_in ? rowoff + gx : 0);
    auto ld_pair = [&](const auto *__restrict__ p, int k) -> P2 {
        using A_ = std::remove_cv_t<std::remove_reference_t<decltype(*p)>>;
        constexpr uint32_t es = sizeof(A_);
        const char *pk = reinterpret_cast<const char *>(p) + (size_t)min(max(k, 0), nz - 1) * plane * es;
        const Pair<A_> w = ld_wide<A_>(pk + lane_at(le * es, k));
        P2 r;
        r.v[0] = Num<A_>::ld(w.v[0]);
        r.v[1] = Num<A_>::ld(w.v[1]);
        return r;
    };
    // Box faces with beta = 1 and with cell coefficients take no branches,
    // as in the sweeps: a cell outside the box carries the boundary term of
    // the face it lies beyond (beta = 1: u = 2g or 0, the face weight being
    // part of the cell's fixed diagonal; cell coefficients: u = g and a
    // coefficient 0 or kBigCoef for harm_face).  Stored faces keep the
    // general face sums.
    const int sd = gx < 0 ? 0 : gx >= nx ? 1 : gy < 0 ? 2 : gy >= ny ? 3 : 4;  // pairs are all in or all out
    auto dir = [&](int d) { return d < 6 && ((G.bcmask >> d) & 1) != 0; };
    auto gval = [&](int d) -> C {
        return d == 0 ? C(G.g[0]) : d == 1 ? C(G.g[1]) : d == 2 ? C(G.g[2]) : d == 3 ? C(G.g[3]) : C(0);
    };
    const C big = kBigCoef<C>;
    const C uout = MODE == COEF_CONST ? (dir(sd) ? C(2) * gval(sd) : C(0)) : gval(sd);
    const C uz_lo = MODE == COEF_CONST ? (dir(4) ? C(2) * C(G.g[4]) : C(0)) : C(G.g[4]);
    const C uz_hi = MODE == COEF_CONST ? (dir(5) ? C(2) * C(G.g[5]) : C(0)) : C(G.g[5]);
    const C eout = dir(sd) ? big : C(0), ez_lo = dir(4) ? big : C(0), ez_hi = dir(5) ? big : C(0);
    // beta = 1: in-plane part of each cell's diagonal
    auto dg_xy = [&](int c) -> C {
        const int g = gx + c;
        return (g > 0 ? C(1) : (dir(0) ? C(2) : C(0))) + (g < nx - 1 ? C(1) : (dir(1) ? C(2) : C(0))) +
               (gy > 0 ? C(1) : (dir(2) ? C(2) : C(0))) + (gy < ny - 1 ? C(1) : (dir(3) ? C(2) : C(0)));
    };
    const C dxy0 = dg_xy(0), dxy1 = dg_xy(1);
    const C wz_lo = dir(4) ? C(2) : C(0), wz_hi = dir(5) ? C(2) : C(0);
    auto mask_out = [&](P2 v, int k, C out, C zlo, C zhi) -> P2 {
        const bool kin = k >= 0 && k < nz;
        const C alt = csel<C>(kin, out, csel<C>(k < 0, zlo, zhi));
        P2 r;
        r.v[0] = csel<C>(kin && c_in, v.v[0], alt);
        r.v[1] = csel<C>(kin && c_in, v.v[1], alt);
        return r;
    };
    auto vmask = [&](P2 v, int k, C fill) {
        const bool ok = k >= 0 && k < nz && c_in;
        P2 r;
        r.v[0] = csel<C>(ok, v.v[0], fill);
        r.v[1] = csel<C>(ok, v.v[1], fill);
        return r;
    };
    // u (and eps) of plane k with the values of the cells outside the box
    auto masku = [&](P2 v, int k) -> P2 {
        if constexpr (is_face_mode(MODE)) return vmask(v, k, C(0));
        else return mask_out(v, k, uout, uz_lo, uz_hi);
    };
    auto maske = [&](P2 v, int k) -> P2 { return mask_out(v, k, eout, ez_lo, ez_hi); };
    // A ring of R = PD + 3 plane slots for u, eps and b: plane p occupies
    // slot (p - z0 + 1) mod R from its load, PD steps before the step that
    // first reads it, until the step after its own.  The steps are unrolled
    // R at a time, so every slot index is a constant and no loaded value
    // moves between registers (such a move would wait for its load at
    // once).  u and eps are masked in place when their plane first becomes
    // the upper neighbour.
    static_assert(PD >= 1 && PD <= 5, "prefetch depth 1..5");
    constexpr int R = PD + 3;
    P2 su0, su1, su2, su3, su4, su5, su6, su7, se0, se1, se2, se3, se4, se5, se6, se7;
    P2 sb0, sb1, sb2, sb3, sb4, sb5, sb6, sb7;
    auto SU = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return su0; else if constexpr (v == 1) return su1;
        else if constexpr (v == 2) return su2; else if constexpr (v == 3) return su3;
        else if constexpr (v == 4) return su4; else if constexpr (v == 5) return su5;
        else if constexpr (v == 6) return su6; else return su7;
    };
    auto SE = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return se0; else if constexpr (v == 1) return se1;
        else if constexpr (v == 2) return se2; else if constexpr (v == 3) return se3;
        else if constexpr (v == 4) return se4; else if constexpr (v == 5) return se5;
        else if constexpr (v == 6) return se6; else return se7;
    };
    auto SB = [&](auto I) -> P2 & {
        constexpr int v = decltype(I)::value % R;
        if constexpr (v == 0) return sb0; else if constexpr (v == 1) return sb1;
        else if constexpr (v == 2) return sb2; else if constexpr (v == 3) return sb3;
        else if constexpr (v == 4) return sb4; else if constexpr (v == 5) return sb5;
        else if constexpr (v == 6) return sb6; else return sb7;
    };
    // every lane loads every plane (planes past the chunk are not used):
    // loads under a condition would make the compiler wait for all
    // outstanding loads where one of them is used
    auto issue = [&](int k, P2 &du, P2 &de, P2 &db) {
        du = ld_pair(u, k);
        if constexpr (CELL) de = ld_pair(eps, k);
        db = ld_pair(b, k);
    };
    auto issue_at = [&](auto I) {
        constexpr int q = decltype(I)::value;
        if constexpr (q < R) issue(z0 - 1 + q, SU(I), SE(I), SB(I));
    };
    auto mask_at = [&](auto I, int p) {
        SU(I) = masku(SU(I), p);
        if constexpr (CELL) SE(I) = maske(SE(I), p);
    };
    issue_at(std::integral_constant<int, 0>{});
    issue_at(std::integral_constant<int, 1>{});
    issue_at(std::integral_constant<int, 2>{});
    issue_at(std::integral_constant<int, 3>{});
    issue_at(std::integral_constant<int, 4>{});
    issue_at(std::integral_constant<int, 5>{});
    issue_at(std::integral_constant<int, 6>{});
    issue_at(std::integral_constant<int, 7>{});
    mask_at(std::integral_constant<int, 0>{}, z0 - 1);
    mask_at(std::integral_constant<int, 1>{}, z0);
    mask_at(std::integral_constant<int, 2>{}, z0 + 1);
    double nrm = 0.0;
    C acc = C(0);
    // the faces of plane k+1 this pair shares: x face to its right, y faces above
    auto share_faces = [&](const P2 &e1, int k1) __attribute__((always_inline)) {
        if constexpr (CELL) {
            const int q1 = k1 & 1;
            if (live && pc < PXW - 1) s_fx[q1][ry][pc] = harm_face(e1.v[1], s_e[ry][lx + 2]);
            if (live && ry < RY - 1) {
                s_fy[q1][ry][lx] = harm_face(e1.v[0], s_e[ry + 1][lx]);
                s_fy[q1][ry][lx + 1] = harm_face(e1.v[1], s_e[ry + 1][lx + 1]);
            }
        }
    };
    C fzb0 = C(0), fzb1 = C(0);  // vertical faces below plane k (cell coefficients)
    auto step = [&](const P2 &um, const P2 &u0, const P2 &up, const P2 &e_m, const P2 &e0, const P2 &e_p,
                    const P2 &b0, int k) __attribute__((always_inline)) {
        if (live) {
            Pair<C> w;
            w.v[0] = u0.v[0];
            w.v[1] = u0.v[1];
            *reinterpret_cast<Pair<C> *>(&s_u[ry][lx]) = w;
            if constexpr (CELL) {
                w.v[0] = e_p.v[0];
                w.v[1] = e_p.v[1];
                *reinterpret_cast<Pair<C> *>(&s_e[ry][lx]) = w;
            }
        }
        lds_barrier();
        share_faces(e_p, k + 1);
        if (core) {
            C rr[2];
            [[maybe_unused]] C fI = C(0);
            if constexpr (CELL) fI = harm_face(e0.v[0], e0.v[1]);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int lc = lx + c;
                const int gxc = gx + c;
                const C uL = c ? u0.v[0] : s_u[ry][lc - 1], uR = c ? s_u[ry][lc + 1] : u0.v[1];
                const C uD = s_u[ry - 1][lc], uU = s_u[ry + 1][lc];
                C off, dg;
                if constexpr (MODE == COEF_CONST) {
                    off = ((uL + uR) + (uD + uU)) + (um.v[c] + up.v[c]);
                    dg = (c ? dxy1 : dxy0) + (csel<C>(k > 0, C(1), wz_lo) + csel<C>(k < nz - 1, C(1), wz_hi));
                } else if constexpr (MODE == COEF_CELL) {
                    const int q = k & 1;
                    const C fL = c ? fI : s_fx[q][ry][pc - 1];
                    const C fR = c ? s_fx[q][ry][pc] : fI;
                    const C fD = s_fy[q][ry - 1][lc], fU = s_fy[q][ry][lc];
                    const C fB = c ? fzb1 : fzb0, fA = harm_face(e0.v[c], e_p.v[c]);
                    if (c) fzb1 = fA;
                    else fzb0 = fA;
                    off = fL * uL;
                    off = fma_c<C>(fR, uR, off);
                    off = fma_c<C>(fD, uD, off);
                    off = fma_c<C>(fU, uU, off);
                    off = fma_c<C>(fB, um.v[c], off);
                    off = fma_c<C>(fA, up.v[c], off);
                    dg = ((fL + fR) + (fD + fU)) + (fB + fA);
                } else {
                six_faces<C, MODE, true>(
                    G, gxc, gy, k, C(1),
                    [&](int d) -> C {
                        return d == 0   ? (c ? u0.v[0] : s_u[ry][lc - 1])
                               : d == 1 ? (c ? s_u[ry][lc + 1] : u0.v[1])
                               : d == 2 ? s_u[ry - 1][lc]
                               : d == 3 ? s_u[ry + 1][lc]
                               : d == 4 ? um.v[c]
                                        : up.v[c];
                    },
                    [&](int d) -> C {
                        if constexpr (!CELL) return C(1);
                        else return d == 0   ? (c ? e0.v[0] : s_e[ry][lc - 1])
                                    : d == 1 ? (c ? s_e[ry][lc + 1] : e0.v[1])
                                    : d == 2 ? s_e[ry - 1][lc]
                                    : d == 3 ? s_e[ry + 1][lc]
                                    : d == 4 ? e_m.v[c]
                                             : e_p.v[c];
                    },
                    [&](int d) -> C {
                        return d == 0   ? face_x(fbx, G, gxc, gy, k)
                               : d == 1 ? face_x(fbx, G, gxc + 1, gy, k)
                               : d == 2 ? face_y(fby, G, gxc, gy, k)
                               : d == 3 ? face_y(fby, G, gxc, gy + 1, k)
                               : d == 4 ? face_z(fbz, G, gxc, gy, k)
                                        : face_z(fbz, G, gxc, gy, k + 1);
                    },
                    off, dg);
                }
                const C uP = u0.v[c];
                rr[c] = b0.v[c] - a * uP - ih2 * (dg * uP - off);
                if constexpr (MODE == COEF_FACED) rr[c] -= C(A.dd[(size_t)k * plane + (size_t)gy * nx + gxc]) * uP;
            }
            acc += rr[0] + rr[1];
            nrm += (double)rr[0] * (double)rr[0] + (double)rr[1] * (double)rr[1];
        }
        if ((k - z0) & 1) {  // second fine plane of a coarse plane: combine rows
            if (live) s_acc[ry][pc] = acc;
            lds_barrier();
            if (core && !(y & 1)) {
                const C v = C(0.125) * (acc + s_acc[ry + 1][pc]);
                const int I = gx >> 1, J = gy >> 1, K = k >> 1;
                bc[((size_t)K * ncy + J) * ncx + I] = N::cv(v);
            }
            acc = C(0);
        }
        lds_barrier();
    };
    // step k = kk + J of an unrolled group: refill slot J (plane k-2, read
    // last by step k-1) with plane k+1+PD (the chunk's upper neighbour plane
    // once past it), mask plane k+1, step
    auto iter = [&](auto J, int k) __attribute__((always_inline)) {
        constexpr int q = decltype(J)::value;
        using I1 = std::integral_constant<int, q + 1>;
        using I2 = std::integral_constant<int, q + 2>;
        using I3 = std::integral_constant<int, q + 3>;
        issue(min(k + 1 + PD, z1), SU(J), SE(J), SB(J));
        mask_at(I3{}, k + 1);
        step(SU(I1{}), SU(I2{}), SU(I3{}), SE(I1{}), SE(I2{}), SE(I3{}), SB(I2{}), k);
    };
    if constexpr (CELL) {
        // faces of the chunk's first plane, and the vertical faces below it
        if (live) {
            Pair<C> w;
            w.v[0] = se1.v[0];
            w.v[1] = se1.v[1];
            *reinterpret_cast<Pair<C> *>(&s_e[ry][lx]) = w;
        }
        lds_barrier();
        share_faces(se1, z0);
        fzb0 = harm_face(se0.v[0], se1.v[0]);
        fzb1 = harm_face(se0.v[1], se1.v[1]);
        lds_barrier();  // the first step rewrites the eps plane
    }
    step(su0, su1, su2, se0, se1, se2, sb1, z0);
    for (int kk = z0 + 1; kk < z1; kk += R) {
        iter(std::integral_constant<int, 0>{}, kk);
        if (kk + 1 >= z1) break;
        iter(std::integral_constant<int, 1>{}, kk + 1);
        if (kk + 2 >= z1) break;
        iter(std::integral_constant<int, 2>{}, kk + 2);
        if (kk + 3 >= z1) break;
        iter(std::integral_constant<int, 3>{}, kk + 3);
        if constexpr (R > 4) { if (kk + 4 >= z1) break; iter(std::integral_constant<int, 4>{}, kk + 4); }
        if constexpr (R > 5) { if (kk + 5 >= z1) break; iter(std::integral_constant<int, 5>{}, kk + 5); }
        if constexpr (R > 6) { if (kk + 6 >= z1) break; iter(std::integral_constant<int, 6>{}, kk + 6); }
        if constexpr (R > 7) { if (kk + 7 >= z1) break; iter(std::integral_constant<int, 7>{}, kk + 7); }
    }
    return nrm;  // this thread's share of ||r||^2 (A.slot >= 0)
}

// One workgroup per tile, or, where a checked pass has more tiles than
// kMaxRedBlocks, the tiles blockIdx.x, blockIdx.x + gridDim.x, ... with a
// barrier between them; the squared norm is reduced per workgroup.
template <class T, int MODE, int TX, int TY, int PD>
__global__ __launch_bounds__((rr_threads<TX, TY>())) void rr_col_k(RrArgs<T> A) {
    if (A.done_in && *A.done_in) return;
    __shared__ typename Num<T>::C smem[rr_lds<MODE, TX, TY>()];
    double nrm = 0.0;
    for (int t = blockIdx.x; t < A.nblk; t += gridDim.x) {
        if (t != (int)blockIdx.x) __syncthreads();  // LDS of the previous tile is still being read
        nrm += rr_col_body<T, MODE, TX, TY, PD>(A, xcd_remap(t, A.nblk), smem);
    }
    if (A.slot >= 0) reduce2_finish<rr_threads<TX, TY>()>(nrm, 0.0, A.ws, A.slot, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, class TC>
__device__ __forceinline__ void prolong_body(T *__restrict__ u, const TC *__restrict__ e, const Geo &G,
                                             const Geo &Gc, const int I, const int j, const int k) {
    using C = typename Num<T>::C;
    if (I >= Gc.nx || j >= G.ny || k >= G.nz) return;
    const int J = j >> 1, K = k >> 1;
    const int sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
    // coarse value with ghost reflection (sign -1 across a Dirichlet face)
    auto ev = [&](int ii, int jj, int kk) -> C {
        C sg = C(1);
        if (ii < 0) { ii = 0; if (Gc.bcmask & 1) sg = -sg; }
        if (ii >= Gc.nx) { ii = Gc.nx - 1; if (Gc.bcmask & 2) sg = -sg; }
        if (jj < 0) { jj = 0; if (Gc.bcmask & 4) sg = -sg; }
        if (jj >= Gc.ny) { jj = Gc.ny - 1; if (Gc.bcmask & 8) sg = -sg; }
        if (kk < 0) { kk = 0; if (Gc.bcmask & 16) sg = -sg; }
        if (kk >= Gc.nz) { kk = Gc.nz - 1; if (Gc.bcmask & 32) sg = -sg; }
        return sg * C(Num<TC>::ld(e[((size_t)kk * Gc.ny + jj) * Gc.nx + ii]));
    };
    C lo = C(0), mid = C(0), hi = C(0);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const C w = (bb ? C(0.25) : C(0.75)) * (cc ? C(0.25) : C(0.75));
            const int jj = J + bb * sj, kk = K + cc * sk;
            lo += w * ev(I - 1, jj, kk);
            mid += w * ev(I, jj, kk);
            hi += w * ev(I + 1, jj, kk);
        }
    const size_t p = ((size_t)k * G.ny + j) * G.nx + 2 * I;
    const C v0 = C(0.75) * mid + C(0.25) * lo;
    const C v1 = C(0.75) * mid + C(0.25) * hi;
    // u += cw * (P e); cw = 1 adds the correction with one rounding as well
    const C cw = C(G.cw);
    if ((G.nx & 1) == 0) {
        Pair<T> o = *reinterpret_cast<const Pair<T> *>(u + p);
        o.v[0] = Num<T>::cv(fma_c<C>(cw, v0, Num<T>::ld(o.v[0])));
        o.v[1] = Num<T>::cv(fma_c<C>(cw, v1, Num<T>::ld(o.v[1])));
        *reinterpret_cast<Pair<T> *>(u + p) = o;
    } else {
        u[p] = Num<T>::cv(fma_c<C>(cw, v0, Num<T>::ld(u[p])));
        if (2 * I + 1 < G.nx) u[p + 1] = Num<T>::cv(fma_c<C>(cw, v1, Num<T>::ld(u[p + 1])));
    }
}

template <class T, class TC>
__global__ __launch_bounds__(256) void prolong_k(T *__restrict__ u, const TC *__restrict__ e, Geo G,
                                                 Geo Gc, const int *__restrict__ done) {
    if (done && *done) return;
    prolong_body<T, TC>(u, e, G, Gc, blockIdx.x * blockDim.x + threadIdx.x,
                        blockIdx.y * blockDim.y + threadIdx.y, blockIdx.z);
}

// Prolongation, column form: u += P e on a level whose axes are all even.
// A thread owns the fine pair (2I, 2I+1) of fine row j and marches up a
// chunk of fine planes (even start).  The trilinear weights are separable:
// each coarse plane is first combined across its two rows (J and J + sj,
// weights 3/4, 1/4) into three values, for coarse columns I-1, I, I+1,
// which stay in registers for both fine planes that read that coarse plane
// (plane K serves fine planes 2K-1 .. 2K+2).  Ghost values outside the box
// reflect the boundary cell, negated across a Dirichlet face; the signs of
// the x and y ghosts are fixed per thread, those of the z ghosts per plane.
template <class T, int BX, int BY>
__global__ __launch_bounds__(BX *BY) void prolong_col_k(T *__restrict__ u, const T *__restrict__ e, Geo G,
                                                        Geo Gc, int kz, const int *__restrict__ done) {
    if (done && *done) return;
    using N = Num<T>;
    using C = typename N::C;
    const int I = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    if (I >= Gc.nx || j >= G.ny) return;  // no barrier follows
    const int k0 = blockIdx.z * kz, k1 = min(k0 + kz, G.nz);
    const int ncx = Gc.nx, ncy = Gc.ny, ncz = Gc.nz;
    const int J = j >> 1;
    int J2 = J + ((j & 1) ? 1 : -1);
    C sy = C(1);
    if (J2 < 0) { J2 = 0; if (Gc.bcmask & 4) sy = C(-1); }
    if (J2 >= ncy) { J2 = ncy - 1; if (Gc.bcmask & 8) sy = C(-1); }
    int Im = I - 1, Ip = I + 1;
    C sxm = C(1), sxp = C(1);
    if (Im < 0) { Im = 0; if (Gc.bcmask & 1) sxm = C(-1); }
    if (Ip >= ncx) { Ip = ncx - 1; if (Gc.bcmask & 2) sxp = C(-1); }
    const size_t cplane = (size_t)ncx * ncy;
    const size_t r1 = (size_t)J * ncx, r2 = (size_t)J2 * ncx;
    const C wy2 = C(0.25) * sy;
    const C cw = C(G.cw);

    struct R3 { C m, c, p; };
    // coarse plane Kc combined across its two rows (and its ghost sign)
    auto rows = [&](int Kc) -> R3 {
        C sz = C(1);
        if (Kc < 0) { Kc = 0; if (Gc.bcmask & 16) sz = C(-1); }
        if (Kc >= ncz) { Kc = ncz - 1; if (Gc.bcmask & 32) sz = C(-1); }
        const T *pl = e + (size_t)Kc * cplane;
        R3 r;
        r.m = sz * sxm * fma_c<C>(C(0.75), N::ld(pl[r1 + Im]), wy2 * N::ld(pl[r2 + Im]));
        r.c = sz * fma_c<C>(C(0.75), N::ld(pl[r1 + I]), wy2 * N::ld(pl[r2 + I]));
        r.p = sz * sxp * fma_c<C>(C(0.75), N::ld(pl[r1 + Ip]), wy2 * N::ld(pl[r2 + Ip]));
        return r;
    };
    const size_t fplane = (size_t)G.nx * G.ny;
    T *urow = u + (size_t)j * G.nx + 2 * I;
    // fine plane k from coarse planes K = k/2 (weight 3/4) and its z
    // neighbour o (1/4), then along x
    auto apply = [&](int k, const R3 &w0, const R3 &o) {
        const C cm = fma_c<C>(C(0.75), w0.m, C(0.25) * o.m);
        const C cc = fma_c<C>(C(0.75), w0.c, C(0.25) * o.c);
        const C cp = fma_c<C>(C(0.75), w0.p, C(0.25) * o.p);
        const C v0 = fma_c<C>(C(0.75), cc, C(0.25) * cm);
        const C v1 = fma_c<C>(C(0.75), cc, C(0.25) * cp);
        Pair<T> *q = reinterpret_cast<Pair<T> *>(urow + (size_t)k * fplane);
        Pair<T> w = *q;
        // u += cw * (P e); cw = 1 adds the correction with one rounding as well
        w.v[0] = N::cv(fma_c<C>(cw, v0, N::ld(w.v[0])));
        w.v[1] = N::cv(fma_c<C>(cw, v1, N::ld(w.v[1])));
        *q = w;
    };
    const int K0 = k0 >> 1;
    R3 wm = rows(K0 - 1), w0 = rows(K0);
    for (int K = K0; 2 * K < k1; ++K) {
        const R3 wp = rows(K + 1);
        apply(2 * K, w0, wm);
        if (2 * K + 1 < k1) apply(2 * K + 1, w0, wp);
        wm = w0;
        w0 = wp;
    }
}

// ||b - A u||^2 and (optionally) ||b + boundary terms||^2 over bricks of
// blockDim.x x blockDim.y cells and kz planes, gx x gy x gz of them; a
// workgroup sums the bricks blockIdx.x, blockIdx.x + gridDim.x, ... (one
// brick each unless the grid has more bricks than kMaxRedBlocks).
template <class T, int MODE>
__global__ __launch_bounds__(256) void norm2_resid_k(const T *__restrict__ u, const T *__restrict__ b,
                                                     const coef_t<T> *__restrict__ eps,
                                                     const coef_t<T> *__restrict__ bx,
                                                     const coef_t<T> *__restrict__ by,
                                                     const coef_t<T> *__restrict__ bz, Geo G, RedWs ws,
                                                     int slot, int bslot, int kz, int gx, int gy, int nbrick,
                                                     const int *__restrict__ done_in,
                                                     const double *__restrict__ dd = nullptr) {
    if (done_in && *done_in) return;
    using N = Num<T>;
    double sr = 0.0, sb = 0.0;
    for (int t = blockIdx.x; t < nbrick; t += gridDim.x) {
        const int i = (t % gx) * blockDim.x + threadIdx.x;
        const int j = ((t / gx) % gy) * blockDim.y + threadIdx.y;
        const int k0 = (t / gx / gy) * kz;
        const int k1 = min(k0 + kz, G.nz);
        if (i >= G.nx || j >= G.ny) continue;
        for (int k = k0; k < k1; ++k) {
            const size_t p = ((size_t)k * G.ny + j) * G.nx + i;
            const double rv = (double)resid_global<T, MODE>(u, b, eps, bx, by, bz, G, i, j, k, dd);
            sr += rv * rv;
            if (bslot >= 0) {
                // b + h^-2 sum_Dirichlet 2 beta_b g  (boundary beta as in the operator)
                double be = 1.0;
                if constexpr (MODE == COEF_CELL) be = (double)Num<coef_t<T>>::ld(eps[p]);
                double add = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const bool at = d == 0   ? i == 0
                                    : d == 1 ? i == G.nx - 1
                                    : d == 2 ? j == 0
                                    : d == 3 ? j == G.ny - 1
                                    : d == 4 ? k == 0
                                             : k == G.nz - 1;
                    if (at && ((G.bcmask >> d) & 1)) {
                        double bf = be;
                        if constexpr (is_face_mode(MODE)) {
                            bf = d == 0   ? (double)face_x(bx, G, i, j, k)
                                 : d == 1 ? (double)face_x(bx, G, i + 1, j, k)
                                 : d == 2 ? (double)face_y(by, G, i, j, k)
                                 : d == 3 ? (double)face_y(by, G, i, j + 1, k)
                                 : d == 4 ? (double)face_z(bz, G, i, j, k)
                                          : (double)face_z(bz, G, i, j, k + 1);
                        }
                        add += 2.0 * bf * G.g[d];
                    }
                }
                const double bb = (double)N::ld(b[p]) + G.ih2 * add;
                sb += bb * bb;
            }
        }
    }
    reduce2_finish<256>(sr, sb, ws, slot, blockIdx.x);
}

}  // namespace mg
