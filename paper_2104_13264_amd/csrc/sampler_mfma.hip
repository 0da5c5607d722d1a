// Batched sampler on the matrix cores: the same sequential draw and the same
// conditionals as the plain path (Sec. 2 Eqs. bayes, pi-approx; App. A
// Eq. proba-ratio-apx), with the per-column products run as 16x16 MFMA tiles
// (FP32 16x16x4, BF16 16x16x32 with FP32 accumulation, or FP64 16x16x4).
// The precision mode PM selects the operands and the vector arithmetic: FP32
// and BF16 vectors are fp32, FP64 vectors are fp64.
//
// Each wavefront owns 16 proposals (the N dimension of every tile) for the
// whole lattice.  Per row, in snake order (row r drawn left to right when r is
// even), the environments of the row's free columns are swept from its far
// end and then the row is drawn:
//   environment sweep  y_s = G_c(s) r_s for both spins (K = Dp chained MFMAs),
//                stored to scratch; r_s' = sum_s W(s', s) v_c(s) y_s
//   drawing      w(s) = v hf <Lam, y_s>, p+ and the draw in fp64, and
//                Lam G_c(s) for both spins, of which each lane keeps its
//                proposal's drawn spin.
// The accumulator layout of tile mt (lane l, register i -> row 4(l/16)+i,
// column l%16) is exactly the B-operand layout of k-chunk q = 4 mt + i of the
// next product, so the recurrences stay in registers; the A operands (the
// shared environment) are pre-permuted to match (operands.hip).
//
// Scaling: a product takes its input vector as it comes and multiplies its
// output by 2^-e, e the binary exponent of the input's largest entry (common to
// all tiles); powers of two are exact, so this equals rescaling the input first.
// ln q is accumulated as two fp64 products, of the drawn weights and of the
// weight totals, each with a separate binary exponent, and evaluated once at
// the end; the spin is +1 iff u * (w+ + w-) < w+.  In FP32 and BF16, weights
// below 2^-24 of |w+| + |w-| are raised to that floor; in FP64, negative
// weights are clamped to 0, as in the plain path.
//
// Proposal j of the launch has id first_id + j % per_step and MH step
// step0 + j / per_step (several steps' proposals may share a launch; the
// proposal distribution does not depend on the chains' state).
#include "common.hpp"

// No implicit fusion of products into sums: the launch variants of the team
// kernel must round alike, and the compiler's choice of which product of an
// expression to fuse may differ between instantiations.  Fused operations are
// written out (fmaf).
#include <type_traits>

#pragma clang fp contract(off)

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

// Precision modes of the team kernel.
constexpr int PM_F32 = 0, PM_BF16 = 1, PM_F64 = 2;
template <int PM>
struct Arith {   // fp32 vectors (FP32 and BF16 operands)
    using E = float;
    using V4 = floatx4;
};
template <>
struct Arith<PM_F64> {
    using E = double;
    using V4 = doublex4;
};
constexpr int team_variants(int NT, int PM) { return PM == PM_F64 ? 1 : tn_team_variants(NT, PM == PM_BF16); }

#define TN_MAX_LX 256

__device__ __forceinline__ int pow2_exponent_f(float m) {
    int e = 0;
    if (m > 0.0f && m <= 3.0e38f) frexpf(m, &e);
    return e;
}
__device__ __forceinline__ int pow2_exponent_f(double m) {
    int e = 0;
    if (m > 0.0 && m <= 1.79e308) frexp(m, &e);
    return e;
}
__device__ __forceinline__ float fma_e(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_e(double a, double b, double c) { return fma(a, b, c); }

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx2 __attribute__((ext_vector_type(2)));

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// Two four-entry bf16 pieces as the eight-entry operand of the 16x16x32 product.
__device__ __forceinline__ bf16x8 cat8(const shortx4 lo, const shortx4 hi) {
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Four floats to bf16 with round-to-nearest-even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ shortx4 bf16x4_rne(const floatx4 v) {
    const floatx2 lo = {v[0], v[1]}, hi = {v[2], v[3]};
    const bf16x2 a = __builtin_convertvector(lo, bf16x2), b = __builtin_convertvector(hi, bf16x2);
    return __builtin_bit_cast(shortx4, uintx2{__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)});
}

// Buffer resource over [base, base + bytes): loads and stores take a 32-bit
// per-lane offset and a wave-uniform column offset; accesses outside the
// range read 0 / are dropped.
// Cache policy of the FP32 y tiles (FP32 and BF16 operands): non-temporal.
// Each byte is written once and read once, a whole row sweep later, and the
// tiles in flight (hundreds of MB) outgrow L2 and the MALL; marked
// non-temporal they do not displace the environment operands, which every
// team of the launch re-reads from L2 (variant 2 at the 64x64, D = 32
// headline: 38.1 -> 35.6 ms per 20-step launch).  The recomputing variant's
// checkpoints (tens of MB per launch) and the FP64 tiles keep the default
// policy: marked non-temporal they ran slower (the BF16 recomputing launch
// 20.3 -> 22.8 ms).
constexpr int SCR_POLICY = 2;   // the nt bit of the buffer instructions' cache policy

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

// The same pointer or offset as a wave-uniform (scalar) value: buffer
// resources and scalar offsets must be uniform, and the compiler cannot
// always prove it.
__device__ __forceinline__ const char *uniform_ptr(const void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const char *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// A operands of one spin's product for one column, per lane: every 16-row
// output block mo = 0..NT-1 with the 4 NT k-chunks of the fp32 or fp64
// 16x16x4 product or the NT chunks of the bf16 products (16 k each).  Tile layout
// per site: [s][mo][mt][64 lanes][4 chunks] (fp32: 16 bytes per lane; bf16: 8;
// fp64: 32).
template <int NT, int PM>
struct ATiles {
    static constexpr int NQ = 4 * NT;
    static constexpr size_t SITE_BYTES = (size_t)2 * NT * NQ * 64 * 4;
    float a[NT][NQ];
};

template <int NT>
struct ATiles<NT, PM_BF16> {
    static constexpr size_t SITE_BYTES = (size_t)2 * NT * NT * 64 * 8;
    shortx4 a[NT][NT];
};

template <int NT>
struct ATiles<NT, PM_F64> {
    static constexpr int NQ = 4 * NT;
    static constexpr size_t SITE_BYTES = (size_t)2 * NT * NQ * 64 * 8;
    double a[NT][NQ];
};

// Sum (or max) over the four 16-lane rows of a wavefront, the same result in
// every lane: the 32-lane and 16-lane swaps of gfx950 (VALU, no LDS traffic).
__device__ __forceinline__ float rows4_max(float v) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
}
// Both sums at once: after the first swap-and-add, lanes 0-31 hold a's
// half-sums and lanes 32-63 b's; the second pairs the 16-lane rows; a last
// swap hands every lane both totals.  Every lane adds in the same order.
__device__ __forceinline__ void rows4_sum2(float &a, float &b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    float v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(q[0]) + __uint_as_float(q[1]);
    auto z = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    a = __uint_as_float(z[0]);
    b = __uint_as_float(z[1]);
}

// The same for fp64 values: the swaps move the two 32-bit halves.
__device__ __forceinline__ void swap32_pair(double v0, double v1, double &r0, double &r1) {
    auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)__double2loint(v0), (uint32_t)__double2loint(v1), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)__double2hiint(v0), (uint32_t)__double2hiint(v1), false, false);
    r0 = __hiloint2double((int)hi[0], (int)lo[0]);
    r1 = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16_pair(double v0, double v1, double &r0, double &r1) {
    auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)__double2loint(v0), (uint32_t)__double2loint(v1), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)__double2hiint(v0), (uint32_t)__double2hiint(v1), false, false);
    r0 = __hiloint2double((int)hi[0], (int)lo[0]);
    r1 = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double rows4_max(double v) {
    double a, b;
    swap32_pair(v, v, a, b);
    v = fmax(a, b);
    swap16_pair(v, v, a, b);
    return fmax(a, b);
}
__device__ __forceinline__ void rows4_sum2(double &a, double &b) {
    double r0, r1;
    swap32_pair(a, b, r0, r1);
    double v = r0 + r1;
    swap16_pair(v, v, r0, r1);
    v = r0 + r1;
    swap32_pair(v, v, r0, r1);
    a = r0;
    b = r1;
}

// LDS arrays indexed by proposal keep the proposal index innermost, so the 16
// proposals of a wavefront touch 16 consecutive entries (no bank conflicts).
constexpr int RS = 4;   // rescale (and ln q renormalisation) period in columns

// Products of both spins' tiles, the four (2 NT) accumulation chains
// interleaved: acc[s] = A[s] x[s].
template <int NT, int PM>
__device__ __forceinline__ void mul_both(const ATiles<NT, PM> (&a)[2], const typename Arith<PM>::V4 (&x0)[NT],
                                         const typename Arith<PM>::V4 (&x1)[NT],
                                         typename Arith<PM>::V4 (&acc)[2][NT]) {
    using V4 = typename Arith<PM>::V4;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int mo = 0; mo < NT; ++mo) acc[sp][mo] = V4{0, 0, 0, 0};
    if constexpr (PM == PM_F64) {
#pragma unroll
        for (int q = 0; q < 4 * NT; ++q)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                acc[0][mo] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0].a[mo][q], x0[q >> 2][q & 3], acc[0][mo], 0, 0, 0);
                acc[1][mo] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1].a[mo][q], x1[q >> 2][q & 3], acc[1][mo], 0, 0, 0);
            }
    } else if constexpr (PM == PM_BF16) {
        shortx4 b0[NT], b1[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            b0[mt] = bf16x4_rne(x0[mt]);
            b1[mt] = bf16x4_rne(x1[mt]);
        }
        // k-chunks in pairs on the 16x16x32 product: a lane's eight operand
        // entries are its four of chunk 2p followed by its four of chunk
        // 2p + 1, on both sides, so every A entry meets the B entry of the
        // same vector index; an odd last chunk on the 16x16x16 product
#pragma unroll
        for (int p = 0; p + 1 < NT; p += 2)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                acc[0][mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8(a[0].a[mo][p], a[0].a[mo][p + 1]),
                                                                     cat8(b0[p], b0[p + 1]), acc[0][mo], 0, 0, 0);
                acc[1][mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8(a[1].a[mo][p], a[1].a[mo][p + 1]),
                                                                     cat8(b1[p], b1[p + 1]), acc[1][mo], 0, 0, 0);
            }
        if constexpr (NT & 1)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                acc[0][mo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0].a[mo][NT - 1], b0[NT - 1], acc[0][mo], 0, 0, 0);
                acc[1][mo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1].a[mo][NT - 1], b1[NT - 1], acc[1][mo], 0, 0, 0);
            }
    } else {
#pragma unroll
        for (int q = 0; q < 4 * NT; ++q)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                acc[0][mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0].a[mo][q], x0[q >> 2][q & 3], acc[0][mo], 0, 0, 0);
                acc[1][mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1].a[mo][q], x1[q >> 2][q & 3], acc[1][mo], 0, 0, 0);
            }
    }
}

// ---------------------------------------------------------------------------
// Teams of TW wavefronts sharing the environment tiles.
//
// Each wave owns SETS sets of 16 proposals (two for D <= 32, one above).  It
// keeps both spins' operands and all its sets' vectors in registers and runs
// the environment sweep of a row and then its drawing, row after row: per
// column the sweep chains 2 NT independent MFMA accumulations per set (both
// spins), stores y_s and mixes r_s' = sum_s W(s', s) v_c(s) y_s in place; the
// drawing multiplies Lam by both G_c(s)^T, forms w(s) = v hf <Lam, y_s> from
// the stored tiles, draws, and keeps the drawn spin's product lane by lane.
// No tile crosses a wave.  With two sets the fp64 draw serves both at once:
// lanes 0-31 decide set 0, lanes 32-63 set 1, and a permlane32 swap hands
// every lane both sets' spins.
//
// The team walks the rows and columns in lock step and fetches the tiles of a
// column once, straight into a ring of LDS stages (global_load_lds, TL columns
// ahead; each wave fetches an equal share), from which every wave reads its
// operands one column ahead.  One barrier per column keeps the ring
// consistent: at column t a wave reads stage t, refills the stage of column
// t - 1 with column t + TL - 1, waits for its own fetch of column t + 1 and
// meets the others at the barrier.  The per-row factor tables are built once
// per team.  Sharing the fetch divides the operand traffic by TW and keeps the
// waves of a team on the same tiles, so they stay in L2 even when other work
// runs between launches.
constexpr int TW = 4;   // waves per team

// Per bond class and launch variant V: TL LDS stages (columns in flight);
// SETS: 16-proposal sets per wave; WPE: waves per SIMD the registers allow;
// ABUF: operand register sets (two: read one column ahead; one: read just in
// time).  The variants differ in launch shape and in where the y tiles live,
// never in the arithmetic of a proposal; an autotuner picks one
// (tn_autotune):
//   V = 0  two sets per wave, two waves per SIMD (D 33-64: one set, one wave)
//   V = 1  one set per wave, two waves per SIMD (half the LDS per team)
//   V = 2  one set per wave, three waves per SIMD
//   last   (V = 3 for D <= 32, V = 1 for BF16 D 33-64) recomputing: no y tiles
//          in scratch.  The sweep keeps only a checkpoint of its state per
//          block of BR columns; the draw, block by block, sweeps the block's
//          columns again from its checkpoint with the y tiles in registers
//          and then draws them.  It moves 1/BR of the tile traffic for half
//          again the products (the per-proposal y tiles of a row outgrow
//          every cache, and BF16 products are cheap next to HBM bytes).
template <int NT, int PM, int V>
struct TeamCfg {
    static_assert(V >= 0 && V < team_variants(NT, PM), "no such variant for this bond class");
    static constexpr bool BF16 = PM == PM_BF16, F64 = PM == PM_F64;
    static constexpr uint32_t STAGE = (uint32_t)ATiles<NT, PM>::SITE_BYTES;   // both spins
    static constexpr uint32_t LANE = STAGE % (TW * 64 * 16) == 0 ? 16 : 4;     // dwordx4 or dword fetches
    static constexpr int LOADS = (int)(STAGE / (TW * 64 * LANE));            // per wave per column
    static_assert(LOADS * TW * 64 * LANE == STAGE, "stage must split evenly");
    static constexpr bool REC = (NT <= 2 && !F64 && V == 3) || (NT > 2 && BF16 && V == 1);
    static constexpr int BR = !REC ? 1 : NT == 1 ? 8 : NT == 2 ? 4 : 2;   // columns per block (registers)
    // D > 32: one team per CU holds the LDS; four BF16 stages fit beside the
    // row tables up to Lx = 256 (about 122 KB), three FP32 ones (about 154 KB)
    static constexpr int TL = (NT <= 2 || BF16) ? 4 : 3;
    static constexpr int SETS = (NT <= 2 && V == 0 && !F64) ? 2 : 1;
    // FP64 at D = 32: two waves per SIMD with a small spill (24 registers)
    // beat one with every value in registers (4.13 against 4.61 ms per 4096
    // proposals at 64x64; two 80 KB teams fill a CU's LDS at Lx = 64)
    static constexpr int WPE = F64 ? 2 : REC ? (NT <= 2 ? 2 : 1) : (NT <= 2 ? (V == 2 ? 3 : 2) : 1);
    static constexpr int ABUF = F64 ? (NT == 1 ? 2 : 1) : ((BF16 || NT <= 2) ? 2 : 1);
    static constexpr int PT = TW * 16 * SETS;   // proposals per team
};

struct TeamSmem {
    int ring, rows, mixP, vS, epart, total;
    __host__ __device__ TeamSmem(int Lx, uint32_t stage, int tl, int pt) {
        ring = 0;                                        // [TL][stage bytes]
        rows = ring + tl * (int)stage;                   // int8 [2 parity][Lx][pt]
        mixP = rows + ((2 * Lx * pt + 15) & ~15);        // float [Lx][s_up][s'][s]
        vS = mixP + Lx * 8 * 4;                          // double [Lx][s_up][s_prev][s]
        epart = vS + Lx * 8 * 8;                         // double [TW][sets][4][16]
        total = epart + pt * 4 * 8;
    }
};

template <uint32_t LANE>
__device__ __forceinline__ void lds_fetch(const char *g, __attribute__((address_space(3))) void *l) {
    static_assert(LANE == 16 || LANE == 4, "fetch width");
    if constexpr (LANE == 16) __builtin_amdgcn_global_load_lds((const void *)g, l, 16, 0, 0);
    else __builtin_amdgcn_global_load_lds((const void *)g, l, 4, 0, 0);
}

// wait until at most N vector-memory operations of this wave are in flight
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Barrier of the team's column steps.  __syncthreads() would also wait for
// every memory operation in flight (the LDS fetches count as such), which
// would drain the ring at every column; here each wave has already waited for
// its own fetch of the stage read next, so a bare s_barrier suffices.  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void team_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int NT, int PM>
__device__ __forceinline__ void lds_tiles(ATiles<NT, PM> &a, const unsigned char *st, int lane) {
    if constexpr (PM == PM_F64) {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) {
                const doublex2 v0 = *(const doublex2 *)(st + ((mo * NT + mt) * 64 + lane) * 32);
                const doublex2 v1 = *(const doublex2 *)(st + ((mo * NT + mt) * 64 + lane) * 32 + 16);
                a.a[mo][4 * mt + 0] = v0[0];
                a.a[mo][4 * mt + 1] = v0[1];
                a.a[mo][4 * mt + 2] = v1[0];
                a.a[mo][4 * mt + 3] = v1[1];
            }
    } else if constexpr (PM == PM_BF16) {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
                a.a[mo][mt] = *(const shortx4 *)(st + ((mo * NT + mt) * 64 + lane) * 8);
    } else {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) {
                const floatx4 v = *(const floatx4 *)(st + ((mo * NT + mt) * 64 + lane) * 16);
#pragma unroll
                for (int i = 0; i < 4; ++i) a.a[mo][4 * mt + i] = v[i];
            }
    }
}

template <int NT, int PM, int V>
__device__ __forceinline__ void team_body(const tn_samp_desc &A, const int unit0, const int eval,
                                          const uint32_t k0, const uint32_t k1, const uint64_t step0) {
    if (unit0 * 16 >= A.B) return;   // a team with no proposal of its instance (uniform)
    using AT = ATiles<NT, PM>;
    using CF = TeamCfg<NT, PM, V>;
    using ET = typename Arith<PM>::E;
    using V4 = typename Arith<PM>::V4;
    constexpr bool F64 = PM == PM_F64;
    constexpr uint32_t YB = sizeof(V4);   // bytes of one y tile per lane
    constexpr int TL = CF::TL, SE = CF::SETS, PT = CF::PT;
    constexpr int CG = 4 / SE;                 // column groups of a set's energy
    const int B = A.B, Lx = A.Lx, Ly = A.Ly, per_step = A.per_step;
    const double *__restrict__ Jh = A.Jh;
    const double *__restrict__ Jv = A.Jv;
    const double *__restrict__ h = A.h;
    const double *__restrict__ fac = A.fac;
    int8_t *__restrict__ S = A.S;
    const uint32_t inst = A.inst;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, grp = lane >> 4;
    // Every lane holds tiles of all SE sets (proposal n of each); the scalar
    // work of the draw is split: with two sets, lanes 0-31 take set 0 and
    // lanes 32-63 set 1 (the lane's draw set ds).
    const int ds = SE == 2 ? (lane >> 5) : 0;
    const int cg = grp % CG;
    auto slot = [&](int st) { return (w * SE + st) * 16 + n; };   // slot in the team
    const int pd = slot(ds);
    const int bd = (unit0 + w * SE + ds) * 16 + n;   // the draw set's proposal
    const bool valid = bd < B;

    extern __shared__ __align__(16) unsigned char smem[];
    const TeamSmem L(Lx, CF::STAGE, TL, PT);
    unsigned char *ring = smem + L.ring;
    float(*mixP)[2][2][2] = (float(*)[2][2][2])(smem + L.mixP);
    double(*vS)[2][2][2] = (double(*)[2][2][2])(smem + L.vS);
    double(*epart)[SE][4][16] = (double(*)[SE][4][16])(smem + L.epart);
    auto rowbuf = [&](int par) { return (int8_t(*)[PT])(smem + L.rows + par * Lx * PT); };

    const uint32_t gstride = 2u * NT * 64 * YB;   // bytes of stored y tiles per column
    __amdgpu_buffer_rsrc_t grs[SE];
#pragma unroll
    for (int st = 0; st < SE; ++st)
        grs[st] = make_rsrc(uniform_ptr(A.gscr + (size_t)(unit0 + w * SE + st) * Lx * (gstride / 4)),
                            uniform_u32((uint32_t)Lx * gstride));
    // this wave's share of a stage: LOADS chunks of 64 lanes x LANE bytes
    const uint32_t share = (uint32_t)w * CF::LOADS * 64 * CF::LANE;
    // Checkpoints of the recomputing variant, in the set's scratch: block b's
    // entry state, r_+ and r_- as the products read them (bf16 in BF16 mode)
    // and the rescale exponent of each lane.
    constexpr uint32_t CPV = CF::BF16 ? 8 : 16;              // bytes per lane of a 4-entry piece
    constexpr uint32_t CPB = 2 * NT * 64 * CPV + 64 * 4;     // bytes per checkpoint
    auto cp_save = [&](int b, const V4 (&v0)[NT], const V4 (&v1)[NT], int e) {
        if constexpr (CF::REC) {
            const uint32_t base = uniform_u32((uint32_t)b * CPB);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) {
                    const V4 &v = sp ? v1[mo] : v0[mo];
                    const uint32_t off = (uint32_t)(((sp * NT + mo) * 64 + lane) * CPV);
                    if constexpr (CF::BF16)
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(uintx2, bf16x4_rne(v)), grs[0], off, base, 0);
                    else
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, v), grs[0], off, base, 0);
                }
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)e, grs[0], (uint32_t)(2 * NT * 64 * CPV + lane * 4), base, 0);
        }
    };
    auto cp_load = [&](int b, V4 (&v0)[NT], V4 (&v1)[NT], int &e) {
        if constexpr (CF::REC) {
            const uint32_t base = uniform_u32((uint32_t)b * CPB);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) {
                    V4 &v = sp ? v1[mo] : v0[mo];
                    const uint32_t off = (uint32_t)(((sp * NT + mo) * 64 + lane) * CPV);
                    if constexpr (CF::BF16) {
                        const uintx2 h = __builtin_amdgcn_raw_buffer_load_b64(grs[0], off, base, 0);
                        v = V4{__uint_as_float(h[0] << 16), __uint_as_float(h[0] & 0xffff0000u),
                               __uint_as_float(h[1] << 16), __uint_as_float(h[1] & 0xffff0000u)};
                    } else {
                        v = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(grs[0], off, base, 0));
                    }
                }
            e = (int)__builtin_amdgcn_raw_buffer_load_b32(grs[0], (uint32_t)(2 * NT * 64 * CPV + lane * 4), base, 0);
        }
    };
    // random words of the draw set's proposal, drawn as the row goes: one
    // Philox block per four sites, kept for the next sites
    const uint32_t jj = (uint32_t)(bd);
    const uint64_t wid = A.first_id + jj % (uint32_t)per_step;
    const uint32_t wst = (uint32_t)(step0 + jj / (uint32_t)per_step);

    double num = 1.0, den = 1.0, E = 0.0;   // ln q = ln(num / den) + nexp ln 2
    int nexp = 0;
    uint32_t n_clamp = 0, n_both = 0, n_near = 0;

    for (int r = 0; r < Ly; ++r) {
        const bool drawR = (r & 1) == 0;
        __syncthreads();   // the previous row's readers are done with the tables
        for (int t = threadIdx.x; t < Lx * 8; t += TW * 64) {
            const int c = t >> 3, su = (t >> 2) & 1, x = (t >> 1) & 1, sg = t & 1;
            const double *f = fac + ((size_t)r * Lx + c) * 6;
            const double v = f[sg] * f[2 + (su ^ sg)];
            const int cw = drawR ? c : c + 1;
            double Wv = 1.0;
            if (cw >= 1 && cw <= Lx - 1) Wv = fac[((size_t)r * Lx + cw) * 6 + ((x == sg) ? 4 : 5)];
            mixP[c][su][x][sg] = (float)(Wv * v);
            vS[c][su][x][sg] = v * Wv;   // the same bond, towards the previous drawn column
        }
        int8_t(*crow)[PT] = rowbuf(r & 1);
        const int8_t(*prow)[PT] = rowbuf((r + 1) & 1);
        if (eval) {
            for (int t = threadIdx.x; t < PT * Lx; t += TW * 64) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = unit0 * 16 + nn;
                crow[c][nn] = bb < B ? S[((size_t)bb * Ly + r) * Lx + c] : (int8_t)1;
            }
        }
        const size_t rowb = (size_t)r * Lx;
        // Operands of the sweep come in its order (from the far end of the
        // row), those of the draw in the draw order.  The recomputing variant
        // reads, per block of BR draw columns, the block's sweep columns and
        // then its draw columns: stream position q of its draw role is
        // column step o = q mod 2 BR of block q / 2 BR.
        auto cols = [&](int t) { return drawR ? Lx - 1 - t : t; };   // sweep step -> column
        auto cold = [&](int t) { return drawR ? t : Lx - 1 - t; };   // draw step -> column
        const char *Gsw = uniform_ptr((const char *)(drawR ? A.GR : A.GL) + rowb * AT::SITE_BYTES);
        const char *Gdr = uniform_ptr((const char *)(drawR ? A.GL : A.GR) + rowb * AT::SITE_BYTES);
        for (int role = 0; role < 2; ++role) {
            const bool sweep = role == 0;
            auto src_of = [&](int q) -> const char * {
                if constexpr (CF::REC) {
                    if (!sweep) {
                        const int b = q / (2 * CF::BR), o = q - b * (2 * CF::BR);
                        if (o < CF::BR)
                            return Gsw + (size_t)cols(min(max(Lx - (b + 1) * CF::BR + o, 0), Lx - 1)) * AT::SITE_BYTES;
                        return Gdr + (size_t)cold(min(b * CF::BR + o - CF::BR, Lx - 1)) * AT::SITE_BYTES;
                    }
                }
                return sweep ? Gsw + (size_t)cols(min(q, Lx - 1)) * AT::SITE_BYTES
                             : Gdr + (size_t)cold(min(q, Lx - 1)) * AT::SITE_BYTES;
            };
            auto issue = [&](int q) {   // stage q % TL <- the operands of stream position q
                const char *src = src_of(q) + share + lane * CF::LANE;
                unsigned char *dst = ring + (q % TL) * CF::STAGE + share;
#pragma unroll
                for (int j = 0; j < CF::LOADS; ++j)
                    lds_fetch<CF::LANE>(src + j * 64 * CF::LANE,
                                        (__attribute__((address_space(3))) void *)(dst + j * 64 * CF::LANE));
            };
            __syncthreads();   // tables and spins of the row; the ring is free
#pragma unroll
            for (int t = 0; t < TL - 1; ++t) issue(t);
            wait_vm<(TL - 2) * CF::LOADS>();   // own share of column 0 has landed
            __syncthreads();
            AT a[CF::ABUF][2];   // [set of registers][spin]
            lds_tiles<NT, PM>(a[0][0], ring, lane);
            lds_tiles<NT, PM>(a[0][1], ring + CF::STAGE / 2, lane);
            // next stream position: own fetch has landed (at most N ops issued
            // after it in flight; N < 0: the step has waited already), the
            // team meets, the operands go to registers
            auto ring_next = [&](int k, int q, auto nops) __attribute__((always_inline)) {
                if constexpr (decltype(nops)::value >= 0) wait_vm<decltype(nops)::value>();
                team_barrier();
                const unsigned char *stg = ring + ((q + 1) % TL) * CF::STAGE;
                lds_tiles<NT, PM>(a[(k ^ 1) % CF::ABUF][0], stg, lane);
                lds_tiles<NT, PM>(a[(k ^ 1) % CF::ABUF][1], stg + CF::STAGE / 2, lane);
            };
            // One sweep column for every set: y_s = G_c(s) r_s, rescaled, goes
            // to keep(st, y); r_s' = sum_s W(s', s) v_c(s) y_s replaces r; the
            // exponent of the next rescale.  mid() runs after the products are
            // issued (the stage fetch).
            auto sweep_col = [&](int k, int t, V4 (&v0)[SE][NT], V4 (&v1)[SE][NT], int (&e)[SE], auto &&mid,
                                 auto &&keep) __attribute__((always_inline)) {
                const int c = cols(t);
                V4 acc[SE][2][NT];
#pragma unroll
                for (int st = 0; st < SE; ++st) mul_both<NT, PM>(a[k % CF::ABUF], v0[st], v1[st], acc[st]);
                mid();
#pragma unroll
                for (int st = 0; st < SE; ++st) {
                    const bool up_minus = r > 0 && prow[c][slot(st)] < 0;
                    ET m[4];   // the mixing weights W(s', s) v_c(s), fp32 (or fp64 in FP64 mode)
                    if constexpr (F64) {
                        const doublex2 m01 = *(const doublex2 *)&vS[c][up_minus ? 1 : 0][0][0];
                        const doublex2 m23 = *(const doublex2 *)&vS[c][up_minus ? 1 : 0][1][0];
                        m[0] = m01[0];
                        m[1] = m01[1];
                        m[2] = m23[0];
                        m[3] = m23[1];
                    } else {
                        const floatx4 mf = *(const floatx4 *)&mixP[c][up_minus ? 1 : 0][0][0];
#pragma unroll
                        for (int i = 0; i < 4; ++i) m[i] = mf[i];
                    }
                    if (t % RS == 0 && t > 0) {
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[st][sp][mo][i] = ldexp(acc[st][sp][mo][i], -e[st]);
                    }
                    keep(st, c, acc[st]);
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            v0[st][mo][i] = fma_e(m[1], acc[st][1][mo][i], m[0] * acc[st][0][mo][i]);
                            v1[st][mo][i] = fma_e(m[3], acc[st][1][mo][i], m[2] * acc[st][0][mo][i]);
                        }
                    if (t % RS == RS - 1) {
                        ET mx = 0;
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int i = 0; i < 4; ++i) mx = fmax(mx, fabs(acc[st][sp][mo][i]));
                        e[st] = pow2_exponent_f(rows4_max(mx));
                    }
                }
            };
            auto init_state = [&](V4 (&v0)[SE][NT], V4 (&v1)[SE][NT], int (&e)[SE]) {
#pragma unroll
                for (int st = 0; st < SE; ++st) {
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt) v0[st][mt] = v1[st][mt] = V4{0, 0, 0, 0};
                    if (grp == 0) v0[st][0][0] = v1[st][0][0] = 1;
                    e[st] = 0;
                }
            };
            if (sweep) {
                V4 v0[SE][NT], v1[SE][NT];   // r_+ and r_- of every set
                int e[SE];
                init_state(v0, v1, e);
                // the y tiles go to scratch for the draw; the recomputing
                // variant instead keeps the state entering each draw block's
                // first sweep column (a checkpoint per BR columns)
                auto store_y = [&](int st, int c, const V4 (&y)[2][NT]) {
                    if constexpr (!CF::REC) {
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo) {
                                if constexpr (F64) {
                                    const doublex2 lo = {y[sp][mo][0], y[sp][mo][1]};
                                    const doublex2 hi = {y[sp][mo][2], y[sp][mo][3]};
                                    const uint32_t off = (uint32_t)(((sp * NT + mo) * 64 + lane) * 32);
                                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, lo), grs[st], off,
                                                                           uniform_u32((uint32_t)c * gstride), 0);
                                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, hi), grs[st], off + 16,
                                                                           uniform_u32((uint32_t)c * gstride), 0);
                                } else {
                                    __builtin_amdgcn_raw_buffer_store_b128(
                                        __builtin_bit_cast(uintx4, y[sp][mo]), grs[st],
                                        (uint32_t)(((sp * NT + mo) * 64 + lane) * 16), uniform_u32((uint32_t)c * gstride),
                                        SCR_POLICY);
                                }
                            }
                    }
                };
                // Own fetch of column t + 1 has landed once at most the loads
                // issued after it are in flight: (TL - 2) stage fetches, in
                // every step (positions past the row's end fetch its last
                // column again).  The y
                // stores are not counted, since the counter may drop for a
                // store before it drops for an earlier load; so the wait sits
                // right after this step's fetch, before this step's stores,
                // where pending stores are those of earlier steps.
                constexpr int NW = (TL - 2) * CF::LOADS;
                auto stepP = [&](int k, int t) {
                    if constexpr (CF::REC)
                        if (t > 0 && (Lx - t) % CF::BR == 0) cp_save((Lx - t) / CF::BR - 1, v0[0], v1[0], e[0]);
                    sweep_col(k, t, v0, v1, e, [&] {
                        issue(t + TL - 1);
                        wait_vm<NW>();
                    }, store_y);
                    ring_next(k, t, std::integral_constant<int, -1>{});
                };
                int t = 0;
                for (; t + 2 <= Lx; t += 2) {
                    stepP(0, t);
                    stepP(1, t + 1);
                }
                if (t < Lx) stepP(0, t);
            } else {
                V4 lam[SE][NT];
#pragma unroll
                for (int st = 0; st < SE; ++st)
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt) lam[st][mt] = V4{0, 0, 0, 0};
                if (grp == 0)
#pragma unroll
                    for (int st = 0; st < SE; ++st) lam[st][0][0] = 1;
                int sprev = 0;
                // Random words: Philox block b serves sites 4b .. 4b + 3 of the
                // row-major site index.  The GW lane groups of a draw set each
                // hold one of GW consecutive blocks (one Philox pass per 4 GW
                // sites instead of one per 4 sites in every group), and the
                // word of a site comes from the group holding its block.
                constexpr int GW = 4 / SE;   // lane groups per draw set
                uint4 words = make_uint4(0u, 0u, 0u, 0u);
                int wblk = -1;
                // One draw column: w(s) = v hf <Lam, y_s>, the draw, and Lam
                // G_c(s) of the drawn spin; mid() runs after the products and
                // the inner products are issued (the stage fetch).
                auto draw_col = [&](int k, int t, const V4 (&y)[SE][2][NT], auto &&mid) __attribute__((always_inline)) {
                    const int c = cold(t);
                    const int8_t up = prow[c][pd];
                    const int8_t given = crow[c][pd];
                    const int i = r * Lx + c;
                    if (!eval && (i >> 2) / GW != wblk) {   // uniform: every lane's sites move together
                        wblk = (i >> 2) / GW;
                        words = tn_philox(make_uint4((uint32_t)(wblk * GW + grp % GW), (uint32_t)wid, wst, (inst << 2) | 0u),
                                          k0, k1);
                    }
                    const int wsrc = n + 16 * ((grp / GW) * GW + (i >> 2) % GW);   // lane holding block i >> 2
                    const uint32_t word = (uint32_t)__builtin_amdgcn_ds_bpermute(wsrc * 4, (int)tn_word(words, i & 3));
                    const bool up_minus = r > 0 && up < 0;
                    const double2 vv = *(const double2 *)&vS[c][up_minus ? 1 : 0][sprev][0];
                    V4 acc[SE][2][NT];
#pragma unroll
                    for (int st = 0; st < SE; ++st) mul_both<NT, PM>(a[k % CF::ABUF], lam[st], lam[st], acc[st]);
                    ET d0[SE], d1[SE];
#pragma unroll
                    for (int st = 0; st < SE; ++st) {
                        d0[st] = 0;
                        d1[st] = 0;
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                            for (int ii = 0; ii < 4; ++ii) {
                                d0[st] = fma_e(lam[st][mo][ii], y[st][0][mo][ii], d0[st]);
                                d1[st] = fma_e(lam[st][mo][ii], y[st][1][mo][ii], d1[st]);
                            }
                    }
                    mid();
#pragma unroll
                    for (int st = 0; st < SE; ++st) rows4_sum2(d0[st], d1[st]);
                    const ET dd0 = (SE == 2 && ds) ? d0[SE - 1] : d0[0];
                    const ET dd1 = (SE == 2 && ds) ? d1[SE - 1] : d1[0];
                    double w0 = vv.x * (double)dd0;
                    double w1 = vv.y * (double)dd1;
                    if constexpr (F64) {
                        // negative weights (ill-conditioning) clamped to 0 and
                        // counted, as in the plain path
                        n_clamp += (w0 < 0.0) + (w1 < 0.0);
                        w0 = fmax(w0, 0.0);
                        w1 = fmax(w1, 0.0);
                    } else {
                        // a weight below the FP32 resolution of |w+| + |w-| (negative
                        // ones included) is not resolved: it is raised to 2^-24 of
                        // that sum (counted), so that every configuration keeps a
                        // positive proposal probability and a finite ln q
                        const double fl = 0x1p-24 * (fabs(w0) + fabs(w1));
                        n_clamp += (w0 < fl) + (w1 < fl);
                        w0 = fmax(w0, fl);
                        w1 = fmax(w1, fl);
                    }
                    const double tot = w0 + w1;
                    const bool bad = !(tot > 0.0 && tot <= 1.79e308);
                    n_both += bad;
                    // s = +1 iff u < w0 / tot, decided as u tot < w0 (p+ = 1/2 if degenerate)
                    const double u = tn_u01(word);
                    const double ut = bad ? u : u * tot, wt = bad ? 0.5 : w0, sc = bad ? 1.0 : tot;
                    const int sd = eval ? (int)given : ((ut < wt) ? 1 : -1);
                    n_near += !eval && fabs(ut - wt) < 1e-6 * sc;
                    crow[c][pd] = (int8_t)sd;   // the lanes of a proposal write the same value
                    num *= bad ? 0.5 : (sd > 0 ? w0 : w1);
                    den *= sc;
                    sprev = sd > 0 ? 0 : 1;
                    // every set's decisions in every lane
                    int sdset[SE];
                    if constexpr (SE == 2) {
                        const auto sw = __builtin_amdgcn_permlane32_swap((uint32_t)sd, (uint32_t)sd, false, false);
                        sdset[0] = (int)sw[0];
                        sdset[SE - 1] = (int)sw[1];
                    } else {
                        sdset[0] = sd;
                    }
                    if (t % RS == RS - 1) {
                        // power-of-two rescale of the output (from the input's largest
                        // entry) and renormalisation of the ln q products
#pragma unroll
                        for (int st = 0; st < SE; ++st) {
                            ET mx = 0;
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int ii = 0; ii < 4; ++ii) mx = fmax(mx, fabs(lam[st][mo][ii]));
                            const int ee = pow2_exponent_f(rows4_max(mx));
#pragma unroll
                            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                                for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                    for (int ii = 0; ii < 4; ++ii) acc[st][sp][mo][ii] = ldexp(acc[st][sp][mo][ii], -ee);
                        }
                        int e1, e2;
                        num = frexp(num, &e1);
                        den = frexp(den, &e2);
                        nexp += e1 - e2;
                    }
#pragma unroll
                    for (int st = 0; st < SE; ++st)
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo) lam[st][mo] = sdset[st] > 0 ? acc[st][0][mo] : acc[st][1][mo];
                };
                if constexpr (!CF::REC) {
                    auto gload = [&](V4 (&gk)[SE][2][NT], int c) {
#pragma unroll
                        for (int st = 0; st < SE; ++st)
#pragma unroll
                            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                                for (int mo = 0; mo < NT; ++mo) {
                                    if constexpr (F64) {
                                        const uint32_t off = (uint32_t)(((s2 * NT + mo) * 64 + lane) * 32);
                                        const doublex2 lo = __builtin_bit_cast(
                                            doublex2, __builtin_amdgcn_raw_buffer_load_b128(grs[st], off, uniform_u32((uint32_t)c * gstride), 0));
                                        const doublex2 hi = __builtin_bit_cast(
                                            doublex2, __builtin_amdgcn_raw_buffer_load_b128(grs[st], off + 16, uniform_u32((uint32_t)c * gstride), 0));
                                        gk[st][s2][mo] = V4{lo[0], lo[1], hi[0], hi[1]};
                                    } else {
                                        gk[st][s2][mo] = __builtin_bit_cast(
                                            floatx4, __builtin_amdgcn_raw_buffer_load_b128(
                                                         grs[st], (uint32_t)(((s2 * NT + mo) * 64 + lane) * 16),
                                                         uniform_u32((uint32_t)c * gstride), SCR_POLICY));
                                    }
                                }
                    };
                    V4 g[2][SE][2][NT];
                    gload(g[0], cold(0));
                    gload(g[1], cold(min(1, Lx - 1)));
                    // own fetch of column t + 1 has landed (ops issued after it:
                    // the y loads of its step and TL - 2 steps of fetches and y
                    // loads; more in the first steps)
                    constexpr int GL = SE * 2 * NT * (F64 ? 2 : 1);   // y loads per step
                    auto stepS = [&](int k, int t) {
                        draw_col(k, t, g[k], [&] {
                            issue(t + TL - 1);
                            gload(g[k], cold(min(t + 2, Lx - 1)));
                        });
                        ring_next(k, t, std::integral_constant<int, GL + (TL - 2) * (CF::LOADS + GL)>{});
                    };
                    int t = 0;
                    for (; t + 2 <= Lx; t += 2) {
                        stepS(0, t);
                        stepS(1, t + 1);
                    }
                    if (t < Lx) stepS(0, t);
                } else {
                    // Per block b of BR draw columns (the last one ragged at
                    // the far end): the sweep of its columns again from its
                    // checkpoint (the far block from the start vector), the
                    // y tiles kept in registers, then its draw.  Only the
                    // stage fetches are vector-memory operations of a step,
                    // besides the checkpoint loads (counted as none: the
                    // waits then err on the long side).
                    constexpr int BR = CF::BR;
                    constexpr int NW = (TL - 2) * CF::LOADS;
                    const int nblk = (Lx + BR - 1) / BR;
                    V4 cv0[SE][NT], cv1[SE][NT];   // the next block's checkpoint, loaded one block ahead
                    int ce[SE];
                    if (nblk > 1) cp_load(0, cv0[0], cv1[0], ce[0]);
                    for (int b = 0; b < nblk; ++b) {
                        V4 v0[SE][NT], v1[SE][NT];
                        int e[SE];
                        if (b == nblk - 1) {
                            init_state(v0, v1, e);
                        } else {
#pragma unroll
                            for (int mt = 0; mt < NT; ++mt) {
                                v0[0][mt] = cv0[0][mt];
                                v1[0][mt] = cv1[0][mt];
                            }
                            e[0] = ce[0];
                            if (b + 1 < nblk - 1) cp_load(b + 1, cv0[0], cv1[0], ce[0]);
                        }
                        V4 yr[BR][SE][2][NT];
                        const int q0 = 2 * BR * b;
#pragma unroll
                        for (int j = 0; j < BR; ++j) {
                            const int t = Lx - (b + 1) * BR + j;   // sweep step of the block's column j
                            if (t >= 0)
                                sweep_col(j, t, v0, v1, e, [&] { issue(q0 + j + TL - 1); },
                                          [&](int st, int, const V4 (&y)[2][NT]) {
#pragma unroll
                                              for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                                                  for (int mo = 0; mo < NT; ++mo) yr[j][st][sp][mo] = y[sp][mo];
                                          });
                            else
                                issue(q0 + j + TL - 1);
                            ring_next(j, q0 + j, std::integral_constant<int, NW>{});
                        }
#pragma unroll
                        for (int i = 0; i < BR; ++i) {
                            const int t = b * BR + i;   // draw step; its column's y is the block's sweep column BR - 1 - i
                            if (t < Lx) draw_col(BR + i, t, yr[BR - 1 - i], [&] { issue(q0 + BR + i + TL - 1); });
                            else issue(q0 + BR + i + TL - 1);
                            ring_next(BR + i, q0 + BR + i, std::integral_constant<int, NW>{});
                        }
                    }
                }
            }
        }
        __syncthreads();   // the drawn row is complete in LDS
        // energy of row r (Eq. ising: field, bonds in the row, bonds to the row
        // above): four column groups per proposal (c = q mod 4), each summed in
        // column order by one lane, then added in a fixed order, whatever the
        // number of lanes per proposal
        for (int q = cg; q < 4; q += CG) {
            double eg = 0.0;
            for (int c = q; c < Lx; c += 4) {
                const double sc = crow[c][pd];
                const double hv = h ? h[rowb + c] : 0.0;
                const double jl = c > 0 ? Jh[(size_t)r * (Lx - 1) + c - 1] * (double)crow[c - 1][pd] : 0.0;
                const double ja = r > 0 ? Jv[(size_t)(r - 1) * Lx + c] * (double)prow[c][pd] : 0.0;
                eg -= sc * (hv + jl + ja);
            }
            epart[w][ds][q][n] = eg;
        }
        if (!eval) {
            for (int t = threadIdx.x; t < PT * Lx; t += TW * 64) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = unit0 * 16 + nn;
                if (bb < B) S[((size_t)bb * Ly + r) * Lx + c] = crow[c][nn];
            }
        }
        __syncthreads();
        if (cg == 0) E += ((epart[w][ds][0][n] + epart[w][ds][1][n]) + epart[w][ds][2][n]) + epart[w][ds][3][n];
    }
    if (cg == 0 && valid) {
        A.logq[bd] = (log(num) - log(den)) + (double)nexp * 0.69314718055994530942;
        A.energy[bd] = E;
        if (n_clamp) atomicAdd(&A.counters[CNT_CLAMPS], (unsigned long long)n_clamp);
        if (n_both) atomicAdd(&A.counters[CNT_BOTH], (unsigned long long)n_both);
        if (n_near && !eval) atomicAdd(&A.counters[CNT_NEAR], (unsigned long long)n_near);
    }
}

template <int NT, int PM, int V>
__global__ void __launch_bounds__(TW * 64) __attribute__((amdgpu_waves_per_eu(TeamCfg<NT, PM, V>::WPE, 8)))
k_sampler_team(tn_samp_desc A, int eval, uint32_t k0, uint32_t k1, uint64_t step0,
               const uint64_t *__restrict__ step_base) {
    team_body<NT, PM, V>(A, blockIdx.x * TW * TeamCfg<NT, PM, V>::SETS, eval, k0, k1, step0 + *step_base);
}

template <int NT, int PM, int V>
__global__ void __launch_bounds__(TW * 64) __attribute__((amdgpu_waves_per_eu(TeamCfg<NT, PM, V>::WPE, 8)))
k_sampler_team_multi(const tn_samp_desc *__restrict__ descs, int n, int eval, uint32_t k0, uint32_t k1,
                     uint64_t step0, const uint64_t *__restrict__ step_base) {
    const int u0 = (int)blockIdx.x * TW * TeamCfg<NT, PM, V>::SETS;
    int lo = 0, hi = n - 1;
    while (lo < hi) {   // last instance whose first unit is <= u0
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].blk0 <= u0) lo = mid;
        else hi = mid - 1;
    }
    const tn_samp_desc A = descs[lo];
    team_body<NT, PM, V>(A, u0 - A.blk0, eval, k0, k1, step0 + *step_base);
}

template <int NT, int PM, int V>
int launch_mfma(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    using CF = TeamCfg<NT, PM, V>;
    const TeamSmem T(ctx->Lx, CF::STAGE, CF::TL, CF::PT);
    auto kern = k_sampler_team<NT, PM, V>;
    if (T.total > 65536)
        TN_HIP(ctx, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        T.total));
    const tn_samp_desc A = tn_samp_desc_of(ctx, B, S, logq, energy, g, per_step, first_id);
    hipLaunchKernelGGL(kern, dim3((B + CF::PT - 1) / CF::PT), dim3(TW * 64), T.total, ctx->stream, A,
                       eval ? 1 : 0, (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

// blocks counts 16-proposal units, a whole number of teams per instance
template <int NT, int PM, int V>
int launch_mfma_multi(tn_ctx *ctx, const tn_samp_desc *descs, int n, int blocks, int maxLx,
                      uint64_t seed, uint64_t step0, int eval) {
    using CF = TeamCfg<NT, PM, V>;
    static_assert(8 % (TW * CF::SETS) == 0, "an instance's eight-unit blocks must split into teams");
    const TeamSmem T(maxLx, CF::STAGE, CF::TL, CF::PT);
    auto kern = k_sampler_team_multi<NT, PM, V>;
    if (T.total > 65536)
        TN_HIP(ctx, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        T.total));
    hipLaunchKernelGGL(kern, dim3((blocks + TW * CF::SETS - 1) / (TW * CF::SETS)), dim3(TW * 64), T.total,
                       ctx->stream, descs, n, eval,
                       (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

// D <= 32 classes: variants 0-3; BF16 D 33-64: variants 0 and 1; FP32 D 33-64
// and FP64 (D <= 32): variant 0 only
template <int NT, int PM>
int launch_variant(tn_ctx *ctx, int V, int B, int8_t *S, bool eval, double *logq, double *energy,
                   float *g, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    if constexpr (NT <= 2 && PM != PM_F64) {
        if (V == 1) return launch_mfma<NT, PM, 1>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
        if (V == 2) return launch_mfma<NT, PM, 2>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
        if (V == 3) return launch_mfma<NT, PM, 3>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    } else if constexpr (PM == PM_BF16) {
        if (V == 1) return launch_mfma<NT, PM, 1>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    }
    return launch_mfma<NT, PM, 0>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
}

template <int NT, int PM>
int launch_variant_multi(tn_ctx *ctx, int V, const tn_samp_desc *descs, int n, int blocks, int maxLx,
                         uint64_t seed, uint64_t step0, int eval) {
    if constexpr (NT <= 2) {
        if (V == 1) return launch_mfma_multi<NT, PM, 1>(ctx, descs, n, blocks, maxLx, seed, step0, eval);
        if (V == 2) return launch_mfma_multi<NT, PM, 2>(ctx, descs, n, blocks, maxLx, seed, step0, eval);
        if (V == 3) return launch_mfma_multi<NT, PM, 3>(ctx, descs, n, blocks, maxLx, seed, step0, eval);
    } else if constexpr (PM == PM_BF16) {
        if (V == 1) return launch_mfma_multi<NT, PM, 1>(ctx, descs, n, blocks, maxLx, seed, step0, eval);
    }
    return launch_mfma_multi<NT, PM, 0>(ctx, descs, n, blocks, maxLx, seed, step0, eval);
}

template <int PM>
int dispatch_nt(tn_ctx *ctx, int V, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    switch (ctx->Dp / 16) {
    case 1: return launch_variant<1, PM>(ctx, V, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 2: return launch_variant<2, PM>(ctx, V, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 3:
        if constexpr (PM != PM_F64)
            return launch_variant<3, PM>(ctx, V, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
        break;
    case 4:
        if constexpr (PM != PM_F64)
            return launch_variant<4, PM>(ctx, V, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
        break;
    default: break;
    }
    return tn_fail(ctx, TN_EINVAL, PM == PM_F64 ? "the batched fp64 sampler supports D <= 32"
                                                : "bond dimension above 64");
}

}  // namespace

int tn_run_mfma(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                uint64_t first_id, int8_t *spins, bool eval, double *logq, double *energy, int variant,
                void *scr) {
    if (batch == 0) return TN_OK;
    if (ctx->Lx > TN_MAX_LX) return tn_fail(ctx, TN_EINVAL, "Lx above 256");
    if (per_step <= 0) return tn_fail(ctx, TN_EINVAL, "proposals per step must be positive");
    if (variant < 0) variant = tn_ctx_variant(ctx);
    const int pm = ctx->prec == TN_BF16 ? PM_BF16 : (ctx->prec == TN_FP64_MFMA ? PM_F64 : PM_F32);
    if (variant >= team_variants(ctx->Dp / 16, pm)) return tn_fail(ctx, TN_EINVAL, "no such sampler variant");
    int rc;
    if (!scr) {
        if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, tn_mfma_scratch_bytes(ctx, batch)))) return rc;
        scr = ctx->gscr;
    }
    float *g = (float *)scr;
    if (pm == PM_BF16)
        return dispatch_nt<PM_BF16>(ctx, variant, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    if (pm == PM_F64)
        return dispatch_nt<PM_F64>(ctx, variant, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    return dispatch_nt<PM_F32>(ctx, variant, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
}

int tn_run_mfma_multi(tn_ctx *ctx, int NT, bool bf16, int variant, const tn_samp_desc *descs, int n,
                      int blocks, int maxLx, uint64_t seed, uint64_t step0, bool eval) {
    if (blocks == 0) return TN_OK;
    if (maxLx > TN_MAX_LX) return tn_fail(ctx, TN_EINVAL, "Lx above 256");
    if (NT < 1 || NT > 4) return tn_fail(ctx, TN_EINVAL, "bond dimension above 64");
    if (variant < 0 || variant >= tn_team_variants(NT, bf16)) return tn_fail(ctx, TN_EINVAL, "no such sampler variant");
    switch (NT * 2 + (bf16 ? 1 : 0)) {
    case 2: return launch_variant_multi<1, PM_F32>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 3: return launch_variant_multi<1, PM_BF16>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 4: return launch_variant_multi<2, PM_F32>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 5: return launch_variant_multi<2, PM_BF16>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 6: return launch_variant_multi<3, PM_F32>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 7: return launch_variant_multi<3, PM_BF16>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    case 8: return launch_variant_multi<4, PM_F32>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    default: return launch_variant_multi<4, PM_BF16>(ctx, variant, descs, n, blocks, maxLx, seed, step0, eval ? 1 : 0);
    }
}
