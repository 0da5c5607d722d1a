// Batched sampler on the matrix cores: the same sequential draw and the same
// conditionals as the plain path (Sec. 2 Eqs. bayes, pi-approx; App. A
// Eq. proba-ratio-apx), with the per-column products run as 16x16 MFMA tiles.
//
// A workgroup owns 16 proposals (the N dimension of every tile) for the whole
// lattice; each of its two groups of 2*NT waves (Dp = 16*NT padded bond) owns
// one output tile (spin s, 16-row block mo) of every column product per wave,
// so the 16 proposals' work is spread over all four SIMDs.  Per column:
//   environment sweep  y_s[mo] = G_c(s)[mo,:] r_s  (NQ chained MFMAs, K = Dp),
//                tiles exchanged through LDS (double buffered, one barrier),
//                r_s' = sum_s W(s',s) v_c(s) y_s, every wave rebuilding its own
//                next B operand r_{s_w}; the y_s tiles go to this workgroup's
//                scratch for the drawing of the row
//   drawing      w(s) = v hf <Lam, y_s>, p+ and the draw in fp64 on every wave
//                (bitwise identical), Lam_s'[mo] = G_c(s)^T[mo,:] Lam for both
//                spins while the draw is taken, exchanged and selected by the
//                drawn spin.
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
// the end; the spin is +1 iff u * (w+ + w-) < w+.
#include "common.hpp"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

#define TN_MAX_LX 256

__device__ __forceinline__ int pow2_exponent_f(float m) {
    int e = 0;
    if (m > 0.0f && m <= 3.0e38f) frexpf(m, &e);
    return e;
}

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx2 __attribute__((ext_vector_type(2)));

// Four floats to bf16 with round-to-nearest-even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ shortx4 bf16x4_rne(const floatx4 v) {
    const floatx2 lo = {v[0], v[1]}, hi = {v[2], v[3]};
    const bf16x2 a = __builtin_convertvector(lo, bf16x2), b = __builtin_convertvector(hi, bf16x2);
    return __builtin_bit_cast(shortx4, uintx2{__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)});
}

// Buffer resource over [base, base + bytes): loads and stores take a 32-bit
// per-lane offset and a wave-uniform column offset; accesses outside the
// range read 0 / are dropped.
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

// A operands of one spin's product for one column: every 16-row output block
// mo = 0..NT-1, each the 4 NT k-chunks of the fp32 16x16x4 product or the NT
// chunks of the bf16 16x16x16 product.  The NT accumulation chains are
// independent and interleaved.  Tile layout per site: [s][mo][chunk][64 lanes].
template <int NT, bool BF16>
struct ATiles;

template <int NT>
struct ATiles<NT, false> {
    static constexpr int NQ = 4 * NT;
    static constexpr size_t SITE_BYTES = (size_t)2 * NT * NQ * 64 * 4;
    static constexpr uint32_t LANE_BYTES = 16;   // a lane's 4 consecutive k-chunks
    float a[NT][NQ];
    // vbase: byte offset of (spin s_w, lane) within a site; soff: site offset.
    // Tile layout per spin: [mo][mt][64 lanes][4 chunks], one 16-byte load
    // per lane for the chunks q = 4 mt .. 4 mt + 3.
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t vbase, uint32_t soff) {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) {
                const floatx4 v = __builtin_bit_cast(
                    floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, vbase + (mo * NT + mt) * 1024, soff, 0));
#pragma unroll
                for (int i = 0; i < 4; ++i) a[mo][4 * mt + i] = v[i];
            }
    }
    __device__ __forceinline__ void mul(const floatx4 (&x)[NT], floatx4 (&acc)[NT]) const {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo) acc[mo] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo)
                acc[mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mo][q], x[q >> 2][q & 3], acc[mo], 0, 0, 0);
    }
};

template <int NT>
struct ATiles<NT, true> {
    static constexpr size_t SITE_BYTES = (size_t)2 * NT * NT * 64 * 8;
    static constexpr uint32_t LANE_BYTES = 8;
    shortx4 a[NT][NT];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t vbase, uint32_t soff) {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
                a[mo][mt] = __builtin_bit_cast(
                    shortx4, __builtin_amdgcn_raw_buffer_load_b64(r, vbase + (mo * NT + mt) * 512, soff, 0));
    }
    __device__ __forceinline__ void mul(const floatx4 (&x)[NT], floatx4 (&acc)[NT]) const {
#pragma unroll
        for (int mo = 0; mo < NT; ++mo) acc[mo] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            const shortx4 bv = bf16x4_rne(x[mt]);
#pragma unroll
            for (int mo = 0; mo < NT; ++mo)
                acc[mo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mo][mt], bv, acc[mo], 0, 0, 0);
        }
    }
};

// Columns of the environment tiles (and, for the drawing group, of the stored
// y_s tiles) are kept in a ring of PF register sets: the set used at column
// step t is refilled with step t + PF.  The step loop is unrolled by PF so that
// the ring is indexed statically and no register copy waits for a load.
template <int NT, bool BF16>
constexpr int prefetch_depth() { return NT <= 2 ? 3 : 2; }

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

// LDS layout of one workgroup (bytes, every part 16-byte aligned), sized by Lx.
template <int NT>
struct SmemLayout {
    int xch, pmx, rows, uni, mixP, vS, eT, epart, lqx, ex, total;
    __host__ __device__ SmemLayout(int Lx) {
        xch = 0;                                    // floatx4 [2 group][2 buf][2 s][NT][64]
        pmx = xch + 2 * 2 * 2 * NT * 64 * 16;       // float [2 group][2 buf][2 s][64]
        rows = pmx + 2 * 2 * 2 * 64 * 4;            // int8 [2 parity][Lx][16]
        uni = rows + 2 * Lx * 16;                   // uint32 [Lx][16]
        mixP = uni + Lx * 16 * 4;                   // float [Lx][s_w][s_up][s]
        vS = mixP + Lx * 8 * 4;                     // double [Lx][s_up][s_prev][s]
        eT = vS + Lx * 8 * 8;                       // double [Lx][4]: h, Jh to the left, Jv above
        epart = eT + Lx * 4 * 8;                    // double [16 column groups][16]
        lqx = epart + 16 * 16 * 8;                  // double [2 group][16] ln q parts
        ex = lqx + 2 * 16 * 8;                      // double [16] energies
        total = ex + 16 * 8;
    }
};

// Snake order: row r is drawn left to right when r is even, right to left
// when odd.  Before a row is drawn, the environments of its free columns are
// swept from its far end; that sweep runs in the same column order as the
// drawing of the row above, so the two run side by side: phase p pairs the
// environment sweep of row p (group p & 1) with the drawing of row p-1 (the
// other group), one column per step and one barrier per step, and the drawn
// spin of a column is in LDS before the environment sweep of the row below
// needs it.  A rightward phase multiplies by G^T (GL tiles), a leftward one by
// G (GR tiles), for both groups.
//
// Each group has two waves, one per spin s_w (four waves, one per SIMD); a
// wave computes all NT output blocks of its spin's product, so per column a
// wave exchanges only the other spin's tiles.  On gfx950 the fp32 MFMA and
// the vector ALU share a SIMD's issue, so the per-column scalar work is kept
// small: table entries are read at computed LDS addresses instead of being
// selected in registers, vectors are rescaled every RS-th column only, and
// the row energy is summed once per row.
//
// Proposal j of the launch has id first_id + j % per_step and MH step
// step0 + j / per_step (several steps' proposals may share a launch; the
// proposal distribution does not depend on the chains' state).
//
// LDS arrays indexed by proposal keep the proposal index innermost, so the 16
// proposals of a wavefront touch 16 consecutive entries (no bank conflicts).
constexpr int RS = 4;   // rescale (and ln q renormalisation) period in columns

template <int NT, bool BF16>
__device__ __forceinline__ void sampler_body(const tn_samp_desc &A, const int blk, const int eval,
                                             const uint32_t k0, const uint32_t k1,
                                             const uint64_t step0) {
    const int B = A.B, Lx = A.Lx, Ly = A.Ly, per_step = A.per_step;
    const double *__restrict__ Jh = A.Jh;
    const double *__restrict__ Jv = A.Jv;
    const double *__restrict__ h = A.h;
    const double *__restrict__ fac = A.fac;
    const void *__restrict__ GRv = A.GR;
    const void *__restrict__ GLv = A.GL;
    int8_t *__restrict__ S = A.S;
    double *__restrict__ logq = A.logq;
    double *__restrict__ energy = A.energy;
    float *__restrict__ gscr = A.gscr;
    const uint64_t first_id = A.first_id;
    const uint32_t inst = A.inst;
    unsigned long long *__restrict__ counters = A.counters;
    constexpr int PF = prefetch_depth<NT, BF16>();
    using AT = ATiles<NT, BF16>;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int gp = w >> 1, sw = w & 1;
    const int n = lane & 15, grp = lane >> 4;
    const int b = blk * 16 + n;
    const bool valid = b < B;
    const bool leader = (sw == 0 && grp == 0);        // one lane per proposal per group

    extern __shared__ __align__(16) unsigned char smem[];
    const SmemLayout<NT> L(Lx);
    floatx4(*xch)[2][2][NT][64] = (floatx4(*)[2][2][NT][64])(smem + L.xch);
    float(*pmx)[2][2][64] = (float(*)[2][2][64])(smem + L.pmx);
    uint32_t(*uni)[16] = (uint32_t(*)[16])(smem + L.uni);
    float(*mixP)[2][2][2] = (float(*)[2][2][2])(smem + L.mixP);
    double(*vS)[2][2][2] = (double(*)[2][2][2])(smem + L.vS);
    double(*eT)[4] = (double(*)[4])(smem + L.eT);
    double(*epart)[16] = (double(*)[16])(smem + L.epart);
    double(*lqx)[16] = (double(*)[16])(smem + L.lqx);
    double *ex = (double *)(smem + L.ex);
    // spins of the rows by parity: [parity][Lx][16]
    auto rowbuf = [&](int par) { return (int8_t(*)[16])(smem + L.rows + par * Lx * 16); };

    const uint32_t gstride = 2u * NT * 64 * 16;       // bytes of stored y tiles per column
    float *gwg = gscr + ((size_t)blk * 2 + gp) * Lx * (gstride / 4);
    const __amdgpu_buffer_rsrc_t grs = make_rsrc(gwg, (uint32_t)Lx * gstride);
    const int NTH = blockDim.x;

    // ln q = ln(num / den): products of the drawn weights and of the weight
    // totals, each kept as an fp64 mantissa with a separate binary exponent
    double num = 1.0, den = 1.0, E = 0.0;
    int nexp = 0;
    uint32_t n_clamp = 0, n_both = 0, n_near = 0;
    int buf = 0;

    for (int p = 0; p <= Ly; ++p) {
        const bool hasP = p < Ly, hasS = p >= 1;
        const bool isP = hasP && gp == (p & 1);
        const bool isS = hasS && gp != (p & 1);
        const bool rightward = (p & 1) != 0;          // column order of this phase
        const int rS = p - 1;                          // row drawn in this phase
        // ---- phase set-up: factor tables, random words, given spins
        for (int t = threadIdx.x; t < Lx * 8; t += NTH) {
            const int c = t >> 3, su = (t >> 2) & 1, x = (t >> 1) & 1, s = t & 1;
            if (hasP) {   // environment sweep of row p: W(s_w = x, s) v_c(s; s_up)
                const double *f = fac + ((size_t)p * Lx + c) * 6;
                const int cb = rightward ? c + 1 : c;   // bond towards the next column
                double Wv = 1.0;
                if (cb >= 1 && cb <= Lx - 1) Wv = fac[((size_t)p * Lx + cb) * 6 + ((x == s) ? 4 : 5)];
                const double v = f[s] * f[2 + (su ^ s)];
                mixP[c][x][su][s] = (float)(Wv * v);
            }
            if (hasS) {   // drawing of row p-1: v_c(s; s_up) hf(s; s_prev)
                const double *f = fac + ((size_t)rS * Lx + c) * 6;
                const int cb = rightward ? c : c + 1;   // bond to the previous column
                double hf = 1.0;
                if (cb >= 1 && cb <= Lx - 1) hf = fac[((size_t)rS * Lx + cb) * 6 + ((x == s) ? 4 : 5)];
                vS[c][su][x][s] = f[s] * f[2 + (su ^ s)] * hf;
            }
        }
        if (hasS) {   // couplings of the drawn row for its energy (Eq. ising)
            for (int c = threadIdx.x; c < Lx; c += NTH) {
                eT[c][0] = h ? h[(size_t)rS * Lx + c] : 0.0;
                eT[c][1] = c > 0 ? Jh[(size_t)rS * (Lx - 1) + c - 1] : 0.0;
                eT[c][2] = rS > 0 ? Jv[(size_t)(rS - 1) * Lx + c] : 0.0;
                eT[c][3] = 0.0;
            }
        }
        if (hasS && !eval) {   // random words of row p-1
            for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                const int c = t >> 4, nn = t & 15;
                const int i = rS * Lx + c;
                const uint32_t j = blk * 16 + nn;
                const uint64_t id = first_id + j % (uint32_t)per_step;
                const uint32_t st = (uint32_t)(step0 + j / (uint32_t)per_step);
                const uint4 x = tn_philox(make_uint4((uint32_t)(i >> 2), (uint32_t)id, st,
                                                     (inst << 2) | 0u), k0, k1);
                uni[c][nn] = tn_word(x, i & 3);
            }
        }
        if (hasS && eval) {   // the given spins of row p-1
            int8_t(*r1)[16] = rowbuf(rS & 1);
            for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = blk * 16 + nn;
                r1[c][nn] = bb < B ? S[((size_t)bb * Ly + rS) * Lx + c] : (int8_t)1;
            }
        }
        __syncthreads();

        const size_t rowP = (size_t)p * Lx, rowSb = (size_t)rS * Lx;
        const void *Gph = rightward ? GLv : GRv;
        const size_t rbase = isP ? rowP : rowSb;
        // environment tiles of this phase's row; per-lane offset of spin s_w's tiles
        const __amdgpu_buffer_rsrc_t ars =
            make_rsrc((const char *)Gph + rbase * AT::SITE_BYTES, (uint32_t)(Lx * AT::SITE_BYTES));
        const uint32_t avb = (uint32_t)(sw * (AT::SITE_BYTES / 2) + lane * AT::LANE_BYTES);
        floatx4 vec[NT];   // r_{s_w} (environment sweep) or Lam (drawing)
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) vec[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        if (grp == 0) vec[0][0] = 1.0f;
        auto colof = [&](int t) { return rightward ? t : Lx - 1 - t; };
        auto gload = [&](floatx4 (&gk)[2][NT], int c) {
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                for (int mo = 0; mo < NT; ++mo)
                    gk[s2][mo] = __builtin_bit_cast(
                        floatx4, __builtin_amdgcn_raw_buffer_load_b128(
                                     grs, (uint32_t)(((s2 * NT + mo) * 64 + lane) * 16), (uint32_t)c * gstride, 0));
        };
        AT a[PF];
        floatx4 g[PF][2][NT];   // stored y_s tiles of the drawn row (drawing group)
        const int8_t(*prowP)[16] = rowbuf((p + 1) & 1);   // row p-1 (above row p)
        const int8_t(*prowS)[16] = rowbuf(p & 1);         // row p-2 (above row p-1)
        int8_t(*crowS)[16] = rowbuf((p + 1) & 1);         // row p-1, written by the drawing

        // One loop per role over whole turns of the ring, then the remaining
        // steps.  The loads are unconditional (the last columns re-read the final
        // one) and fenced from the scheduler, each role issues its first ring
        // entries in ring order, and the two roles share no code path before
        // their loops: the compiler can then count the loads in flight and waits
        // only for the ring entry it uses.
        if (isS) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int ck = colof(min(k, Lx - 1));
                gload(g[k], ck);
                a[k].load(ars, avb, (uint32_t)(ck * AT::SITE_BYTES));
                __builtin_amdgcn_sched_barrier(0);
            }
            int sprev = 0;   // index of the previous spin (0: +1, 1: -1); unused at t = 0
            auto stepS = [&](int k, int t) {
                const int c = colof(t);
                const int cn = colof(min(t + PF, Lx - 1));
                // spin above, random word, given spin; the factor pair
                // v_c(s) hf(s) for (s_up, s_prev) read at its address
                const int8_t up = prowS[c][n];
                const uint32_t word = uni[c][n];
                const int8_t given = crowS[c][n];
                const bool up_minus = rS > 0 && up < 0;
                const double2 vv = *(const double2 *)&vS[c][up_minus ? 1 : 0][sprev][0];
                // Lam G_c(s_w) does not depend on the draw
                floatx4 acc[NT];
                a[k].mul(vec, acc);
                float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
                for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d0 = fmaf(vec[mo][i], g[k][0][mo][i], d0);
                        d1 = fmaf(vec[mo][i], g[k][1][mo][i], d1);
                    }
                gload(g[k], cn);
                a[k].load(ars, avb, (uint32_t)(cn * AT::SITE_BYTES));
                __builtin_amdgcn_sched_barrier(0);
                rows4_sum2(d0, d1);
                double w0 = vv.x * (double)d0;
                double w1 = vv.y * (double)d1;
                n_clamp += (w0 < 0.0) + (w1 < 0.0);
                w0 = fmax(w0, 0.0);
                w1 = fmax(w1, 0.0);
                const double tot = w0 + w1;
                const bool bad = !(tot > 0.0 && tot <= 1.79e308);
                n_both += bad;
                // s = +1 iff u < w0 / tot, decided as u tot < w0 (p+ = 1/2 if degenerate)
                const double u = tn_u01(word);
                const double ut = bad ? u : u * tot, wt = bad ? 0.5 : w0, sc = bad ? 1.0 : tot;
                const int s = eval ? (int)given : ((ut < wt) ? 1 : -1);
                n_near += !eval && fabs(ut - wt) < 1e-6 * sc;
                crowS[c][n] = (int8_t)s;   // every drawing lane writes the same value
                num *= bad ? 0.5 : (s > 0 ? w0 : w1);
                den *= sc;
                sprev = s > 0 ? 0 : 1;
                if (t % RS == RS - 1) {
                    // power-of-two rescale of the output (from the input's largest entry)
                    // and renormalisation of the ln q products
                    float mx = 0.0f;
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(vec[mo][i]));
                    const int e = pow2_exponent_f(rows4_max(mx));
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[mo][i] = ldexpf(acc[mo][i], -e);
                    int e1, e2;
                    num = frexp(num, &e1);
                    den = frexp(den, &e2);
                    nexp += e1 - e2;
                }
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) xch[gp][buf][sw][mo][lane] = acc[mo];
                __syncthreads();
                const int sd = s > 0 ? 0 : 1;
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) vec[mo] = xch[gp][buf][sd][mo][lane];
                buf ^= 1;
            };
            int t0 = 0;
            for (; t0 + PF <= Lx; t0 += PF) {
#pragma unroll
                for (int k = 0; k < PF; ++k) stepS(k, t0 + k);
            }
#pragma unroll
            for (int k = 0; k < PF - 1; ++k)
                if (t0 + k < Lx) stepS(k, t0 + k);
        } else if (isP) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                a[k].load(ars, avb, (uint32_t)(colof(min(k, Lx - 1)) * AT::SITE_BYTES));
                __builtin_amdgcn_sched_barrier(0);
            }
            int e = 0;   // pending power-of-two scale of the next product's output
            auto stepP = [&](int k, int t) {
                const int c = colof(t);
                floatx4 acc[NT];
                a[k].mul(vec, acc);
                const floatx4 mt = *(const floatx4 *)&mixP[c][sw][0][0];   // [s_up][s]
                const bool resc = t % RS == 0 && t > 0;                      // apply e
                const bool meas = t % RS == RS - 1;                          // measure e
                if (resc) {
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[mo][i] = ldexpf(acc[mo][i], -e);
                }
#pragma unroll
                for (int mo = 0; mo < NT; ++mo)
                    __builtin_amdgcn_raw_buffer_store_b128(
                        __builtin_bit_cast(uintx4, acc[mo]), grs,
                        (uint32_t)(((sw * NT + mo) * 64 + lane) * 16), (uint32_t)c * gstride, 0);
                a[k].load(ars, avb, (uint32_t)(colof(min(t + PF, Lx - 1)) * AT::SITE_BYTES));
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) xch[gp][buf][sw][mo][lane] = acc[mo];
                float mx = 0.0f;
                if (meas) {
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(acc[mo][i]));
                    pmx[gp][buf][sw][lane] = mx;
                }
                __syncthreads();
                // r_{s_w} for the next column: W(s_w, s) v_c(s) mixing of both y_s
                const bool up_minus = p > 0 && prowP[c][n] < 0;
                const float m0 = up_minus ? mt[2] : mt[0], m1 = up_minus ? mt[3] : mt[1];
                const float mown = sw == 0 ? m0 : m1, moth = sw == 0 ? m1 : m0;
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) {
                    const floatx4 yo = xch[gp][buf][1 - sw][mo][lane];
#pragma unroll
                    for (int i = 0; i < 4; ++i) vec[mo][i] = mown * acc[mo][i] + moth * yo[i];
                }
                if (meas) e = pow2_exponent_f(rows4_max(fmaxf(mx, pmx[gp][buf][1 - sw][lane])));
                buf ^= 1;
            };
            int t0 = 0;
            for (; t0 + PF <= Lx; t0 += PF) {
#pragma unroll
                for (int k = 0; k < PF; ++k) stepP(k, t0 + k);
            }
#pragma unroll
            for (int k = 0; k < PF - 1; ++k)
                if (t0 + k < Lx) stepP(k, t0 + k);
        } else {   // idle group (first and last phase): keep the barrier count
            for (int t = 0; t < Lx; ++t) {
                __syncthreads();
                buf ^= 1;
            }
        }
        __syncthreads();   // the drawn row is complete in LDS

        if (hasS) {
            // energy of row p-1 (Eq. ising: field, bonds in the row, bonds to the row
            // above): 16 column groups per proposal, summed in a fixed order
            const int8_t(*cur)[16] = rowbuf((p + 1) & 1);
            const int8_t(*abv)[16] = rowbuf(p & 1);
            {
                const int nn = threadIdx.x & 15, cg = threadIdx.x >> 4;
                double e = 0.0;
                for (int c = cg; c < Lx; c += 16) {
                    const double sc = cur[c][nn];
                    const double sl = c > 0 ? (double)cur[c - 1][nn] : 0.0;
                    const double sa = rS > 0 ? (double)abv[c][nn] : 0.0;
                    e -= sc * (eT[c][0] + eT[c][1] * sl + eT[c][2] * sa);
                }
                epart[cg][nn] = e;
            }
            if (!eval) {
                for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                    const int nn = t / Lx, c = t % Lx;
                    const int bb = blk * 16 + nn;
                    if (bb < B) S[((size_t)bb * Ly + rS) * Lx + c] = cur[c][nn];
                }
            }
            __syncthreads();
            if (threadIdx.x < 16) {
                double e = 0.0;
                for (int cg = 0; cg < 16; ++cg) e += epart[cg][threadIdx.x];
                E += e;   // held by threads 0..15 (proposal threadIdx.x)
            }
        }
    }
    // combine the two groups' ln q parts; flush the counters
    if (leader) {
        lqx[gp][n] = (log(num) - log(den)) + (double)nexp * 0.69314718055994530942;
        if (valid) {
            if (n_clamp) atomicAdd(&counters[CNT_CLAMPS], (unsigned long long)n_clamp);
            if (n_both) atomicAdd(&counters[CNT_BOTH], (unsigned long long)n_both);
            if (n_near && !eval) atomicAdd(&counters[CNT_NEAR], (unsigned long long)n_near);
        }
    }
    if (threadIdx.x < 16) ex[threadIdx.x] = E;
    __syncthreads();
    if (gp == 0 && leader && valid) {
        logq[b] = lqx[0][n] + lqx[1][n];
        energy[b] = ex[n];
    }
}

// ---------------------------------------------------------------------------
// Used where both spins' operands and vectors fit one wave's registers: FP32
// with D <= 32 (two waves per SIMD) and BF16 with D <= 64 (one wave per SIMD
// from D = 33).
template <int NT, bool BF16>
constexpr bool team_kernel_fits() { return BF16 ? NT <= 4 : NT <= 2; }

// Products of both spins' tiles, the four (2 NT) accumulation chains
// interleaved: acc[s] = A[s] x[s].
template <int NT, bool BF16>
__device__ __forceinline__ void mul_both(const ATiles<NT, BF16> (&a)[2], const floatx4 (&x0)[NT],
                                         const floatx4 (&x1)[NT], floatx4 (&acc)[2][NT]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int mo = 0; mo < NT; ++mo) acc[sp][mo] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (BF16) {
        shortx4 b0[NT], b1[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            b0[mt] = bf16x4_rne(x0[mt]);
            b1[mt] = bf16x4_rne(x1[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                acc[0][mo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0].a[mo][mt], b0[mt], acc[0][mo], 0, 0, 0);
                acc[1][mo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1].a[mo][mt], b1[mt], acc[1][mo], 0, 0, 0);
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
// Teams of TW wavefronts, 16 proposals each, sharing the environment tiles.
//
// Each wave keeps both spins' operands and vectors in registers and runs the
// environment sweep of a row and then its drawing, row after row, for its own
// 16 proposals: per column the sweep chains 2 NT independent MFMA
// accumulations (both spins), stores y_s and mixes r_s' = sum_s W(s', s)
// v_c(s) y_s in place; the drawing multiplies Lam by both G_c(s)^T, forms
// w(s) = v hf <Lam, y_s> from the stored tiles, draws, and keeps the drawn
// spin's product lane by lane.  No tile crosses a wave.
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

// Per bond class: TL LDS stages (columns in flight); UNI: the row's random
// words precomputed in LDS (else drawn by each wave as it goes); WPE: waves per
// SIMD the registers allow.
template <int NT, bool BF16>
struct TeamCfg {
    static constexpr uint32_t STAGE = (uint32_t)ATiles<NT, BF16>::SITE_BYTES;   // both spins
    static constexpr uint32_t LANE = STAGE % (TW * 64 * 16) == 0 ? 16 : 4;     // dwordx4 or dword fetches
    static constexpr int LOADS = (int)(STAGE / (TW * 64 * LANE));            // per wave per column
    static_assert(LOADS * TW * 64 * LANE == STAGE, "stage must split evenly");
    static constexpr int TL = NT <= 2 ? 4 : 2;
    static constexpr bool UNI = NT <= 2;
    static constexpr int WPE = NT <= 2 ? 2 : 1;
    static constexpr int ABUF = 2;   // operand register sets (read one column ahead)
};

struct TeamSmem {
    int ring, rows, uni, mixP, vS, epart, total;
    __host__ __device__ TeamSmem(int Lx, uint32_t stage, int tl, bool with_uni) {
        ring = 0;                                        // [TL][stage bytes]
        rows = ring + tl * (int)stage;                   // int8 [2 parity][Lx][TW*16]
        uni = rows + ((2 * Lx * TW * 16 + 15) & ~15);    // uint32 [Lx][TW*16] (if with_uni)
        mixP = uni + (with_uni ? Lx * TW * 16 * 4 : 0);  // float [Lx][s_up][s'][s]
        vS = mixP + Lx * 8 * 4;                          // double [Lx][s_up][s_prev][s]
        epart = vS + Lx * 8 * 8;                         // double [TW][4][16]
        total = epart + TW * 4 * 16 * 8;
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

template <int NT, bool BF16>
__device__ __forceinline__ void lds_tiles(ATiles<NT, BF16> &a, const unsigned char *st, int lane) {
    if constexpr (BF16) {
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

template <int NT, bool BF16>
__device__ __forceinline__ void team_body(const tn_samp_desc &A, const int unit0, const int eval,
                                          const uint32_t k0, const uint32_t k1, const uint64_t step0) {
    using AT = ATiles<NT, BF16>;
    using CF = TeamCfg<NT, BF16>;
    constexpr int TL = CF::TL;
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
    const int pn = w * 16 + n;                 // proposal slot in the team
    const int blk = unit0 + w;                 // this wave's 16-proposal unit
    const int b = blk * 16 + n;
    const bool valid = b < B;
    constexpr int PT = TW * 16;                // proposals per team

    extern __shared__ __align__(16) unsigned char smem[];
    const TeamSmem L(Lx, CF::STAGE, TL, CF::UNI);
    unsigned char *ring = smem + L.ring;
    uint32_t(*uni)[PT] = (uint32_t(*)[PT])(smem + L.uni);
    float(*mixP)[2][2][2] = (float(*)[2][2][2])(smem + L.mixP);
    double(*vS)[2][2][2] = (double(*)[2][2][2])(smem + L.vS);
    double(*epart)[4][16] = (double(*)[4][16])(smem + L.epart);
    auto rowbuf = [&](int par) { return (int8_t(*)[PT])(smem + L.rows + par * Lx * PT); };

    const uint32_t gstride = 2u * NT * 64 * 16;   // bytes of stored y tiles per column
    const char *gwg = uniform_ptr(A.gscr + (size_t)blk * Lx * (gstride / 4));
    const __amdgpu_buffer_rsrc_t grs = make_rsrc(gwg, uniform_u32((uint32_t)Lx * gstride));
    // this wave's share of a stage: LOADS chunks of 64 lanes x LANE bytes
    const uint32_t share = (uint32_t)w * CF::LOADS * 64 * CF::LANE;

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
            double hf = 1.0;
            if (cw >= 1 && cw <= Lx - 1) hf = fac[((size_t)r * Lx + cw) * 6 + ((x == sg) ? 4 : 5)];
            vS[c][su][x][sg] = v * hf;
        }
        int8_t(*crow)[PT] = rowbuf(r & 1);
        const int8_t(*prow)[PT] = rowbuf((r + 1) & 1);
        if (!eval && CF::UNI) {
            for (int t = threadIdx.x; t < PT * Lx; t += TW * 64) {
                const int c = t / PT, nn = t % PT;
                const int i = r * Lx + c;
                const uint32_t j = (uint32_t)unit0 * 16 + nn;
                const uint64_t id = A.first_id + j % (uint32_t)per_step;
                const uint32_t st = (uint32_t)(step0 + j / (uint32_t)per_step);
                const uint4 x = tn_philox(make_uint4((uint32_t)(i >> 2), (uint32_t)id, st,
                                                     (inst << 2) | 0u), k0, k1);
                uni[c][nn] = tn_word(x, i & 3);
            }
        } else if (eval) {
            for (int t = threadIdx.x; t < PT * Lx; t += TW * 64) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = unit0 * 16 + nn;
                crow[c][nn] = bb < B ? S[((size_t)bb * Ly + r) * Lx + c] : (int8_t)1;
            }
        }
        const size_t rowb = (size_t)r * Lx;
        for (int role = 0; role < 2; ++role) {
            const bool sweep = role == 0;
            const bool rightward = sweep ? !drawR : drawR;
            const char *Gb = uniform_ptr((const char *)(rightward ? A.GL : A.GR) + rowb * AT::SITE_BYTES);
            auto colof = [&](int t) { return rightward ? t : Lx - 1 - t; };
            auto issue = [&](int t) {   // stage t % TL <- column colof(min(t, Lx - 1))
                const char *src = Gb + (size_t)colof(min(t, Lx - 1)) * AT::SITE_BYTES + share + lane * CF::LANE;
                unsigned char *dst = ring + (t % TL) * CF::STAGE + share;
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
            AT a[CF::ABUF][2];   // [set][spin]
            lds_tiles<NT, BF16>(a[0][0], ring, lane);
            lds_tiles<NT, BF16>(a[0][1], ring + CF::STAGE / 2, lane);
            if (sweep) {
                floatx4 v0[NT], v1[NT];
#pragma unroll
                for (int mt = 0; mt < NT; ++mt) v0[mt] = v1[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                if (grp == 0) v0[0][0] = v1[0][0] = 1.0f;
                int e = 0;
                auto stepP = [&](int k, int t) {
                    const int c = colof(t);
                    floatx4 acc[2][NT];
                    mul_both<NT, BF16>(a[k % CF::ABUF], v0, v1, acc);
                    issue(t + TL - 1);
                    const bool up_minus = r > 0 && prow[c][pn] < 0;
                    const floatx4 m = *(const floatx4 *)&mixP[c][up_minus ? 1 : 0][0][0];
                    if (t % RS == 0 && t > 0) {
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[sp][mo][i] = ldexpf(acc[sp][mo][i], -e);
                    }
#pragma unroll
                    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo)
                            __builtin_amdgcn_raw_buffer_store_b128(
                                __builtin_bit_cast(uintx4, acc[sp][mo]), grs,
                                (uint32_t)(((sp * NT + mo) * 64 + lane) * 16), uniform_u32((uint32_t)c * gstride), 0);
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            v0[mo][i] = m[0] * acc[0][mo][i] + m[1] * acc[1][mo][i];
                            v1[mo][i] = m[2] * acc[0][mo][i] + m[3] * acc[1][mo][i];
                        }
                    if (t % RS == RS - 1) {
                        float mx = 0.0f;
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(acc[sp][mo][i]));
                        e = pow2_exponent_f(rows4_max(mx));
                    }
#ifdef TN_TEAM_FENCE
                    __builtin_amdgcn_sched_barrier(0);
#endif
                    // own fetch of column t + 1 has landed: at most the ops
                    // issued after it are in flight (fewer in the first steps,
                    // which follow the prologue's fetches)
                    if (t >= TL - 2) wait_vm<2 * NT + (TL - 2) * (CF::LOADS + 2 * NT)>();
                    else wait_vm<(TL - 2) * CF::LOADS + 2 * NT>();
                    team_barrier();
                    const unsigned char *st = ring + ((t + 1) % TL) * CF::STAGE;
                    lds_tiles<NT, BF16>(a[(k ^ 1) % CF::ABUF][0], st, lane);
                    lds_tiles<NT, BF16>(a[(k ^ 1) % CF::ABUF][1], st + CF::STAGE / 2, lane);
                };
                int t = 0;
                for (; t + 2 <= Lx; t += 2) {
                    stepP(0, t);
                    stepP(1, t + 1);
                }
                if (t < Lx) stepP(0, t);
            } else {
                auto gload = [&](floatx4 (&gk)[2][NT], int c) {
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo)
                            gk[s2][mo] = __builtin_bit_cast(
                                floatx4, __builtin_amdgcn_raw_buffer_load_b128(
                                             grs, (uint32_t)(((s2 * NT + mo) * 64 + lane) * 16),
                                             uniform_u32((uint32_t)c * gstride), 0));
                };
                floatx4 g[2][2][NT];
                gload(g[0], colof(0));
                gload(g[1], colof(min(1, Lx - 1)));
                floatx4 lam[NT];
#pragma unroll
                for (int mt = 0; mt < NT; ++mt) lam[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                if (grp == 0) lam[0][0] = 1.0f;
                int sprev = 0;
                // random words drawn as the row goes (when not in LDS): one
                // Philox block per four sites, kept for the next sites
                uint4 words = make_uint4(0u, 0u, 0u, 0u);
                int wblk = -1;
                const uint32_t jj = (uint32_t)unit0 * 16 + pn;
                const uint64_t wid = A.first_id + jj % (uint32_t)per_step;
                const uint32_t wst = (uint32_t)(step0 + jj / (uint32_t)per_step);
                auto stepS = [&](int k, int t) {
                    const int c = colof(t);
                    const int8_t up = prow[c][pn];
                    uint32_t word;
                    if constexpr (CF::UNI) {
                        word = uni[c][pn];
                    } else {
                        const int i = r * Lx + c;
                        if (!eval && (i >> 2) != wblk) {
                            wblk = i >> 2;
                            words = tn_philox(make_uint4((uint32_t)wblk, (uint32_t)wid, wst, (inst << 2) | 0u), k0, k1);
                        }
                        word = tn_word(words, i & 3);
                    }
                    const int8_t given = crow[c][pn];
                    const bool up_minus = r > 0 && up < 0;
                    const double2 vv = *(const double2 *)&vS[c][up_minus ? 1 : 0][sprev][0];
                    floatx4 acc[2][NT];
                    mul_both<NT, BF16>(a[k % CF::ABUF], lam, lam, acc);
                    float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            d0 = fmaf(lam[mo][i], g[k][0][mo][i], d0);
                            d1 = fmaf(lam[mo][i], g[k][1][mo][i], d1);
                        }
                    issue(t + TL - 1);
                    gload(g[k], colof(min(t + 2, Lx - 1)));
                    rows4_sum2(d0, d1);
                    double w0 = vv.x * (double)d0;
                    double w1 = vv.y * (double)d1;
                    n_clamp += (w0 < 0.0) + (w1 < 0.0);
                    w0 = fmax(w0, 0.0);
                    w1 = fmax(w1, 0.0);
                    const double tot = w0 + w1;
                    const bool bad = !(tot > 0.0 && tot <= 1.79e308);
                    n_both += bad;
                    const double u = tn_u01(word);
                    const double ut = bad ? u : u * tot, wt = bad ? 0.5 : w0, sc = bad ? 1.0 : tot;
                    const int sd = eval ? (int)given : ((ut < wt) ? 1 : -1);
                    n_near += !eval && fabs(ut - wt) < 1e-6 * sc;
                    crow[c][pn] = (int8_t)sd;
                    num *= bad ? 0.5 : (sd > 0 ? w0 : w1);
                    den *= sc;
                    sprev = sd > 0 ? 0 : 1;
                    if (t % RS == RS - 1) {
                        float mx = 0.0f;
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                            for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(lam[mo][i]));
                        const int ee = pow2_exponent_f(rows4_max(mx));
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[sp][mo][i] = ldexpf(acc[sp][mo][i], -ee);
                        int e1, e2;
                        num = frexp(num, &e1);
                        den = frexp(den, &e2);
                        nexp += e1 - e2;
                    }
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo) lam[mo] = sd > 0 ? acc[0][mo] : acc[1][mo];
#ifdef TN_TEAM_FENCE
                    __builtin_amdgcn_sched_barrier(0);
#endif
                    // own fetch of column t + 1 has landed (ops issued after it:
                    // the y loads of its step and TL - 2 steps of fetches and y
                    // loads; more in the first steps)
                    wait_vm<2 * NT + (TL - 2) * (CF::LOADS + 2 * NT)>();
                    team_barrier();
                    const unsigned char *st = ring + ((t + 1) % TL) * CF::STAGE;
                    lds_tiles<NT, BF16>(a[(k ^ 1) % CF::ABUF][0], st, lane);
                    lds_tiles<NT, BF16>(a[(k ^ 1) % CF::ABUF][1], st + CF::STAGE / 2, lane);
                };
                int t = 0;
                for (; t + 2 <= Lx; t += 2) {
                    stepS(0, t);
                    stepS(1, t + 1);
                }
                if (t < Lx) stepS(0, t);
            }
        }
        __syncthreads();   // the drawn row is complete in LDS
        {
            double eg = 0.0;
            for (int c = grp; c < Lx; c += 4) {
                const double sc = crow[c][pn];
                const double hv = h ? h[rowb + c] : 0.0;
                const double jl = c > 0 ? Jh[(size_t)r * (Lx - 1) + c - 1] * (double)crow[c - 1][pn] : 0.0;
                const double ja = r > 0 ? Jv[(size_t)(r - 1) * Lx + c] * (double)prow[c][pn] : 0.0;
                eg -= sc * (hv + jl + ja);
            }
            epart[w][grp][n] = eg;
        }
        if (!eval) {
            for (int t = threadIdx.x; t < PT * Lx; t += TW * 64) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = unit0 * 16 + nn;
                if (bb < B) S[((size_t)bb * Ly + r) * Lx + c] = crow[c][nn];
            }
        }
        __syncthreads();
        if (grp == 0) E += ((epart[w][0][n] + epart[w][1][n]) + epart[w][2][n]) + epart[w][3][n];
    }
    if (grp == 0 && valid) {
        A.logq[b] = (log(num) - log(den)) + (double)nexp * 0.69314718055994530942;
        A.energy[b] = E;
        if (n_clamp) atomicAdd(&A.counters[CNT_CLAMPS], (unsigned long long)n_clamp);
        if (n_both) atomicAdd(&A.counters[CNT_BOTH], (unsigned long long)n_both);
        if (n_near && !eval) atomicAdd(&A.counters[CNT_NEAR], (unsigned long long)n_near);
    }
}

template <int NT, bool BF16>
__global__ void __launch_bounds__(TW * 64) __attribute__((amdgpu_waves_per_eu(TeamCfg<NT, BF16>::WPE, 8)))
k_sampler_team(tn_samp_desc A, int eval, uint32_t k0, uint32_t k1, uint64_t step0,
               const uint64_t *__restrict__ step_base) {
    team_body<NT, BF16>(A, blockIdx.x * TW, eval, k0, k1, step0 + *step_base);
}

template <int NT, bool BF16>
__global__ void __launch_bounds__(TW * 64) __attribute__((amdgpu_waves_per_eu(TeamCfg<NT, BF16>::WPE, 8)))
k_sampler_team_multi(const tn_samp_desc *__restrict__ descs, int n, uint32_t k0, uint32_t k1,
                     uint64_t step0, const uint64_t *__restrict__ step_base) {
    const int u0 = (int)blockIdx.x * TW;
    int lo = 0, hi = n - 1;
    while (lo < hi) {   // last instance whose first unit is <= u0
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].blk0 <= u0) lo = mid;
        else hi = mid - 1;
    }
    const tn_samp_desc A = descs[lo];
    team_body<NT, BF16>(A, u0 - A.blk0, 0, k0, k1, step0 + *step_base);
}

// One instance: the arguments by value; the MH step is step0 + *step_base.
template <int NT, bool BF16>
__global__ void __launch_bounds__(256)
k_sampler_mfma(tn_samp_desc A, int eval, uint32_t k0, uint32_t k1, uint64_t step0,
               const uint64_t *__restrict__ step_base) {
    sampler_body<NT, BF16>(A, blockIdx.x, eval, k0, k1, step0 + *step_base);
}

// Several instances in one launch: instance i owns the blocks from
// descs[i].blk0 (ascending) on.
template <int NT, bool BF16>
__global__ void __launch_bounds__(256)
k_sampler_mfma_multi(const tn_samp_desc *__restrict__ descs, int n, uint32_t k0, uint32_t k1,
                     uint64_t step0, const uint64_t *__restrict__ step_base) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {   // last instance whose first block is <= blockIdx.x
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].blk0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const tn_samp_desc A = descs[lo];
    sampler_body<NT, BF16>(A, (int)blockIdx.x - A.blk0, 0, k0, k1, step0 + *step_base);
}

template <int NT, bool BF16>
int launch_mfma(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    const int blocks = (B + 15) / 16;
    if constexpr (team_kernel_fits<NT, BF16>()) {
        const TeamSmem T(ctx->Lx, TeamCfg<NT, BF16>::STAGE, TeamCfg<NT, BF16>::TL, TeamCfg<NT, BF16>::UNI);
        auto kern = k_sampler_team<NT, BF16>;
        if (T.total > 65536)
            TN_HIP(ctx, hipFuncSetAttribute((const void *)kern,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, T.total));
        const tn_samp_desc A = tn_samp_desc_of(ctx, B, S, logq, energy, g, per_step, first_id);
        hipLaunchKernelGGL(kern, dim3((B + TW * 16 - 1) / (TW * 16)), dim3(TW * 64), T.total, ctx->stream,
                           A, eval ? 1 : 0, (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
        TN_HIP(ctx, hipGetLastError());
        return TN_OK;
    }
    const SmemLayout<NT> L(ctx->Lx);
    auto kern = k_sampler_mfma<NT, BF16>;
    if (L.total > 65536)
        TN_HIP(ctx, hipFuncSetAttribute((const void *)kern,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, L.total));
    const tn_samp_desc A = tn_samp_desc_of(ctx, B, S, logq, energy, g, per_step, first_id);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), L.total, ctx->stream, A, eval ? 1 : 0,
                       (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

template <int NT, bool BF16>
int launch_mfma_multi(tn_ctx *ctx, const tn_samp_desc *descs, int n, int blocks, int maxLx,
                      uint64_t seed, uint64_t step0) {
    if constexpr (team_kernel_fits<NT, BF16>()) {
        // blocks counts 16-proposal units, TW-aligned per instance
        const TeamSmem T(maxLx, TeamCfg<NT, BF16>::STAGE, TeamCfg<NT, BF16>::TL, TeamCfg<NT, BF16>::UNI);
        auto kern = k_sampler_team_multi<NT, BF16>;
        if (T.total > 65536)
            TN_HIP(ctx, hipFuncSetAttribute((const void *)kern,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, T.total));
        hipLaunchKernelGGL(kern, dim3((blocks + TW - 1) / TW), dim3(TW * 64), T.total, ctx->stream, descs, n,
                           (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
        TN_HIP(ctx, hipGetLastError());
        return TN_OK;
    }
    const SmemLayout<NT> L(maxLx);
    auto kern = k_sampler_mfma_multi<NT, BF16>;
    if (L.total > 65536)
        TN_HIP(ctx, hipFuncSetAttribute((const void *)kern,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, L.total));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), L.total, ctx->stream, descs, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), step0, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

template <bool BF16>
int dispatch_nt(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    switch (ctx->Dp / 16) {
    case 1: return launch_mfma<1, BF16>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 2: return launch_mfma<2, BF16>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 3: return launch_mfma<3, BF16>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 4: return launch_mfma<4, BF16>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    default: return tn_fail(ctx, TN_EINVAL, "bond dimension above 64");
    }
}

}  // namespace

int tn_run_mfma(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                uint64_t first_id, int8_t *spins, bool eval, double *logq, double *energy) {
    if (batch == 0) return TN_OK;
    if (ctx->Lx > TN_MAX_LX) return tn_fail(ctx, TN_EINVAL, "Lx above 256");
    if (per_step <= 0) return tn_fail(ctx, TN_EINVAL, "proposals per step must be positive");
    int rc;
    if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, tn_mfma_scratch_bytes(ctx, batch)))) return rc;
    float *g = (float *)ctx->gscr;
    if (ctx->prec == TN_BF16)
        return dispatch_nt<true>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    return dispatch_nt<false>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
}

int tn_run_mfma_multi(tn_ctx *ctx, int NT, bool bf16, const tn_samp_desc *descs, int n, int blocks,
                      int maxLx, uint64_t seed, uint64_t step0) {
    if (blocks == 0) return TN_OK;
    if (maxLx > TN_MAX_LX) return tn_fail(ctx, TN_EINVAL, "Lx above 256");
    switch (NT * 2 + (bf16 ? 1 : 0)) {
    case 2: return launch_mfma_multi<1, false>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 3: return launch_mfma_multi<1, true>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 4: return launch_mfma_multi<2, false>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 5: return launch_mfma_multi<2, true>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 6: return launch_mfma_multi<3, false>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 7: return launch_mfma_multi<3, true>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 8: return launch_mfma_multi<4, false>(ctx, descs, n, blocks, maxLx, seed, step0);
    case 9: return launch_mfma_multi<4, true>(ctx, descs, n, blocks, maxLx, seed, step0);
    default: return tn_fail(ctx, TN_EINVAL, "bond dimension above 64");
    }
}
