// gfx950 kernels of the 2D parallel tempering library.
//
// Round structure (Algorithm 1): every replica performs mcs sweeps, f and g
// of its final state are known, one swap step runs, the bottom-right replica
// is recorded.  Replica configurations never move: a swap exchanges the
// position labels of two replica slots (pos_slot / slot_pos), which is the
// same as exchanging the configurations.
//
// Sweep layout: one workgroup owns one replica slot and keeps its int8 spins
// in LDS, starting at LDS address 0, so a neighbour index is its LDS byte
// address.  Spins are numbered colour-major; a lane takes a quad of 4
// consecutive spins of the current colour class, which share one
// Philox4x32-10 call and one 16-byte load per structure row.  Same-colour
// spins have no coupling between them, so updating a whole class in
// parallel equals updating it one spin at a time (chromatic Gibbs), and the
// workgroup barrier between classes keeps the sweep order.
//
// Two drivers share the sweep:
//   k_round_sweep + k_swap_track  one launch pair per round (any grid size);
//   k_persistent (+ k_finalize)   one cooperative launch for many rounds,
//                                 every replica resident in LDS; no grid
//                                 barrier: the two partners of a swap pair
//                                 exchange (f, g) through per-position
//                                 mailboxes and take the same decision.
#include "tdpt_internal.h"

#include <math.h>

namespace tdpt {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef short v2s __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, the key bumped by
// the published Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0, y2;
        if (rnd < 2) {
            // the first rounds mix in words that are often uniform: plain
            // xors let the compiler keep those parts scalar
            y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
            y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
        } else {
            // three-input xor in one gfx950 bitop3 (truth table 0x96)
            y0 = (uint32_t)__builtin_amdgcn_bitop3_b32((int)(m1 >> 32), (int)x1, (int)k0, 0x96);
            y2 = (uint32_t)__builtin_amdgcn_bitop3_b32((int)(m0 >> 32), (int)x3, (int)k1, 0x96);
        }
        x1 = (uint32_t)m1;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double philox_u53(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1)
{
    philox10(c0, c1, c2, c3, k0, k1);
    return ((double)(c0 >> 5) * 67108864.0 + (double)(c1 >> 6)) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------- heat-bath decision
// The decision is the double-precision expression
//   +1  iff  (double)u < ldexp(1 / (1 + exp(-ldexp(beta * h, -11))), 32)
// i.e. P(+1) = sigma(2 beta h) with h in Q12.
//
// heat_bath_up pre-tests it in single precision in product form: with
// e = exp(-x) the spin goes up iff t = u (1 + e) < 2^32 (no reciprocal).
// Error of the float t near t = 2^32: e is exp2 of y = h * cb, whose
// relative error is at most 3 * 2^-24 (rounding of cb, of h, of the
// product), so e carries a relative error below 2.1 |y| 2^-24 + 2^-23
// (v_exp_f32 is good to 1 ulp).  Near the boundary u e <= 2^32, so for
// y in [-32, 0] that term is below 2^14.1, and for y > 0 below
// 2^32 (1.1 * 2^-24 + 2^-23) < 2^9.7; rounding u and the fma add
// 2^8 each.  Whenever |t - 2^32| >= 2^16 the float answer is therefore the
// exact one; otherwise the lane is flagged and the double expression
// decides (about 2^-15 of all updates).  u = 0 with e = inf gives a NaN
// t, which fails the margin test and is flagged too; e = inf with u > 0
// gives t = inf, down, which is also the exact answer (p < 2^-96).
__device__ __attribute__((noinline)) int heat_bath_exact(double beta, int h, uint32_t u)
{
    const double x = ldexp(beta * (double)h, -11);
    const double p = 1.0 / (1.0 + exp(-x));
    return ((double)u < ldexp(p, 32)) ? 1 : -1;
}

// The pre-test's margin d = t - 2^32 (computed exactly whenever t < 2^32,
// where the float spacing is at most 256): the spin goes up iff d < 0, i.e.
// iff d's sign bit is set (t >= 2^32, and t = inf, give +0 or more), and the
// lane needs the double expression iff !(|d| >= 2^16), which includes a NaN t.
__device__ __forceinline__ float heat_bath_margin(int h, float cb, uint32_t u)
{
    const float e = __builtin_amdgcn_exp2f(-((float)h * cb));  // cb = beta log2(e) / 2048
    const float uf = (float)u;
    return __builtin_fmaf(uf, e, uf) - 4294967296.0f;
}

__device__ __forceinline__ bool margin_ambiguous(float d) { return !(fabsf(d) >= 65536.0f); }

__device__ __forceinline__ bool heat_bath_up(int h, float cb, uint32_t u, bool &ambiguous)
{
    const float d = heat_bath_margin(h, cb, u);
    ambiguous = margin_ambiguous(d);
    return (__float_as_uint(d) >> 31) != 0u;
}

// Byte j = 0xff when d_j's sign bit is set, else 0: v_perm_b32 selectors 9
// and 11 replicate the sign bits of the low and the high operand.
__device__ __forceinline__ uint32_t sign_bytes4(const float d[4])
{
    const uint32_t lo = __builtin_amdgcn_perm(__float_as_uint(d[1]), __float_as_uint(d[0]), 0x0c0c0b09u);
    const uint32_t hi = __builtin_amdgcn_perm(__float_as_uint(d[3]), __float_as_uint(d[2]), 0x0b090c0cu);
    return lo | hi;
}

// ------------------------------------------------------ structure access
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, kRsrcWord3);
}

struct Rsrc {
    __amdgpu_buffer_rsrc_t a, b, ch, bias;
    __amdgpu_buffer_rsrc_t cw, kh;  // general constraints: weights, linear part (ch: indices)
};

__device__ __forceinline__ Rsrc make_rsrc(const DevProblem &P)
{
    Rsrc r;
    // descriptors a layout does not use cover no bytes: a load through one
    // returns zeros instead of touching memory
    r.cw = rsrc(nullptr, 0);
    r.kh = rsrc(nullptr, 0);
    if (P.bits) {
        const int bytes = P.wd * P.n_pad * 4;
        r.a = rsrc(P.nb_pos, bytes);
        r.b = P.pair16 ? rsrc(P.nb_J2, bytes) : rsrc(P.nb_J, bytes);
        r.ch = rsrc(P.ch_pos, P.n_pad * 8);
        r.bias = rsrc(P.h0, P.n_pad * 4);
        return r;
    }
    if (P.narrow) {
        const int bytes = (P.wd / 2) * P.n_pad * 4;
        r.a = rsrc(P.nbi, bytes);
        r.b = rsrc(P.nbj, bytes);
        if (P.gen) {
            r.ch = rsrc(P.cn_idx, P.wcg * P.n_pad * 4);
            r.cw = rsrc(P.cn_w, P.wcg * P.n_pad * 4);
            r.kh = rsrc(P.kh, P.n_pad * 4);
        } else {
            r.ch = rsrc(P.chp, P.n_pad * 4);
        }
    } else {
        const int bytes = P.wd * P.n_pad * 4;
        r.a = rsrc(P.nb_idx, bytes);
        r.b = rsrc(P.nb_J, bytes);
        if (P.gen) {
            r.ch = rsrc(P.cn_idx, P.wcg * P.n_pad * 4);
            r.cw = rsrc(P.cn_w, P.wcg * P.n_pad * 4);
            r.kh = rsrc(P.kh, P.n_pad * 4);
        } else {
            r.ch = rsrc(P.ch_idx, P.n_pad * 8);
        }
    }
    r.bias = rsrc(P.bias, P.n_pad * 4);
    return r;
}

__device__ __forceinline__ v4i bload(const __amdgpu_buffer_rsrc_t &r, int voff, int soff)
{
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}

// The replica a byte-layout sweep workgroup holds sits at LDS byte 0: the
// sweep kernels declare no static LDS, so their dynamic LDS starts there.
// Reading it through an LDS pointer with the constant base 0 lets a
// neighbour's index serve directly as the gather address (a pointer to the
// dynamic array would add its link-time base to every index).  The kernels
// check the assumption once and refuse to run if it does not hold.
typedef __attribute__((address_space(3))) int8_t lds8_t;
typedef __attribute__((address_space(3))) uint32_t lds32_t;
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u4v lds_u4_t;
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u2v lds_u2_t;

__device__ __forceinline__ lds8_t *replica_lds() { return (lds8_t *)(uintptr_t)0u; }

__device__ __forceinline__ bool replica_at_zero(int8_t *lds)
{
    return (uint32_t)(uintptr_t)(lds8_t *)lds == 0u;
}

// Error word value when a sweep kernel finds its dynamic LDS elsewhere.
constexpr int64_t kErrLdsBase = 2;
// Error word value when a bit-packed sweep kernel of one form is launched on
// a problem laid out in the other.
constexpr int64_t kErrBitsForm = 3;

// Per-slot parameters of the current round.
struct SlotParams {
    double beta;
    float cb;      // beta * log2(e) / 2048, rounded to float
    int twoP;      // 2 * P_q of the slot's column
    uint32_t pos;  // grid position (Philox counter word)
};

// beta / p_q: the problem's ladders, or copies of them in LDS.
__device__ __forceinline__ SlotParams slot_params(const DevProblem &P, int pos, const double *beta,
                                                  const int32_t *p_q)
{
    SlotParams sp;
    const int i = pos / P.J, j = pos - i * P.J;
    sp.beta = beta[i];
    sp.cb = (float)(sp.beta * (1.4426950408889634 / 2048.0));
    sp.twoP = 2 * p_q[j];
    sp.pos = (uint32_t)pos;
    return sp;
}

// Structure of one quad (4 consecutive colour-major spins): one 16-byte
// load per structure row.  Up to 8 neighbours per spin every row is held at
// once; wider rows are streamed in chunks by quad_fields (kStream), which
// keeps them out of spill territory.  WD = 0 stands for a width known only
// at run time (P.wd, a multiple of 8 above 48), streamed the same way.
// NARROW, here and in the sweep templates below, is the structure layout:
// kWide (0), kPacked (1) or kPackedGen (2); nonzero means packed problem
// rows.
template <int NARROW, int WD>
struct QuadS {
    static constexpr bool kStream = WD > 8 || WD == 0;
    static constexpr int K = kStream ? 1 : (NARROW ? WD / 2 : WD);
    v4i a[K];    // narrow: index pairs; wide: indices
    v4i b[K];    // narrow: coupling pairs; wide: couplings
    v4i c0, c1;  // narrow: copy pairs in c0; wide: two copy rows
    v4i bias;    // fields (zero when the instance has none)
    int voff;    // byte offset of the quad in a structure row
};

// Layouts the packed-slot sweeps may run with one spin per lane.
template <int NARROW, int WD>
constexpr bool kSpinLanes = NARROW == kPacked && WD >= 2 && WD <= 8;

// Layouts whose structure the packed-slot sweeps may hold in registers.
template <int NARROW, int WD>
constexpr bool kHoistable = NARROW == kPacked && WD <= 4;

template <int NARROW, int WD>
__device__ __forceinline__ void load_quad(const DevProblem &P, const Rsrc &Rs, int q, QuadS<NARROW, WD> &Q)
{
    const int voff = q * 16;
    const int row = P.n_pad * 4;
    Q.voff = voff;
    if constexpr (!QuadS<NARROW, WD>::kStream) {
#pragma unroll
        for (int k = 0; k < QuadS<NARROW, WD>::K; ++k) {
            Q.a[k] = bload(Rs.a, voff, k * row);
            Q.b[k] = bload(Rs.b, voff, k * row);
        }
    }
    if constexpr (NARROW == kPacked) {
        Q.c0 = bload(Rs.ch, voff, 0);
    } else if (NARROW == kWide && !P.gen) {
        Q.c0 = bload(Rs.ch, voff, 0);
        Q.c1 = bload(Rs.ch, voff, row);
    }
    if (P.has_bias) Q.bias = bload(Rs.bias, voff, 0);
    else Q.bias = v4i{0, 0, 0, 0};
}

__device__ __forceinline__ int sbyte(uint32_t w, int j)
{
    return (int)(int8_t)(w >> (8 * j));
}

// Half the penalty field of the 4 spins of a quad under general constraints:
// kh + sum_k w_k s_k over the constraint ELL, streamed 4 rows at a time (the
// width is a multiple of 4; padding rows name the zero spin with weight 0).
__device__ __forceinline__ void quad_constraint_sum(const DevProblem &P, const Rsrc &Rs, const lds8_t *s,
                                                    int voff, int cs[4])
{
    const v4i k = bload(Rs.kh, voff, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) cs[j] = k[j];
    const int row = P.n_pad * 4;
    for (int k0 = 0; k0 < P.wcg; k0 += 4) {
        v4i ci[4], cw[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ci[c] = bload(Rs.ch, voff, (k0 + c) * row);
            cw[c] = bload(Rs.cw, voff, (k0 + c) * row);
        }
        int sv[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) sv[c][j] = s[ci[c][j]];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[j] += cw[c][j] * sv[c][j];
    }
}

// Local fields of the 4 spins of a quad from the LDS spins s: hp = problem
// part (couplings and field), cs = half the penalty field (the sum of the
// copy neighbours, or the general-constraint sum).  NARROW
// instances keep every field below 2^22, so the 16-bit dot products are
// exact.
template <int NARROW, int WD>
__device__ __forceinline__ void quad_fields(const DevProblem &P, const Rsrc &Rs, const lds8_t *s,
                                            const QuadS<NARROW, WD> &Q, int hp[4], int cs[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) hp[j] = Q.bias[j];
    if constexpr (QuadS<NARROW, WD>::kStream) {
        // rows streamed in chunks of kChunk (pairs or neighbours)
        const int K = NARROW ? (WD ? WD : P.wd) / 2 : (WD ? WD : P.wd);
        constexpr int kChunk = NARROW ? 4 : 8;
        const int row = P.n_pad * 4;
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += kChunk) {
            v4i a[kChunk], b[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c)
                if (k0 + c < K) {
                    a[c] = bload(Rs.a, Q.voff, (k0 + c) * row);
                    b[c] = bload(Rs.b, Q.voff, (k0 + c) * row);
                }
            if constexpr (NARROW) {
                int8_t lo[kChunk][4], hi[kChunk][4];
#pragma unroll
                for (int c = 0; c < kChunk; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (k0 + c < K) {
                            const int iw = a[c][j];
                            lo[c][j] = s[iw & 0xffff];
                            hi[c][j] = s[(unsigned)iw >> 16];
                        }
#pragma unroll
                for (int c = 0; c < kChunk; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (k0 + c < K) {
                            const int jw = b[c][j];
                            v2s sv, jv;
                            sv.x = lo[c][j];
                            sv.y = hi[c][j];
                            jv.x = (short)(jw & 0xffff);
                            jv.y = (short)((unsigned)jw >> 16);
                            hp[j] = __builtin_amdgcn_sdot2(jv, sv, hp[j], false);
                        }
            } else {
#pragma unroll
                for (int c = 0; c < kChunk; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (k0 + c < K) hp[j] += b[c][j] * (int)s[a[c][j]];
            }
        }
        if constexpr (NARROW == kPackedGen) {
            quad_constraint_sum(P, Rs, s, Q.voff, cs);
        } else if constexpr (NARROW == kPacked) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = Q.c0[j];
                cs[j] = (int)s[c & 0xffff] + (int)s[(unsigned)c >> 16];
            }
        } else if (P.gen) {
            quad_constraint_sum(P, Rs, s, Q.voff, cs);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[j] = (int)s[Q.c0[j]] + (int)s[Q.c1[j]];
        }
        return;
    } else if constexpr (NARROW) {
        // every LDS read of the quad is issued before the first product, so
        // their latencies overlap
        int8_t lo[WD / 2][4], hi[WD / 2][4], ca[4], cb[4];
#pragma unroll
        for (int k2 = 0; k2 < WD / 2; ++k2)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int iw = Q.a[k2][j];  // plain int: bit-cast a value, not a vector lane
                lo[k2][j] = s[iw & 0xffff];
                hi[k2][j] = s[(unsigned)iw >> 16];
            }
        if constexpr (NARROW == kPacked) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = Q.c0[j];
                ca[j] = s[c & 0xffff];
                cb[j] = s[(unsigned)c >> 16];
            }
        }
#pragma unroll
        for (int k2 = 0; k2 < WD / 2; ++k2)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jw = Q.b[k2][j];
                v2s sv, jv;
                sv.x = lo[k2][j];
                sv.y = hi[k2][j];
                jv.x = (short)(jw & 0xffff);
                jv.y = (short)((unsigned)jw >> 16);
                hp[j] = __builtin_amdgcn_sdot2(jv, sv, hp[j], false);
            }
        if constexpr (NARROW == kPackedGen) {
            quad_constraint_sum(P, Rs, s, Q.voff, cs);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[j] = (int)ca[j] + (int)cb[j];
        }
    } else {
#pragma unroll
        for (int k = 0; k < WD; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) hp[j] += Q.b[k][j] * (int)s[Q.a[k][j]];
        if (P.gen) {
            quad_constraint_sum(P, Rs, s, Q.voff, cs);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[j] = (int)s[Q.c0[j]] + (int)s[Q.c1[j]];
        }
    }
}

// Heat-bath update of the 4 spins of quad q (LDS bytes s) given their
// fields.  live_bytes has 0xff in byte j when spin 4q+j is a real spin (not
// class padding); padding spins stay 0.  Padding rows have zero couplings,
// field and copies, so their h and copy sums are 0 and they add nothing to
// the energy changes.  dfa accumulates the change of f, dga half the change
// of g (24-bit multiplies are exact for NARROW instances, whose fields and
// energy changes stay below 2^22).
template <int NARROW>
__device__ __forceinline__ void quad_update(const DevProblem &P, lds8_t *s, int q, const int hp[4], const int cs[4],
                                            uint32_t live_bytes, const uint32_t u[4], const SlotParams &sp,
                                            int &dfa, int &dga)
{
    lds32_t *wp = (lds32_t *)(s + q * 4);
    const uint32_t ow = *wp;
    int hh[4];
    float d[4];
    bool amb_any = false;  // padding lanes may set it too: the exact path skips them
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if constexpr (NARROW) hh[j] = __mul24(sp.twoP, cs[j]) + hp[j];
        else hh[j] = sp.twoP * cs[j] + hp[j];
        d[j] = heat_bath_margin(hh[j], sp.cb, u[j]);
        amb_any |= margin_ambiguous(d[j]);
    }
    uint32_t up = sign_bytes4(d);  // byte j = 0xff when spin j goes up
    if (__builtin_expect(amb_any, 0)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (margin_ambiguous(d[j]) && ((live_bytes >> (8 * j)) & 1u)) {
                const uint32_t byte = heat_bath_exact(sp.beta, hh[j], u[j]) > 0 ? 0xffu : 0u;
                up = (up & ~(0xffu << (8 * j))) | (byte << (8 * j));
            }
        }
    }
    // byte j: +1 (0x01) when up, -1 (0xff) otherwise, 0 for padding
    const uint32_t nw = (0xffffffffu ^ (up & 0xfefefefeu)) & live_bytes;
    *wp = nw;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int ds = sbyte(nw, j) - sbyte(ow, j);
        if constexpr (NARROW) {
            dfa -= __mul24(ds, hp[j]);
            dga -= __mul24(ds, cs[j]);
        } else {
            dfa -= ds * hp[j];
            dga -= ds * cs[j];
        }
    }
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// All sweeps of one round of the slot held at LDS address 0; leaves the
// change of f and g summed over the block in red[0..1] (LDS scratch of
// 2 * (blockDim / 64) int64), written and meant to be read by thread 0 only.
// A lane walks its quads q0 + tid, q0 + tid + blockDim, .. of every class.
// at_end() runs on every thread after its last quad, before the closing
// barrier (the reduction's, which also ends the last class); on return the
// spins are final for the whole block.
// The class phases of all sweeps of one round for the replica at s, walked
// by `lanes` lanes of which this one is number `lane` (quads lane,
// lane + lanes, .. of every class); adds the changes of f and g that this
// lane made to df and dg.  Every thread of the block calls it (the phases
// end in block barriers, the last one excepted).
// The class phases of all sweeps of one round for the replica at s, walked
// by `lanes` lanes of which this one is number `lane` (quads lane,
// lane + lanes, .. of every class); adds the changes of f and g that this
// lane made to df and dg.  Every thread of the block calls it (the phases
// end in block barriers, the last one excepted).
// HOIST (packed copy-edge layout, at most 4 problem neighbours, no fields):
// when there are two colour classes of at most `lanes` quads each (small
// bipartite instances), every lane holds the structure of its (at most) one
// quad per class in registers for the whole round instead of loading it
// again in every phase, whose latency then no longer waits on the cache
// (the classes' loop unrolled, so both quads stay in registers, and the
// Philox key read once per round).  It costs about 75 registers, so only
// the packed-slot sweeps, which run such replicas, use it.
template <int NARROW, int WD, bool HOIST = false>
__device__ __forceinline__ void sweep_phases(const DevProblem &P, const Rsrc &Rs, lds8_t *s, const SlotParams &sp,
                                             int64_t n_round, int lane, int lanes, int64_t &df, int64_t &dg)
{
    const int mcs = P.mcs;
    if constexpr (HOIST && kHoistable<NARROW, WD>) {
        const uint32_t key0 = P.key0, key1 = P.key1;
        const int qa = P.cls_start[0] >> 2, qb = P.cls_start[1] >> 2, qc = P.cls_start[2] >> 2;
        if (P.n_colors == 2 && !P.has_bias && qb - qa <= lanes && qc - qb <= lanes) {
            QuadS<NARROW, WD> QQ[2];
            const int qq[2] = {qa + lane, qb + lane};
            const bool has[2] = {qq[0] < qb, qq[1] < qc};
            const int live_end[2] = {P.cls_live[0], P.cls_live[1]};
#pragma unroll
            for (int c = 0; c < 2; ++c)
                if (has[c]) load_quad<NARROW, WD>(P, Rs, qq[c], QQ[c]);
            for (int k = 0; k < mcs; ++k) {
                const uint32_t t = (uint32_t)((n_round - 1) * mcs + k);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    int dfa = 0, dga = 0;
                    if (has[c]) {
                        const int q = qq[c];
                        uint32_t u[4] = {(uint32_t)q, t, sp.pos, 0u};
                        philox10(u[0], u[1], u[2], u[3], key0, key1);
                        int hp[4], cs[4];
                        quad_fields<NARROW, WD>(P, Rs, s, QQ[c], hp, cs);
                        const int rem = live_end[c] - q * 4;
                        const uint32_t live_bytes =
                            rem >= 4 ? 0xffffffffu : rem <= 0 ? 0u : ((1u << (8 * rem)) - 1u);
                        quad_update<NARROW>(P, s, q, hp, cs, live_bytes, u, sp, dfa, dga);
                    }
                    df += dfa;
                    dg += 2 * (int64_t)dga;
                    if (k + 1 < mcs || c == 0) __syncthreads();
                }
            }
            return;
        }
    }
    for (int k = 0; k < mcs; ++k) {
        const uint32_t t = (uint32_t)((n_round - 1) * mcs + k);
        for (int c = 0; c < P.n_colors; ++c) {
            const int q0 = P.cls_start[c] >> 2, q1 = P.cls_start[c + 1] >> 2;
            const int live_end = P.cls_live[c];
            int dfa = 0, dga = 0;
            for (int q = q0 + lane; q < q1; q += lanes) {
                QuadS<NARROW, WD> Q;
                load_quad<NARROW, WD>(P, Rs, q, Q);
                // the quad's random words do not depend on the spins: they are
                // computed while its structure loads are in flight
                uint32_t u[4] = {(uint32_t)q, t, sp.pos, 0u};
                philox10(u[0], u[1], u[2], u[3], P.key0, P.key1);
                int hp[4], cs[4];
                quad_fields<NARROW, WD>(P, Rs, s, Q, hp, cs);
                const int rem = live_end - q * 4;
                const uint32_t live_bytes = rem >= 4 ? 0xffffffffu : rem <= 0 ? 0u : ((1u << (8 * rem)) - 1u);
                quad_update<NARROW>(P, s, q, hp, cs, live_bytes, u, sp, dfa, dga);
            }
            df += dfa;
            dg += 2 * (int64_t)dga;
            if (k + 1 < mcs || c + 1 < P.n_colors) __syncthreads();
        }
    }
}

__device__ __forceinline__ int bload1(const __amdgpu_buffer_rsrc_t &r, int voff, int soff)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// Structure of one spin in the packed copy-edge layout (K = WD / 2 pairs).
template <int WD>
struct SpinS {
    int a[WD / 2], b[WD / 2], ch, bias;
};

template <int WD>
__device__ __forceinline__ void load_spin(const DevProblem &P, const Rsrc &Rs, int i, SpinS<WD> &S)
{
    const int voff = i * 4, row = P.n_pad * 4;
#pragma unroll
    for (int k = 0; k < WD / 2; ++k) {
        S.a[k] = bload1(Rs.a, voff, k * row);
        S.b[k] = bload1(Rs.b, voff, k * row);
    }
    S.ch = bload1(Rs.ch, voff, 0);
    S.bias = P.has_bias ? bload1(Rs.bias, voff, 0) : 0;
}

// One spin per lane: lanes 4m..4m+3 of a replica's lane group take the 4
// spins of one quad; each computes the quad's Philox words and uses its own
// (the same word, field and decision as the quad-per-lane update, so the
// same trajectory).  A quarter of the fields, heat-bath decisions and
// gathers per lane shortens each colour phase when the replica's lanes are
// latency-bound (few replicas on the GPU); the Philox work is repeated 4
// times, so it loses when the GPU is full.
template <int WD>
__device__ __forceinline__ void spin_update(const DevProblem &P, lds8_t *s, int q, int j, const SpinS<WD> &S,
                                            int live_end, uint32_t t, const SlotParams &sp, uint32_t key0,
                                            uint32_t key1, int &dfa, int &dga)
{
    uint32_t u[4] = {(uint32_t)q, t, sp.pos, 0u};
    philox10(u[0], u[1], u[2], u[3], key0, key1);
    const uint32_t uj = j == 0 ? u[0] : j == 1 ? u[1] : j == 2 ? u[2] : u[3];
    const int i = 4 * q + j;
    int8_t lo[WD / 2], hi[WD / 2];
#pragma unroll
    for (int k = 0; k < WD / 2; ++k) {
        lo[k] = s[S.a[k] & 0xffff];
        hi[k] = s[(unsigned)S.a[k] >> 16];
    }
    const int8_t c0 = s[S.ch & 0xffff], c1 = s[(unsigned)S.ch >> 16];
    const int8_t old = s[i];
    int hp = S.bias;
#pragma unroll
    for (int k = 0; k < WD / 2; ++k) {
        v2s sv, jv;
        sv.x = lo[k];
        sv.y = hi[k];
        jv.x = (short)(S.b[k] & 0xffff);
        jv.y = (short)((unsigned)S.b[k] >> 16);
        hp = __builtin_amdgcn_sdot2(jv, sv, hp, false);
    }
    const int cs = (int)c0 + (int)c1;
    const int hh = __mul24(sp.twoP, cs) + hp;
    bool amb;
    bool up = heat_bath_up(hh, sp.cb, uj, amb);
    const bool live = i < live_end;
    if (__builtin_expect(amb && live, 0)) up = heat_bath_exact(sp.beta, hh, uj) > 0;
    const int nw = live ? (up ? 1 : -1) : 0;
    s[i] = (int8_t)nw;
    const int ds = nw - (int)old;
    dfa -= __mul24(ds, hp);
    dga -= __mul24(ds, cs);
}

// The round's phases when each of the NC colour classes has at most one
// quad per 4 lanes: every lane holds its (at most) one spin per class of
// structure in registers for the whole round (2 WD / 2 + 2 words a class).
template <int NC, int WD>
__device__ __forceinline__ void spin_phases_held(const DevProblem &P, const Rsrc &Rs, lds8_t *s,
                                                 const SlotParams &sp, int64_t n_round, int j, int ql,
                                                 uint32_t key0, uint32_t key1, int64_t &df, int64_t &dg)
{
    SpinS<WD> SS[NC];
    int qq[NC], live_end[NC];
    bool has[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        qq[c] = (P.cls_start[c] >> 2) + ql;
        has[c] = qq[c] < (P.cls_start[c + 1] >> 2);
        live_end[c] = P.cls_live[c];
        if (has[c]) load_spin<WD>(P, Rs, 4 * qq[c] + j, SS[c]);
    }
    const int mcs = P.mcs;
    for (int k = 0; k < mcs; ++k) {
        const uint32_t t = (uint32_t)((n_round - 1) * mcs + k);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            int dfa = 0, dga = 0;
            if (has[c]) spin_update<WD>(P, s, qq[c], j, SS[c], live_end[c], t, sp, key0, key1, dfa, dga);
            df += dfa;
            dg += 2 * (int64_t)dga;
            if (k + 1 < mcs || c + 1 < NC) __syncthreads();
        }
    }
}

// The class phases of a round with one spin per lane (lanes a multiple of
// 4); with 2 to 4 colour classes of at most lanes / 4 quads each, the
// structure is held in registers for the round (spin_phases_held).
template <int NARROW, int WD>
__device__ __forceinline__ void sweep_phases_spin(const DevProblem &P, const Rsrc &Rs, lds8_t *s,
                                                  const SlotParams &sp, int64_t n_round, int lane, int lanes,
                                                  int64_t &df, int64_t &dg)
{
    if constexpr (NARROW == kPacked && WD >= 2 && WD <= 8) {
        const int mcs = P.mcs, n_colors = P.n_colors;
        const uint32_t key0 = P.key0, key1 = P.key1;
        const int j = lane & 3, ql = lane >> 2, qn = lanes >> 2;
        bool held = n_colors >= 2 && n_colors <= 4;
        for (int c = 0; held && c < n_colors; ++c)
            held = (P.cls_start[c + 1] >> 2) - (P.cls_start[c] >> 2) <= qn;
        if (held) {
            if (n_colors == 2) spin_phases_held<2, WD>(P, Rs, s, sp, n_round, j, ql, key0, key1, df, dg);
            else if (n_colors == 3) spin_phases_held<3, WD>(P, Rs, s, sp, n_round, j, ql, key0, key1, df, dg);
            else spin_phases_held<4, WD>(P, Rs, s, sp, n_round, j, ql, key0, key1, df, dg);
            return;
        }
        for (int k = 0; k < mcs; ++k) {
            const uint32_t t = (uint32_t)((n_round - 1) * mcs + k);
            for (int c = 0; c < n_colors; ++c) {
                const int q0 = P.cls_start[c] >> 2, q1 = P.cls_start[c + 1] >> 2;
                const int live_end = P.cls_live[c];
                int dfa = 0, dga = 0;
                for (int q = q0 + ql; q < q1; q += qn) {
                    SpinS<WD> S;
                    load_spin<WD>(P, Rs, 4 * q + j, S);
                    spin_update<WD>(P, s, q, j, S, live_end, t, sp, key0, key1, dfa, dga);
                }
                df += dfa;
                dg += 2 * (int64_t)dga;
                if (k + 1 < mcs || c + 1 < n_colors) __syncthreads();
            }
        }
    }
}

template <int NARROW, int WD, typename AtEnd>
__device__ __forceinline__ void sweep_round(const DevProblem &P, const Rsrc &Rs, lds8_t *s,
                                            const SlotParams &sp, int64_t n_round, int64_t *red,
                                            AtEnd &&at_end)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    int64_t df = 0, dg = 0;
    sweep_phases<NARROW, WD>(P, Rs, s, sp, n_round, tid, nthr, df, dg);
    at_end();
    const int64_t a = wave_sum64(df), b = wave_sum64(dg);
    const int wave = tid >> 6, nw = nthr >> 6;
    if ((tid & 63) == 0) { red[2 + 2 * wave] = a; red[3 + 2 * wave] = b; }
    __syncthreads();
    if (tid == 0) {
        int64_t sa = 0, sb = 0;
        for (int w = 0; w < nw; ++w) { sa += red[2 + 2 * w]; sb += red[3 + 2 * w]; }
        red[0] = sa;
        red[1] = sb;
    }
}

__device__ __forceinline__ void copy_bytes16(int8_t *dst, const int8_t *src, int bytes)
{
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (int v = threadIdx.x; v < (bytes >> 4); v += blockDim.x) d[v] = s[v];
}

// LDS of the sweep kernels: [0, stride) spins, then int64 scratch.
__device__ __forceinline__ int64_t *lds_scratch(int8_t *lds, int stride)
{
    return reinterpret_cast<int64_t *>(lds + stride);
}

// --------------------------------------------------- one launch per round
// One round of one slot: load its spins into LDS, mcs sweeps, store.
template <int NARROW, int WD>
__device__ __forceinline__ void round_sweep_body(const DevProblem &P, int slot, int8_t *lds)
{
    if (!replica_at_zero(lds)) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&P.hdr[kHdrError], kErrLdsBase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    int64_t *red = lds_scratch(lds, P.stride);
    copy_bytes16(lds, P.states + (size_t)slot * P.stride, P.stride);
    const int64_t n_round = P.hdr[kHdrRounds] + 1;
    const SlotParams sp = slot_params(P, P.slot_pos[slot], P.beta, P.p_q);
    const Rsrc Rs = make_rsrc(P);
    __syncthreads();
    sweep_round<NARROW, WD>(P, Rs, replica_lds(), sp, n_round, red, [] {});
    if (threadIdx.x == 0) {
        P.f[slot] += red[0];
        P.g[slot] += red[1];
    }
    copy_bytes16(P.states + (size_t)slot * P.stride, lds, P.stride);
}

template <int NARROW, int WD>
__global__ __launch_bounds__(kMaxBlock) void k_round_sweep(DevProblem P)
{
    extern __shared__ __align__(16) int8_t lds[];
    round_sweep_body<NARROW, WD>(P, blockIdx.x, lds);
}

// Batched round: block b serves slot b - first_block[p] of member p, where
// first_block is the prefix sum of the members' replica counts.
template <int NARROW, int WD>
__global__ __launch_bounds__(kMaxBlock) void k_batch_sweep(const DevProblem *__restrict__ table,
                                                         const int *__restrict__ first_block, int count)
{
    extern __shared__ __align__(16) int8_t lds[];
    const int b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    round_sweep_body<NARROW, WD>(table[lo], b - first_block[lo], lds);
}

// One round of `rpb` consecutive slots of one problem in one workgroup: the
// block's threads split into rpb groups of 2^lshift lanes (lshift <= 6 keeps
// a group inside one wave; larger groups span whole waves), group k sweeping
// slot slot0 + k, whose spins sit at LDS offset k * stride.  Replicas of a
// few dozen quads per class then share a wave instead of each leaving most
// of one idle.  Slots past the problem's last are skipped; their groups
// still take every barrier.  The same updates, in the same order per slot,
// as round_sweep_body.
template <int NARROW, int WD>
__device__ __forceinline__ void multi_round_body(const DevProblem &P, int slot0, int rpb, int lshift, int spin,
                                                 int8_t *lds)
{
    if (!replica_at_zero(lds)) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&P.hdr[kHdrError], kErrLdsBase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int tid = threadIdx.x;
    const int nsub = min(rpb, P.R - slot0);
    const int sub = tid >> lshift, lane = tid & ((1 << lshift) - 1);
    const bool live = sub < nsub;
    int64_t *red = lds_scratch(lds, rpb * P.stride);  // [2k] f, [2k + 1] g of group k
    copy_bytes16(lds, P.states + (size_t)slot0 * P.stride, nsub * P.stride);
    for (int i = tid; i < 2 * rpb; i += blockDim.x) red[i] = 0;
    const int slot = slot0 + min(sub, nsub - 1);
    const int64_t n_round = P.hdr[kHdrRounds] + 1;
    const SlotParams sp = slot_params(P, P.slot_pos[slot], P.beta, P.p_q);
    const Rsrc Rs = make_rsrc(P);
    __syncthreads();
    int64_t df = 0, dg = 0;
    // a skipped group starts past every class, so it takes the barriers only
    if (kSpinLanes<NARROW, WD> && spin)
        sweep_phases_spin<NARROW, WD>(P, Rs, replica_lds() + sub * P.stride, sp, n_round,
                                      live ? lane : (1 << 30), 1 << lshift, df, dg);
    else
        sweep_phases<NARROW, WD, true>(P, Rs, replica_lds() + sub * P.stride, sp, n_round,
                                       live ? lane : (1 << 30), 1 << lshift, df, dg);
    // sum over each group: within its wave segment, then across its waves
    const int seg = lshift < 6 ? (1 << lshift) : 64;
    for (int off = seg >> 1; off > 0; off >>= 1) {
        df += __shfl_xor(df, off, 64);
        dg += __shfl_xor(dg, off, 64);
    }
    if (live && (tid & (seg - 1)) == 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&red[2 * sub]), (unsigned long long)df);
        atomicAdd(reinterpret_cast<unsigned long long *>(&red[2 * sub + 1]), (unsigned long long)dg);
    }
    __syncthreads();
    if (live && lane == 0) {
        P.f[slot] += red[2 * sub];
        P.g[slot] += red[2 * sub + 1];
    }
    copy_bytes16(P.states + (size_t)slot0 * P.stride, lds, nsub * P.stride);
}

// One round of one problem with rpb slots per workgroup (ceil(R / rpb)
// workgroups).
template <int NARROW, int WD>
__global__ __launch_bounds__(kMultiBlock, 2) void k_round_sweep_multi(DevProblem P)
{
    extern __shared__ __align__(16) int8_t lds[];
    multi_round_body<NARROW, WD>(P, blockIdx.x * P.rpb, P.rpb, P.lshift, P.spin, lds);
}

// Batched round with rpb slots per workgroup: first_block is the prefix sum
// of the members' workgroup counts, ceil(R / rpb) each.
template <int NARROW, int WD>
__global__ __launch_bounds__(kMultiBlock, 2) void k_batch_sweep_multi(const DevProblem *__restrict__ table,
                                                               const int *__restrict__ first_block, int count,
                                                               int rpb, int lshift, int spin)
{
    extern __shared__ __align__(16) int8_t lds[];
    const int b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    multi_round_body<NARROW, WD>(table[lo], (b - first_block[lo]) * rpb, rpb, lshift, spin, lds);
}

__device__ __forceinline__ bool metropolis(double x, double u)
{
    return x >= 0.0 || u <= exp(x);
}

// The same decision with lu = log(u) taken in advance, so that only a
// comparison remains once x is known.  u is 0 or at least 2^-53, so |ln u|
// < 37; log and exp are good to a few ulp, hence |lu - ln u| < 2^-40 and
// exp(x) is within a relative 2^-40 of e^x.  If x exceeds lu by more than
// 2^-30, e^x > u (1 + 2^-31) and the computed exp(x) is above u: accept;
// below lu by more than 2^-30 likewise reject; in between the expression
// itself decides.  u = 0 gives lu = -inf and acceptance, as u <= exp(x).
__device__ __forceinline__ bool metropolis_pre(double x, double u, double lu)
{
    if (x >= 0.0 || x > lu + 0x1p-30) return true;
    if (x < lu - 0x1p-30) return false;
    return u <= exp(x);
}

// Swap exponent of the pair (left / upper position a, right / lower
// position b): P pairs lie on row `line` with left column k (Eq. 2), beta
// pairs on column `line` with upper row k (Eq. 3).
__device__ __forceinline__ double pair_exponent(const double *beta, const int32_t *p_q, bool dir_beta, int k,
                                                int line, int64_t fa, int64_t ga, int64_t fb, int64_t gb)
{
    if (!dir_beta) {
        const int64_t dpg = ((int64_t)p_q[k + 1] - p_q[k]) * (gb - ga);
        return ldexp(beta[line] * (double)dpg, -12);
    }
    const int64_t ea = fa + (int64_t)p_q[line] * ga;
    const int64_t eb = fb + (int64_t)p_q[line] * gb;
    const double dbeta = beta[k + 1] - beta[k];
    return ldexp(dbeta * (double)(eb - ea), -12);
}

// Uniform of the pair's decision in round n.
__device__ __forceinline__ double pair_uniform(const DevProblem &P, bool dir_beta, int k, int line, int64_t n)
{
    return philox_u53((uint32_t)k, (uint32_t)n, (uint32_t)line, dir_beta ? 2u : 1u, P.key0, P.key1);
}

__device__ __forceinline__ bool pair_accept(const DevProblem &P, const double *beta, const int32_t *p_q,
                                            bool dir_beta, int k, int line, int64_t n, int64_t fa, int64_t ga,
                                            int64_t fb, int64_t gb)
{
    return metropolis(pair_exponent(beta, p_q, dir_beta, k, line, fa, ga, fb, gb),
                      pair_uniform(P, dir_beta, k, line, n));
}

__device__ __forceinline__ void round_schedule(const DevProblem &P, int64_t n, bool &dir_beta, int &first)
{
    first = (n % 2 == 0) ? 1 : 0;
    dir_beta = (P.flags & 1u) ? true : (((n - 1) / 2) % 2 == 1);
}

// One swap step of Algorithm 1 plus bottom-right tracking; one workgroup.
__device__ __forceinline__ void swap_track_body(const DevProblem &P)
{
    __shared__ int improved;
    __shared__ int br_slot;
    const int tid = threadIdx.x;
    const int64_t n = P.hdr[kHdrRounds] + 1;
    bool dir_beta;
    int first;
    round_schedule(P, n, dir_beta, first);
    const int len = dir_beta ? P.I : P.J;
    const int lines = dir_beta ? P.J : P.I;
    const int per = (len - first) / 2;
    for (int w = tid; w < lines * per; w += blockDim.x) {
        const int line = w / per, k = first + 2 * (w - (w / per) * per);
        const int a = dir_beta ? k * P.J + line : line * P.J + k;
        const int b = dir_beta ? a + P.J : a + 1;
        const int sa = P.pos_slot[a], sb = P.pos_slot[b];
        const bool acc = pair_accept(P, P.beta, P.p_q, dir_beta, k, line, n, P.f[sa], P.g[sa], P.f[sb], P.g[sb]);
        const int ci = dir_beta ? line * (P.I - 1) + k : line * (P.J - 1) + k;
        int64_t *att = dir_beta ? P.b_att : P.p_att;
        int64_t *acp = dir_beta ? P.b_acc : P.p_acc;
        att[ci] += 1;
        if (acc) {
            acp[ci] += 1;
            P.pos_slot[a] = sb; P.pos_slot[b] = sa;
            P.slot_pos[sb] = a; P.slot_pos[sa] = b;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int s = P.pos_slot[P.R - 1];
        br_slot = s;
        improved = 0;
        const int64_t sweeps = n * P.mcs;
        const int64_t f = P.f[s], g = P.g[s];
        if (n - 1 < P.trace_cap) { P.trace_f[n - 1] = f; P.trace_g[n - 1] = g; }
        if (g == 0) {
            if (P.has_target && P.hdr[kHdrFirstHit] < 0 && f <= P.f_target) P.hdr[kHdrFirstHit] = sweeps;
            if (f < P.hdr[kHdrBestF]) {
                P.hdr[kHdrBestF] = f;
                P.hdr[kHdrBestSweep] = sweeps;
                improved = 1;
            }
        }
    }
    __syncthreads();
    if (improved) copy_bytes16(P.best_state, P.states + (size_t)br_slot * P.stride, P.stride);
    if (P.hist_n && tid == 0) {
        const int8_t *st = P.states + (size_t)br_slot * P.stride;
        uint32_t bin = 0;
        for (int k = 0; k < P.hist_n; ++k) bin |= (uint32_t)(st[P.hist_rank[k]] > 0) << k;
        P.hist[bin] += 1u;
    }
    __syncthreads();
    if (tid == 0) P.hdr[kHdrRounds] = n;
}

__global__ __launch_bounds__(kSmallBlock) void k_swap_track(DevProblem P) { swap_track_body(P); }

__global__ __launch_bounds__(kSmallBlock) void k_batch_swap(const DevProblem *__restrict__ table)
{
    swap_track_body(table[blockIdx.x]);
}

// ------------------------------------------------ persistent (cooperative)
// Mailbox of grid position p in round n: two 64-bit words written by the
// slot that sits at p, each carrying the round's tag in its low 16 bits so
// either word can be checked on its own:
//   w0 = f << 16 | tag  (f as a 48-bit two's-complement number),
//   w1 = g << 16 | tag  (g as a 48-bit unsigned number).
// The host runs this driver only where |f| < 2^30 and g < 2^47.
// Ring of kRing rounds: positions p and q that pair in round n pair again in
// round n + 4, and no slot can move into p or q while their occupants have
// not finished round n, so round n's entry is read before round n + kRing
// rewrites it.
__device__ __forceinline__ uint64_t mb_tag(int64_t n) { return (uint64_t)((n & 0x7fff) | 0x8000); }

__device__ __forceinline__ uint64_t mb_load(const uint64_t *m)
{
    return __hip_atomic_load(const_cast<uint64_t *>(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool mb_take(uint64_t w0, uint64_t w1, uint64_t tag, int64_t &f, int64_t &g)
{
    if ((w0 & 0xffff) != tag || (w1 & 0xffff) != tag) return false;
    f = (int64_t)w0 >> 16;
    g = (int64_t)(w1 >> 16);
    return true;
}

__device__ __forceinline__ bool mb_wait(const uint64_t *m, uint64_t tag, int64_t &f, int64_t &g, int64_t *hdr)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        if (mb_take(mb_load(m), mb_load(m + 1), tag, f, g)) return true;
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > 200000000ull) {  // 2 s of the 100 MHz clock
            __hip_atomic_store(&hdr[kHdrError], (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// The pairing of grid position pos in round n: k >= 0 when it has a partner,
// then `other` is the partner's position and `left` tells whether pos is the
// left (P pairs) or upper (beta pairs) one.
struct RoundPair {
    bool dir_beta, left;
    int k, line, other;
};

__device__ __forceinline__ RoundPair round_pair(const DevProblem &P, int64_t n, int pos)
{
    RoundPair r;
    int first;
    round_schedule(P, n, r.dir_beta, first);
    const int i = pos / P.J, j = pos - i * P.J;
    const int x = r.dir_beta ? i : j;
    r.line = r.dir_beta ? j : i;
    const int len = r.dir_beta ? P.I : P.J;
    r.k = -1;
    r.left = false;
    r.other = pos;
    if (x >= first && ((x - first) & 1) == 0 && x + 1 < len) { r.k = x; r.left = true; }
    else if (x >= first + 1 && ((x - first) & 1) == 1) { r.k = x - 1; }
    if (r.k >= 0) {
        const int a = r.dir_beta ? r.k * P.J + r.line : r.line * P.J + r.k;
        const int b = r.dir_beta ? a + P.J : a + 1;
        r.other = r.left ? b : a;
    }
    return r;
}

// One block per replica slot; runs n_rounds rounds.  Per round: sweep in
// LDS, post (f, g) in the mailbox of the slot's grid position, read the
// partner position's mailbox, take the pair's decision (both partners draw
// the same Philox number and reach the same answer), move, and, if the slot
// now sits bottom-right, record it.  Best states are kept per slot and
// merged by k_finalize.  The partner's entry is first read while the block
// reduces its energy change (a partner that finished earlier has posted by
// then), and the pair's uniform and its logarithm are computed while that
// read is in flight.
template <int NARROW, int WD>
__device__ __forceinline__ void persistent_body(const DevProblem &P, int slot, int64_t n_rounds, int8_t *lds)
{
    if (!replica_at_zero(lds)) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&P.hdr[kHdrError], kErrLdsBase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    int64_t *red = lds_scratch(lds, P.stride);
    // per-slot state kept by thread 0 in LDS: [0] f, [1] g, [2] best key
    int64_t *st = red + 2 + 2 * (kMaxBlock / 64);
    int *sh = reinterpret_cast<int *>(st + 3);  // [0] position, [1] improved, [2] abort
    // copies of the beta and penalty ladders, read every round
    double *lbeta = reinterpret_cast<double *>(sh + 4);
    int32_t *lpq = reinterpret_cast<int32_t *>(lbeta + P.I);
    const int tid = threadIdx.x;
    for (int i = tid; i < P.I; i += blockDim.x) lbeta[i] = P.beta[i];
    for (int j = tid; j < P.J; j += blockDim.x) lpq[j] = P.p_q[j];
    copy_bytes16(lds, P.states + (size_t)slot * P.stride, P.stride);
    if (tid == 0) {
        st[0] = P.f[slot];
        st[1] = P.g[slot];
        st[2] = INT64_MAX;
        sh[0] = P.slot_pos[slot];
    }
    const int64_t n0 = P.hdr[kHdrRounds];
    const Rsrc Rs = make_rsrc(P);
    __syncthreads();
    for (int64_t rr = 1; rr <= n_rounds; ++rr) {
        const int64_t n = n0 + rr;
        const int pos = __builtin_amdgcn_readfirstlane(sh[0]);
        const SlotParams sp = slot_params(P, pos, lbeta, lpq);
        const RoundPair rp = round_pair(P, n, pos);
        uint64_t *mb = P.mbox + 2 * ((size_t)(n & (kRing - 1)) * P.R);
        uint64_t pw0 = 0, pw1 = 0;
        const bool stamp = P.stage_cap > 0 && n - 1 - P.stage_round0 >= 0 && n - 1 - P.stage_round0 < P.stage_cap;
        uint64_t ts[4] = {0, 0, 0, 0};
        if (stamp && tid == 0) ts[0] = __builtin_amdgcn_s_memrealtime();
        sweep_round<NARROW, WD>(P, Rs, replica_lds(), sp, n, red, [&] {
            if (tid == 0 && rp.k >= 0) {
                pw0 = mb_load(&mb[2 * rp.other]);
                pw1 = mb_load(&mb[2 * rp.other + 1]);
            }
        });
        if (tid == 0) {
            if (stamp) ts[1] = __builtin_amdgcn_s_memrealtime();
            const int64_t f = st[0] + red[0];
            const int64_t g = st[1] + red[1];
            st[0] = f;
            st[1] = g;
            const uint64_t tag = mb_tag(n);
            __hip_atomic_store(&mb[2 * pos], ((uint64_t)f << 16) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&mb[2 * pos + 1], ((uint64_t)g << 16) | tag, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            const bool dir_beta = rp.dir_beta, left = rp.left;
            const int k = rp.k, line = rp.line, other = rp.other;
            int newpos = pos;
            int abort = 0;
            if (k >= 0) {
                const double u = pair_uniform(P, dir_beta, k, line, n);
                const double lu = log(u);
                // keep u and lu ahead of the partner's read instead of sunk behind it
                __asm__ volatile("" ::"v"(u), "v"(lu));
                int64_t fo = 0, go = 0;
                if (!mb_take(pw0, pw1, tag, fo, go) && !mb_wait(&mb[2 * other], tag, fo, go, P.hdr)) abort = 1;
                if (stamp) ts[2] = __builtin_amdgcn_s_memrealtime();
                const int64_t fa = left ? f : fo, ga = left ? g : go;
                const int64_t fb = left ? fo : f, gb = left ? go : g;
                const bool acc =
                    !abort && metropolis_pre(pair_exponent(lbeta, lpq, dir_beta, k, line, fa, ga, fb, gb), u, lu);
                if (left && !abort) {
                    const int ci = dir_beta ? line * (P.I - 1) + k : line * (P.J - 1) + k;
                    __hip_atomic_fetch_add(dir_beta ? &P.b_att[ci] : &P.p_att[ci], (int64_t)1,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (acc)
                        __hip_atomic_fetch_add(dir_beta ? &P.b_acc[ci] : &P.p_acc[ci], (int64_t)1,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (acc) newpos = other;
            }
            int improved = 0;
            if (newpos == P.R - 1 && !abort) {
                const int64_t sweeps = n * P.mcs;
                if (P.hist_n) {
                    const lds8_t *rep = replica_lds();
                    uint32_t bin = 0;
                    for (int k = 0; k < P.hist_n; ++k) bin |= (uint32_t)(rep[P.hist_rank[k]] > 0) << k;
                    __hip_atomic_fetch_add(&P.hist[bin], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (n - 1 < P.trace_cap) { P.trace_f[n - 1] = f; P.trace_g[n - 1] = g; }
                if (g == 0) {
                    if (P.has_target && f <= P.f_target)
                        __hip_atomic_fetch_min(P.hit_min, sweeps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int64_t key = ((f + kKeyOffset) << 32) | (int64_t)(uint32_t)sweeps;
                    if (key < st[2]) {
                        st[2] = key;
                        improved = 1;
                    }
                }
            }
            sh[0] = newpos;
            sh[1] = improved;
            sh[2] = abort;
            if (stamp) {
                ts[3] = __builtin_amdgcn_s_memrealtime();
                if (k < 0) ts[2] = ts[1];
                uint64_t *o = P.stage + ((size_t)(n - 1 - P.stage_round0) * P.R + slot) * 4;
                o[0] = ts[0];
                o[1] = ts[1];
                o[2] = ts[2];
                o[3] = ts[3];
            }
        }
        __syncthreads();
        if (sh[2]) break;
        if (sh[1]) {
            copy_bytes16(P.slot_best + (size_t)slot * P.stride, lds, P.stride);
            __syncthreads();
        }
    }
    copy_bytes16(P.states + (size_t)slot * P.stride, lds, P.stride);
    if (tid == 0) {
        const int pos = sh[0];
        P.f[slot] = st[0];
        P.g[slot] = st[1];
        P.slot_pos[slot] = pos;
        P.pos_slot[pos] = slot;
        P.slot_key[slot] = st[2];
    }
}

// The slot a persistent workgroup serves (the identity unless a test asks
// for another order).
__device__ __forceinline__ int persistent_slot(const DevProblem &P, int b)
{
    return (int)(((int64_t)b * P.slot_mul + P.slot_add) % P.R);
}

template <int NARROW, int WD>
__global__ __launch_bounds__(kMaxBlock, 4) void k_persistent(DevProblem P, int64_t n_rounds)
{
    extern __shared__ __align__(16) int8_t lds[];
    persistent_body<NARROW, WD>(P, persistent_slot(P, blockIdx.x), n_rounds, lds);
}

// Index of the table member whose block range holds block b (first_block is
// the prefix sum of the members' block counts).
__device__ __forceinline__ int member_of(const int *__restrict__ first_block, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Persistent driver over a batch: one cooperative launch runs n_rounds
// rounds of every member of a layout group, block b serving slot
// b - first_block[m] of member m.  Each member's slots exchange through that
// member's own mailboxes, so members never wait for one another.
template <int NARROW, int WD>
__global__ __launch_bounds__(kMaxBlock, 4) void k_batch_persistent(const DevProblem *__restrict__ table,
                                                                 const int *__restrict__ first_block, int count,
                                                                 int64_t n_rounds)
{
    extern __shared__ __align__(16) int8_t lds[];
    const int m = member_of(first_block, count, blockIdx.x);
    persistent_body<NARROW, WD>(table[m], persistent_slot(table[m], blockIdx.x - first_block[m]), n_rounds, lds);
}

// Before a persistent launch: clear the per-slot best keys and the hit word.
__device__ __forceinline__ void scratch_reset_body(const DevProblem &P, int i)
{
    if (i < P.R) P.slot_key[i] = INT64_MAX;
    if (i == 0) P.hit_min[0] = INT64_MAX;
}

__global__ void k_scratch_reset(DevProblem P) { scratch_reset_body(P, blockIdx.x * blockDim.x + threadIdx.x); }

// The same for every member of a batch (one workgroup per member).
__global__ __launch_bounds__(kSmallBlock) void k_batch_scratch_reset(const DevProblem *__restrict__ table)
{
    const DevProblem &P = table[blockIdx.x];
    for (int i = threadIdx.x; i < P.R; i += blockDim.x) scratch_reset_body(P, i);
}

// After a persistent launch: merge the per-slot bests and the first hit into
// the problem's tracking and advance its round count (one workgroup).
__device__ __forceinline__ void finalize_body(const DevProblem &P, int64_t n_rounds)
{
    __shared__ int64_t bk[kSmallBlock];
    __shared__ int bs[kSmallBlock];
    const int tid = threadIdx.x;
    int64_t key = INT64_MAX;
    int who = -1;
    for (int r = tid; r < P.R; r += blockDim.x) {
        const int64_t k = P.slot_key[r];
        if (k < key) { key = k; who = r; }
    }
    bk[tid] = key;
    bs[tid] = who;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off && bk[tid + off] < bk[tid]) { bk[tid] = bk[tid + off]; bs[tid] = bs[tid + off]; }
        __syncthreads();
    }
    __shared__ int take;
    if (tid == 0) {
        take = -1;
        const int64_t best = bk[0];
        if (best != INT64_MAX) {
            const int64_t bf = (best >> 32) - kKeyOffset;
            const int64_t bw = best & 0xffffffffll;
            const int64_t of = P.hdr[kHdrBestF];
            if (of == INT64_MAX || bf < of) {
                P.hdr[kHdrBestF] = bf;
                P.hdr[kHdrBestSweep] = bw;
                take = bs[0];
            }
        }
        const int64_t hm = P.hit_min[0];
        if (hm != INT64_MAX && P.hdr[kHdrFirstHit] < 0) P.hdr[kHdrFirstHit] = hm;
        P.hdr[kHdrRounds] += n_rounds;
    }
    __syncthreads();
    if (take >= 0) copy_bytes16(P.best_state, P.slot_best + (size_t)take * P.stride, P.stride);
}

__global__ __launch_bounds__(kSmallBlock) void k_finalize(DevProblem P, int64_t n_rounds) { finalize_body(P, n_rounds); }

// The same for every member of a batch (one workgroup per member).
__global__ __launch_bounds__(kSmallBlock) void k_batch_finalize(const DevProblem *__restrict__ table, int64_t n_rounds)
{
    finalize_body(table[blockIdx.x], n_rounds);
}

// ------------------------------------------------------ bit-packed layout
// For replicas too large for an int8 copy in LDS.  A workgroup holds
// kBitSlots replicas as bits, interleaved by word (uint32 4 w + r is word w
// of replica r), so one 16-byte LDS read returns a neighbour's word of all
// of them and every structure load serves kBitSlots updates.  With b_k the
// neighbour's bit (s_k = 2 b_k - 1), sum_k J_k s_k = -sum_k J_k +
// 2 sum_k J_k b_k; h0 = b - sum_k J_k is precomputed, and J_k b_k is one
// 24-bit multiply-add (couplings of this layout stay below 2^23).
//
// A class starts on a 32-bit boundary of the bit numbering and lane l of a
// wave takes quad l (+ multiples of the block size) of the class, so the 8
// quads of one word belong to 8 consecutive lanes of one wave: they OR
// their new nibbles together across lanes and one of them stores the word.
// Every lane of a wave that has any quad left runs the update (lanes past
// the class end with no live spin), so the lanes of a word are converged.

// OR of x over the aligned group of 8 lanes containing this lane, in the
// group's last lane (DPP: quad_perm swaps, then a shift by 4 within a row).
// a * b + c on 24-bit operands as one instruction (the compiler otherwise
// pairs the products into three-input adds: three instructions per two
// products instead of two)
__device__ __forceinline__ int mad24(int a, int b, int c)
{
    int r;
    __asm__("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Bit (pos mod 32) of w in one instruction: v_bfe_u32 reads only the low 5
// bits of its offset operand, so positions stored as 512 word + bit need no
// mask first (the compiler's bit-field extract masks the offset itself).
__device__ __forceinline__ uint32_t bit_of(uint32_t w, int pos)
{
    uint32_t r;
    __asm__("v_bfe_u32 %0, %1, %2, 1" : "=v"(r) : "v"(w), "v"(pos));
    return r;
}

__device__ __forceinline__ uint32_t or8_last(uint32_t x)
{
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    return x;
}

// q: the lane's quad, which may lie past the class end (q1); its structure
// and spins are read at min(q, q1 - 1) and then it has no live spin.
template <int WD, bool TRACK>
__device__ __forceinline__ void bits_update_quad(const DevProblem &P, const Rsrc &Rs, int q,
                                                 int q1, int c, unsigned live, uint32_t t,
                                                 const SlotParams (&sp)[kBitSlots],
                                                 int (&dfa)[kBitSlots], int (&dga)[kBitSlots])
{
    const int qs = min(q, q1 - 1);
    const int voff = qs * 16;
    const int row = P.n_pad * 4;
    int acc[4][kBitSlots], cs[4][kBitSlots];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < kBitSlots; ++r) { acc[j][r] = 0; cs[j][r] = 0; }
#pragma unroll
    for (int k = 0; k < WD; ++k) {
        const v4i pk = bload(Rs.a, voff, k * row);
        const v4i jk = bload(Rs.b, voff, k * row);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // 512 word + bit: the word group's LDS byte address is pos >> 5
            const int pos = pk[j];
            const u4v nw = *(const lds_u4_t *)(uintptr_t)(uint32_t)(pos >> 5);
            const uint32_t w4[4] = {nw.x, nw.y, nw.z, nw.w};
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r)
                acc[j][r] = mad24((int)bit_of(w4[r], pos), jk[j], acc[j][r]);
        }
    }
    const v4i c0 = bload(Rs.ch, voff, 0);
    const v4i c1 = bload(Rs.ch, voff, row);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // a missing copy neighbour reads a bit of the always-zero word group
        // past the last class; row 0 carries the count kc of present copy
        // neighbours in bits 29..30, so the copy sum is 2 (b0 + b1) - kc
        const int p0 = c0[j], p1 = c1[j];
        const u4v n0 = *(const lds_u4_t *)(uintptr_t)__builtin_amdgcn_ubfe((uint32_t)p0, 5, 18);
        const u4v n1 = *(const lds_u4_t *)(uintptr_t)(uint32_t)(p1 >> 5);
        const uint32_t a4[4] = {n0.x, n0.y, n0.z, n0.w}, b4[4] = {n1.x, n1.y, n1.z, n1.w};
        const int nkc = -(int)((uint32_t)p0 >> 29);
#pragma unroll
        for (int r = 0; r < kBitSlots; ++r) {
            const int b0 = (int)bit_of(a4[r], p0);
            const int b1 = (int)bit_of(b4[r], p1);
            cs[j][r] = 2 * (b0 + b1) + nkc;
        }
    }
    const v4i h0 = bload(Rs.bias, voff, 0);
    const int bpos = qs * 4 - P.cls_start[c] + P.bit_start[c];
    const int wq = bpos >> 5, off = bpos & 31;
    uint32_t o4[4] = {0u, 0u, 0u, 0u};
    if (TRACK) {
        const u4v ow = *(const lds_u4_t *)(uintptr_t)(uint32_t)(wq * 16);
        o4[0] = ow.x; o4[1] = ow.y; o4[2] = ow.z; o4[3] = ow.w;
    }
    uint32_t nw4[kBitSlots];
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) {
        uint32_t u[4] = {(uint32_t)q, t, sp[r].pos, 0u};
        philox10(u[0], u[1], u[2], u[3], P.key0, P.key1);
        int hp[4], hh[4];
        float d[4];
        bool amb_any = false;  // dead lanes may set it too: the exact path skips them
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hp[j] = h0[j] + 2 * acc[j][r];
            hh[j] = mad24(cs[j][r], sp[r].twoP, hp[j]);  // |2 P_q| < 2^23 in this layout
            d[j] = heat_bath_margin(hh[j], sp[r].cb, u[j]);
            amb_any |= margin_ambiguous(d[j]);
        }
        // bit j set when spin j goes up: the sign bytes masked to 1, 2, 4, 8
        // and summed
        uint32_t up = __builtin_amdgcn_sad_u8(sign_bytes4(d) & 0x08040201u, 0u, 0u);
        if (__builtin_expect(amb_any, 0)) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (margin_ambiguous(d[j]) && ((live >> j) & 1u)) {
                    const uint32_t bit = heat_bath_exact(sp[r].beta, hh[j], u[j]) > 0 ? 1u : 0u;
                    up = (up & ~(1u << j)) | (bit << j);
                }
            }
        }
        up &= live;
        if (TRACK) {
            const uint32_t old = (o4[r] >> off) & 15u;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // s_new - s_old = 2 (bit_new - bit_old); dead spins change nothing.
                // df = -(s_new - s_old) hp, dg = -2 (s_new - s_old) cs
                const int db = (((live >> j) & 1u) ? ((int)((up >> j) & 1u) - (int)((old >> j) & 1u)) : 0);
                dfa[r] -= 2 * db * hp[j];
                dga[r] -= 4 * db * cs[j][r];
            }
        }
        nw4[r] = up << off;  // 0 for a lane past the class end
    }
    // the group's word, from its first quad; a group wholly past the class
    // end owns no word and stores nothing
    const int qg = q - (int)(threadIdx.x & 7);
    const int wg = (qg * 4 - P.cls_start[c] + P.bit_start[c]) >> 5;
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) {
        const uint32_t word = or8_last(nw4[r]);
        if ((threadIdx.x & 7) == 7 && qg < q1) *(lds32_t *)(uintptr_t)(uint32_t)(16 * wg + 4 * r) = word;
    }
}

// f and g of the kBitSlots replicas from scratch, over the live spins of quad
// q of class c (ef accumulates 2 f, eg accumulates g / 2).  With b_i the
// spin's bit and A_i = sum_k J_k b_k over its problem neighbours,
// sum_k J_k s_k = h0_i + 2 A_i - b_i (h0 = b - sum_k J_k), so
// 2 f = -sum_i s_i (h0_i + 2 A_i + b_i); a copy edge whose ends differ
// adds 4 to g, seen from both ends.
template <int WD>
__device__ __forceinline__ void bits_energy_quad(const DevProblem &P, const Rsrc &Rs,
                                                 const __amdgpu_buffer_rsrc_t &rb, int q, int c,
                                                 unsigned live, int64_t (&ef)[kBitSlots], int (&eg)[kBitSlots])
{
    const int voff = q * 16;
    const int row = P.n_pad * 4;
    int acc[4][kBitSlots];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < kBitSlots; ++r) acc[j][r] = 0;
#pragma unroll
    for (int k = 0; k < WD; ++k) {
        const v4i pk = bload(Rs.a, voff, k * row);
        const v4i jk = bload(Rs.b, voff, k * row);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pos = pk[j];
            const u4v nw = *(const lds_u4_t *)(uintptr_t)(uint32_t)(pos >> 5);
            const uint32_t w4[4] = {nw.x, nw.y, nw.z, nw.w};
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r)
                acc[j][r] = mad24((int)bit_of(w4[r], pos), jk[j], acc[j][r]);
        }
    }
    const v4i c0 = bload(Rs.ch, voff, 0);
    const v4i c1 = bload(Rs.ch, voff, row);
    const v4i h0 = bload(Rs.bias, voff, 0);
    const v4i bb = bload(rb, voff, 0);
    const int bpos = q * 4 - P.cls_start[c] + P.bit_start[c];
    const int wq = bpos >> 5, off = bpos & 31;
    const u4v ow = *(const lds_u4_t *)(uintptr_t)(uint32_t)(wq * 16);
    const uint32_t o4[4] = {ow.x, ow.y, ow.z, ow.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((live >> j) & 1u)) continue;
        const int p0 = c0[j], p1 = c1[j];
        const int kc = (int)((uint32_t)p0 >> 29);  // copy neighbours present: row 0 first
        const u4v n0 = *(const lds_u4_t *)(uintptr_t)__builtin_amdgcn_ubfe((uint32_t)p0, 5, 18);
        const u4v n1 = *(const lds_u4_t *)(uintptr_t)(uint32_t)(p1 >> 5);
        const uint32_t a4[4] = {n0.x, n0.y, n0.z, n0.w}, b4[4] = {n1.x, n1.y, n1.z, n1.w};
#pragma unroll
        for (int r = 0; r < kBitSlots; ++r) {
            const uint32_t bi = (o4[r] >> (off + j)) & 1u;
            const int64_t t = (int64_t)(h0[j] + 2 * acc[j][r]) + bb[j];
            ef[r] += bi ? -t : t;
            const uint32_t d0 = (bi ^ bit_of(a4[r], p0)) & (kc >= 1 ? 1u : 0u);
            const uint32_t d1 = (bi ^ bit_of(b4[r], p1)) & (kc >= 2 ? 1u : 0u);
            eg[r] += (int)(d0 + d1);
        }
    }
}

// ------------------------------------------- bit-packed layout, pair form
// Each 32-bit word holds the same 16 spins of two replicas, one per 16-bit
// half, so one shift and mask read a neighbour's spin in both and one packed
// 16-bit multiply-add (v_pk_mad_u16) adds its coupling to both replicas'
// sums.  The sums 2 sum_k J_k b_k stay below 2^15 in magnitude (the host's
// condition for this form), so the halves' arithmetic modulo 2^16 is exact
// once each half is read back sign-extended.

// acc + j2 * s in each 16-bit half, as one instruction (written as a vector
// of two 16-bit numbers the compiler pairs the words of a replica group into
// 64-bit values and spills them)
__device__ __forceinline__ uint32_t pair_mad(uint32_t j2, uint32_t s, uint32_t acc)
{
    uint32_t r;
    __asm__("v_pk_mad_u16 %0, %1, %2, %3" : "=v"(r) : "v"(j2), "v"(s), "v"(acc));
    return r;
}

// The spin at position pos in both replicas of word w, one bit per half (the
// shift reads only the low 5 bits of pos, which the compiler drops the mask
// for).
__device__ __forceinline__ uint32_t pair_bits(uint32_t w, int pos) { return (w >> (pos & 31)) & 0x00010001u; }

// Half h (0: low) of a pair of 16-bit sums, sign-extended.
__device__ __forceinline__ int pair_half(uint32_t acc, int h)
{
    return h ? ((int)acc >> 16) : (int)(short)(acc & 0xffffu);
}

// OR of x over the aligned group of 4 lanes containing this lane, in all 4.
__device__ __forceinline__ uint32_t or4_all(uint32_t x)
{
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    return x;
}

// bits_update_quad for the pair form.  The 4 lanes of a half word (16 spins)
// are an aligned lane quad; they OR their nibbles across lanes and the last
// of them stores the half's two words (one per replica pair) as one 8-byte
// write.
template <int WD, bool TRACK>
__device__ __forceinline__ void pair_update_quad(const DevProblem &P, const Rsrc &Rs, int q,
                                                 int q1, int c, unsigned live, uint32_t t,
                                                 const SlotParams (&sp)[kBitSlots],
                                                 int (&dfa)[kBitSlots], int (&dga)[kBitSlots])
{
    const int qs = min(q, q1 - 1);
    const int voff = qs * 16;
    const int row = P.n_pad * 4;
    uint32_t acc[4][2];  // [spin][replica pair]: 2 sum_k J_k b_k, one replica per half
#pragma unroll
    for (int j = 0; j < 4; ++j) { acc[j][0] = 0u; acc[j][1] = 0u; }
#pragma unroll
    for (int k = 0; k < WD; ++k) {
        const v4i pk = bload(Rs.a, voff, k * row);
        const v4i jk = bload(Rs.b, voff, k * row);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pos = pk[j];
            const u2v nw = *(const lds_u2_t *)(uintptr_t)(uint32_t)(pos >> 5);
            acc[j][0] = pair_mad((uint32_t)jk[j], pair_bits(nw.x, pos), acc[j][0]);
            acc[j][1] = pair_mad((uint32_t)jk[j], pair_bits(nw.y, pos), acc[j][1]);
        }
    }
    const v4i c0 = bload(Rs.ch, voff, 0);
    const v4i c1 = bload(Rs.ch, voff, row);
    int cs[4][kBitSlots];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // as in the plain form: the copy sum is 2 (b0 + b1) - kc, the two
        // present-neighbour bits counted per half (at most 2 each)
        const int p0 = c0[j], p1 = c1[j];
        const u2v n0 = *(const lds_u2_t *)(uintptr_t)__builtin_amdgcn_ubfe((uint32_t)p0, 5, 18);
        const u2v n1 = *(const lds_u2_t *)(uintptr_t)(uint32_t)(p1 >> 5);
        const int nkc = -(int)((uint32_t)p0 >> 29);
        const uint32_t ca = pair_bits(n0.x, p0) + pair_bits(n1.x, p1);
        const uint32_t cb = pair_bits(n0.y, p0) + pair_bits(n1.y, p1);
        cs[j][0] = 2 * (int)(ca & 0xffffu) + nkc;
        cs[j][1] = 2 * (int)(ca >> 16) + nkc;
        cs[j][2] = 2 * (int)(cb & 0xffffu) + nkc;
        cs[j][3] = 2 * (int)(cb >> 16) + nkc;
    }
    const v4i h0 = bload(Rs.bias, voff, 0);
    const int bpos = qs * 4 - P.cls_start[c] + P.bit_start[c];
    const int b15 = bpos & 15;
    uint32_t o2[2] = {0u, 0u};
    if (TRACK) {
        const u2v ow = *(const lds_u2_t *)(uintptr_t)(uint32_t)(bpos >> 1 & ~7);
        o2[0] = ow.x;
        o2[1] = ow.y;
    }
    uint32_t nw2[2] = {0u, 0u};
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) {
        uint32_t u[4] = {(uint32_t)q, t, sp[r].pos, 0u};
        philox10(u[0], u[1], u[2], u[3], P.key0, P.key1);
        int hp[4], hh[4];
        float d[4];
        bool amb_any = false;  // dead lanes may set it too: the exact path skips them
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hp[j] = h0[j] + pair_half(acc[j][r >> 1], r & 1);
            hh[j] = mad24(cs[j][r], sp[r].twoP, hp[j]);  // |2 P_q| < 2^23 in this layout
            d[j] = heat_bath_margin(hh[j], sp[r].cb, u[j]);
            amb_any |= margin_ambiguous(d[j]);
        }
        uint32_t up = __builtin_amdgcn_sad_u8(sign_bytes4(d) & 0x08040201u, 0u, 0u);
        if (__builtin_expect(amb_any, 0)) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (margin_ambiguous(d[j]) && ((live >> j) & 1u)) {
                    const uint32_t bit = heat_bath_exact(sp[r].beta, hh[j], u[j]) > 0 ? 1u : 0u;
                    up = (up & ~(1u << j)) | (bit << j);
                }
            }
        }
        up &= live;
        const int sh = b15 + 16 * (r & 1);
        if (TRACK) {
            const uint32_t old = (o2[r >> 1] >> sh) & 15u;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int db = (((live >> j) & 1u) ? ((int)((up >> j) & 1u) - (int)((old >> j) & 1u)) : 0);
                dfa[r] -= 2 * db * hp[j];
                dga[r] -= 4 * db * cs[j][r];
            }
        }
        nw2[r >> 1] |= up << sh;  // 0 for a lane past the class end
    }
    // the half's two words, from its first quad; a half wholly past the class
    // end stores nothing (its words are class padding and stay zero)
    const int qh = q - (int)(threadIdx.x & 3);
    const uint32_t w0 = or4_all(nw2[0]), w1 = or4_all(nw2[1]);
    if ((threadIdx.x & 3) == 3 && qh < q1) {
        const int bh = qh * 4 - P.cls_start[c] + P.bit_start[c];  // a multiple of 16
        *(lds_u2_t *)(uintptr_t)(uint32_t)(bh >> 1) = u2v{w0, w1};
    }
}

// bits_energy_quad for the pair form (acc holds 2 A_i per half).
template <int WD>
__device__ __forceinline__ void pair_energy_quad(const DevProblem &P, const Rsrc &Rs,
                                                 const __amdgpu_buffer_rsrc_t &rb, int q, int c,
                                                 unsigned live, int64_t (&ef)[kBitSlots], int (&eg)[kBitSlots])
{
    const int voff = q * 16;
    const int row = P.n_pad * 4;
    uint32_t acc[4][2];
#pragma unroll
    for (int j = 0; j < 4; ++j) { acc[j][0] = 0u; acc[j][1] = 0u; }
#pragma unroll
    for (int k = 0; k < WD; ++k) {
        const v4i pk = bload(Rs.a, voff, k * row);
        const v4i jk = bload(Rs.b, voff, k * row);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pos = pk[j];
            const u2v nw = *(const lds_u2_t *)(uintptr_t)(uint32_t)(pos >> 5);
            acc[j][0] = pair_mad((uint32_t)jk[j], pair_bits(nw.x, pos), acc[j][0]);
            acc[j][1] = pair_mad((uint32_t)jk[j], pair_bits(nw.y, pos), acc[j][1]);
        }
    }
    const v4i c0 = bload(Rs.ch, voff, 0);
    const v4i c1 = bload(Rs.ch, voff, row);
    const v4i h0 = bload(Rs.bias, voff, 0);
    const v4i bb = bload(rb, voff, 0);
    const int bpos = q * 4 - P.cls_start[c] + P.bit_start[c];
    const u2v ow = *(const lds_u2_t *)(uintptr_t)(uint32_t)(bpos >> 1 & ~7);
    const uint32_t o2[2] = {ow.x, ow.y};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((live >> j) & 1u)) continue;
        const int p0 = c0[j], p1 = c1[j];
        const int kc = (int)((uint32_t)p0 >> 29);  // copy neighbours present: row 0 first
        const u2v n0 = *(const lds_u2_t *)(uintptr_t)__builtin_amdgcn_ubfe((uint32_t)p0, 5, 18);
        const u2v n1 = *(const lds_u2_t *)(uintptr_t)(uint32_t)(p1 >> 5);
        const uint32_t a2[2] = {n0.x, n0.y}, b2[2] = {n1.x, n1.y};
#pragma unroll
        for (int r = 0; r < kBitSlots; ++r) {
            const int up16 = 16 * (r & 1);
            const uint32_t bi = (o2[r >> 1] >> ((bpos & 15) + up16 + j)) & 1u;
            const int64_t t = (int64_t)(h0[j] + pair_half(acc[j][r >> 1], r & 1)) + bb[j];
            ef[r] += bi ? -t : t;
            const uint32_t d0 = (bi ^ bit_of(a2[r >> 1], p0 + up16)) & (kc >= 1 ? 1u : 0u);
            const uint32_t d1 = (bi ^ bit_of(b2[r >> 1], p1 + up16)) & (kc >= 2 ? 1u : 0u);
            eg[r] += (int)(d0 + d1);
        }
    }
}

// The int8 copy of slot's replica from the first spin of class c on (4-byte
// aligned: rows are 16-byte multiples, classes start on quads).
__device__ __forceinline__ int8_t *slot_row(const DevProblem &P, int slot, int c)
{
    return P.states + (size_t)slot * P.stride + P.cls_start[c];
}

// Bits (1 = spin +1) of the class-local spins k0 .. k0 + N - 1 (k0 and N
// multiples of 4) of a class's int8 row st, 4 spins per load; a load starts
// only below live, so it stays within the class's quads, and spins from live
// on (class padding, 0 in the int8 copy) read as 0.
template <int N>
__device__ __forceinline__ uint32_t run_bits(const int8_t *st, int k0, int live)
{
    uint32_t d[N / 4];
#pragma unroll
    for (int m = 0; m < N / 4; ++m) d[m] = k0 + 4 * m < live ? *(const uint32_t *)(st + k0 + 4 * m) : 0u;
    uint32_t bits = 0;
#pragma unroll
    for (int m = 0; m < N / 4; ++m) {
        // bit 8 j set where byte j is +1 (0x01; -1 is 0xff, padding 0)
        const uint32_t one = d[m] & ~(d[m] >> 7) & 0x01010101u;
        bits |= ((one | one >> 7 | one >> 14 | one >> 21) & 15u) << (4 * m);
    }
    return bits;
}

// The inverse of run_bits: spins below live get +1 (bit set) or -1, the
// bytes of class padding in the last 4-byte store stay 0.
template <int N>
__device__ __forceinline__ void run_store(int8_t *st, int k0, int live, uint32_t bits)
{
#pragma unroll
    for (int m = 0; m < N / 4; ++m) {
        const int rem = live - (k0 + 4 * m);
        if (rem <= 0) continue;
        const uint32_t nib = (bits >> (4 * m)) & 15u;
        const uint32_t set = (nib & 1u) | (nib & 2u) << 7 | (nib & 4u) << 14 | (nib & 8u) << 21;
        uint32_t word = 0xffffffffu ^ (set * 0xfeu);  // 0x01 where set, 0xff elsewhere
        if (rem < 4) word &= (1u << (8 * rem)) - 1u;
        *(uint32_t *)(st + k0 + 4 * m) = word;
    }
}

// One round of up to kBitSlots slots (slot0 ..): unpack the int8 states into
// LDS bits, mcs sweeps, pack them back.  TRACK: f and g follow every update
// exactly (cheap for few sweeps per round); otherwise they are recomputed
// from the final states of the round (cheaper from about 4 sweeps on).
template <int WD, bool TRACK, bool PAIR>
__device__ __forceinline__ void round_sweep_bits_body(const DevProblem &P, int slot0, int8_t *lds)
{
    // the replicas' words sit at LDS byte 0 (the update addresses them there)
    if (!replica_at_zero(lds)) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&P.hdr[kHdrError], kErrLdsBase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // the form is a template argument (one sweep loop per kernel schedules
    // far better than both behind a branch); the host launches the one that
    // matches the problem's structure
    if (P.pair16 != (PAIR ? 1 : 0)) {
        if (threadIdx.x == 0)
            __hip_atomic_store(&P.hdr[kHdrError], kErrBitsForm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    uint32_t *W = reinterpret_cast<uint32_t *>(lds);
    // words of the replicas, one always-zero word group, then int64 scratch
    int64_t *red = reinterpret_cast<int64_t *>(lds + (size_t)(P.n_words + 1) * 16);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ns = min(kBitSlots, P.R - slot0);
    // unpack: word i of group w from the spins whose bits it holds (the extra
    // word group w = n_words holds no spin and stays zero); bit x of the word
    // is spin bit 32 w + x of replica i & 3 (plain form) or spin bit
    // 32 w + 16 ((i >> 1) & 1) + (x & 15) of replica 2 (i & 1) + (x >> 4)
    // (pair form)
    for (int i = tid; i < (P.n_words + 1) * kBitSlots; i += nthr) {
        const int w = i >> 2;
        uint32_t bits = 0;
        if (w < P.n_words) {
            int c = 0;
            while (c + 1 < P.n_colors && P.bit_start[c + 1] <= 32 * w) ++c;
            const int live = P.cls_live[c] - P.cls_start[c];
            const int k0 = 32 * w - P.bit_start[c];  // class-local spin of bit 0 of the group
            if constexpr (PAIR) {
                const int r = 2 * (i & 1), kh = k0 + 16 * ((i >> 1) & 1);
                if (r < ns) bits = run_bits<16>(slot_row(P, slot0 + r, c), kh, live);
                if (r + 1 < ns) bits |= run_bits<16>(slot_row(P, slot0 + r + 1, c), kh, live) << 16;
            } else {
                const int r = i & 3;
                if (r < ns) bits = run_bits<32>(slot_row(P, slot0 + r, c), k0, live);
            }
        }
        W[i] = bits;
    }
    SlotParams sp[kBitSlots];
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) sp[r] = slot_params(P, r < ns ? P.slot_pos[slot0 + r] : 0, P.beta, P.p_q);
    const Rsrc Rs = make_rsrc(P);
    const int64_t n_round = P.hdr[kHdrRounds] + 1;
    __syncthreads();
    int64_t df[kBitSlots], dg[kBitSlots];
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) { df[r] = 0; dg[r] = 0; }
    for (int k = 0; k < P.mcs; ++k) {
        const uint32_t t = (uint32_t)((n_round - 1) * P.mcs + k);
        for (int c = 0; c < P.n_colors; ++c) {
            const int q0 = P.cls_start[c] >> 2, q1 = P.cls_start[c + 1] >> 2;
            const int live_end = P.cls_live[c];
            int dfa[kBitSlots], dga[kBitSlots];
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r) { dfa[r] = 0; dga[r] = 0; }
            // a wave runs while any of its lanes has a quad; lanes past the
            // class end update their (clamped) quad with no live spin
            const int wave0 = tid & ~63;
            for (int base = q0; base + wave0 < q1; base += nthr) {
                const int q = base + tid;
                const int rem = q < q1 ? live_end - q * 4 : 0;
                const unsigned live = rem >= 4 ? 15u : rem <= 0 ? 0u : ((1u << rem) - 1u);
                if constexpr (PAIR) pair_update_quad<WD, TRACK>(P, Rs, q, q1, c, live, t, sp, dfa, dga);
                else bits_update_quad<WD, TRACK>(P, Rs, q, q1, c, live, t, sp, dfa, dga);
            }
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r) { df[r] += dfa[r]; dg[r] += dga[r]; }
            __syncthreads();
        }
    }
    if (!TRACK) {
        // f and g of the final states: 2 f into df, g / 2 into dg
        const __amdgpu_buffer_rsrc_t rb = rsrc(P.bias, P.n_pad * 4);
        for (int c = 0; c < P.n_colors; ++c) {
            const int q0 = P.cls_start[c] >> 2, q1 = P.cls_start[c + 1] >> 2;
            const int live_end = P.cls_live[c];
            int eg[kBitSlots];
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r) eg[r] = 0;
            for (int q = q0 + tid; q < q1; q += nthr) {
                const int rem = live_end - q * 4;
                const unsigned live = rem >= 4 ? 15u : rem <= 0 ? 0u : ((1u << rem) - 1u);
                if constexpr (PAIR) pair_energy_quad<WD>(P, Rs, rb, q, c, live, df, eg);
                else bits_energy_quad<WD>(P, Rs, rb, q, c, live, df, eg);
            }
#pragma unroll
            for (int r = 0; r < kBitSlots; ++r) dg[r] += eg[r];
        }
    }
    const int wave = tid >> 6, nw = nthr >> 6;
#pragma unroll
    for (int r = 0; r < kBitSlots; ++r) {
        const int64_t a = wave_sum64(df[r]), b = wave_sum64(dg[r]);
        if ((tid & 63) == 0) { red[2 * (wave * kBitSlots + r)] = a; red[2 * (wave * kBitSlots + r) + 1] = b; }
    }
    __syncthreads();
    if (tid < ns) {
        int64_t a = 0, b = 0;
        for (int w = 0; w < nw; ++w) { a += red[2 * (w * kBitSlots + tid)]; b += red[2 * (w * kBitSlots + tid) + 1]; }
        if (TRACK) {
            P.f[slot0 + tid] += a;
            P.g[slot0 + tid] += b;
        } else {
            P.f[slot0 + tid] = a / 2;
            P.g[slot0 + tid] = 2 * b;
        }
    }
    // pack back: live spins only (class padding stays 0 in the int8 copy)
    for (int i = tid; i < P.n_words * kBitSlots; i += nthr) {
        const int w = i >> 2;
        int c = 0;
        while (c + 1 < P.n_colors && P.bit_start[c + 1] <= 32 * w) ++c;
        const int live = P.cls_live[c] - P.cls_start[c];
        const int k0 = 32 * w - P.bit_start[c];
        const uint32_t bits = W[i];
        if constexpr (PAIR) {
            const int r = 2 * (i & 1), kh = k0 + 16 * ((i >> 1) & 1);
            if (r < ns) run_store<16>(slot_row(P, slot0 + r, c), kh, live, bits & 0xffffu);
            if (r + 1 < ns) run_store<16>(slot_row(P, slot0 + r + 1, c), kh, live, bits >> 16);
        } else {
            const int r = i & 3;
            if (r < ns) run_store<32>(slot_row(P, slot0 + r, c), k0, live, bits);
        }
    }
}

template <int WD, bool TRACK, bool PAIR>
__global__ __launch_bounds__(TRACK ? kBitsBlock : kBitsBlockScratch) void k_round_sweep_bits(DevProblem P)
{
    extern __shared__ __align__(16) int8_t lds[];
    round_sweep_bits_body<WD, TRACK, PAIR>(P, blockIdx.x * kBitSlots, lds);
}

template <int WD, bool TRACK, bool PAIR>
__global__ __launch_bounds__(TRACK ? kBitsBlock : kBitsBlockScratch) void k_batch_sweep_bits(
    const DevProblem *__restrict__ table,
                                                              const int *__restrict__ first_block, int count)
{
    extern __shared__ __align__(16) int8_t lds[];
    const int b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    round_sweep_bits_body<WD, TRACK, PAIR>(table[lo], (b - first_block[lo]) * kBitSlots, lds);
}

// ---------------------------------------------------- initial states, f, g
// Initial spin v at position p when the caller gives none: Philox counter
// (v >> 2, 0, p, 3), output word v & 3, +1 iff its top bit is set.
__global__ void k_init_states(DevProblem P)
{
    const int slot = blockIdx.y;
    int8_t *s = P.states + (size_t)slot * P.stride;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < P.stride; r += gridDim.x * blockDim.x) {
        int8_t v = 0;
        if (r < P.n_pad) {
            const int o = P.orig[r];
            if (o >= 0) {
                uint32_t x0 = (uint32_t)o >> 2, x1 = 0u, x2 = (uint32_t)slot, x3 = 3u;
                philox10(x0, x1, x2, x3, P.key0, P.key1);
                const uint32_t w[4] = {x0, x1, x2, x3};
                v = (w[o & 3] >> 31) ? 1 : -1;
            }
        }
        s[r] = v;
    }
}

// f = -sum_{i<j} J s_i s_j - sum b s and g (sum_copy (s_a - s_b)^2, or the
// general constraints' g0 - sum_i s_i (2 kh_i + sum_j Kh_ij s_j)) of every
// slot, from scratch (one workgroup per slot).
__global__ __launch_bounds__(kSmallBlock) void k_energy(DevProblem P)
{
    __shared__ int64_t red[kSmallBlock / 64][2];
    const int slot = blockIdx.x;
    const int8_t *s = P.states + (size_t)slot * P.stride;
    int64_t f2 = 0, g2 = 0;
    for (int r = threadIdx.x; r < P.n_pad; r += blockDim.x) {
        const int si = s[r];
        if (si == 0) continue;
        int64_t hp = 0;
        int ca, cb;
        if (P.narrow) {
            for (int k2 = 0; k2 < P.wd / 2; ++k2) {
                const uint32_t ia = P.nbi[(size_t)k2 * P.n_pad + r];
                const uint32_t jb = P.nbj[(size_t)k2 * P.n_pad + r];
                hp += (int64_t)(int16_t)(jb & 0xffff) * s[ia & 0xffff];
                hp += (int64_t)(int16_t)(jb >> 16) * s[ia >> 16];
            }
            const uint32_t c = P.gen ? 0u : P.chp[r];
            ca = P.gen ? P.n_pad : (int)(c & 0xffff);
            cb = P.gen ? P.n_pad : (int)(c >> 16);
        } else {
            for (int k = 0; k < P.wd; ++k)
                hp += (int64_t)P.nb_J[(size_t)k * P.n_pad + r] * s[P.nb_idx[(size_t)k * P.n_pad + r]];
            ca = P.gen ? P.n_pad : P.ch_idx[r];
            cb = P.gen ? P.n_pad : P.ch_idx[P.n_pad + r];
        }
        f2 -= si * hp + 2 * (int64_t)P.bias[r] * si;
        if (P.gen) {
            int64_t c = 2 * (int64_t)P.kh[r];
            for (int k = 0; k < P.wcg; ++k)
                c += (int64_t)P.cn_w[(size_t)k * P.n_pad + r] * s[P.cn_idx[(size_t)k * P.n_pad + r]];
            g2 -= 2 * si * c;
        } else {
            if (ca != P.n_pad) { const int d = si - s[ca]; g2 += d * d; }
            if (cb != P.n_pad) { const int d = si - s[cb]; g2 += d * d; }
        }
    }
    const int64_t a = wave_sum64(f2), b = wave_sum64(g2);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[wave][0] = a; red[wave][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t fa = 0, ga = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { fa += red[w][0]; ga += red[w][1]; }
        P.f[slot] = fa / 2;
        P.g[slot] = ga / 2 + (P.gen ? P.g0 : 0);
    }
}

// ------------------------------------------------- readback into device buffers
// Status words of every batch member (rounds done, first hit, best f, best
// sweep), in the caller's member order.
__global__ void k_batch_status(const DevProblem *__restrict__ table, int count, const int32_t *__restrict__ order,
                               int64_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t *h = table[i].hdr;
    int64_t *o = out + 4 * (size_t)order[i];
    o[0] = h[kHdrRounds];
    o[1] = h[kHdrFirstHit];
    o[2] = h[kHdrBestF];
    o[3] = h[kHdrBestSweep];
}

__global__ void k_gather_energies(DevProblem P, int64_t *f, int64_t *g)
{
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= P.R) return;
    const int slot = P.pos_slot[pos];
    if (f) f[pos] = P.f[slot];
    if (g) g[pos] = P.g[slot];
}

// out[pos][orig(r)] = spin r of the slot at pos; blockIdx.y strides over positions
__global__ void k_gather_states(DevProblem P, int n, int8_t *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.n_pad) return;
    const int o = P.orig[r];
    if (o < 0) return;
    for (int pos = blockIdx.y; pos < P.R; pos += gridDim.y)
        out[(size_t)pos * n + o] = P.states[(size_t)P.pos_slot[pos] * P.stride + r];
}

__global__ void k_gather_best(DevProblem P, int8_t *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.n_pad) return;
    const int o = P.orig[r];
    if (o >= 0) out[o] = P.best_state[r];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_batch_status(const DevProblem *table, int count, const int32_t *order, int64_t *out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_status, dim3((count + 255) / 256), dim3(256), 0, s, table, count, order, out);
    return hipGetLastError();
}

hipError_t launch_gather_energies(const DevProblem &p, int64_t *f, int64_t *g, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_energies, dim3((p.R + 255) / 256), dim3(256), 0, s, p, f, g);
    return hipGetLastError();
}

hipError_t launch_gather_states(const DevProblem &p, int n, int8_t *out, hipStream_t s)
{
    dim3 grid((p.n_pad + 255) / 256, p.R < 65535 ? p.R : 65535);
    hipLaunchKernelGGL(k_gather_states, grid, dim3(256), 0, s, p, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_best(const DevProblem &p, int8_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_best, dim3((p.n_pad + 255) / 256), dim3(256), 0, s, p, out);
    return hipGetLastError();
}

hipError_t launch_init_states(const DevProblem &p, hipStream_t s)
{
    dim3 grid((p.stride + 255) / 256, p.R);
    hipLaunchKernelGGL(k_init_states, grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_energy(const DevProblem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(p.R), dim3(kSmallBlock), 0, s, p);
    return hipGetLastError();
}

// Dynamic LDS of a sweep workgroup: the spins plus int64 scratch.
static size_t sweep_lds(const DevProblem &p)
{
    return (size_t)p.stride + 8 * (2 + 2 * (kMaxBlock / 64) + 3) + 16;
}

// The persistent workgroup adds its copies of the ladders.
static size_t persistent_lds(const DevProblem &p)
{
    return sweep_lds(p) + 8 * (size_t)p.I + 4 * (size_t)p.J + 8;
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t lds)
{
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NARROW, int WD>
static hipError_t round_sweep_t(const DevProblem &p, hipStream_t s)
{
    if (p.rpb > 1 || p.spin) {
        const size_t lds = (size_t)p.rpb * p.stride + 16 * (size_t)p.rpb + 16;
        hipError_t e = allow_lds(k_round_sweep_multi<NARROW, WD>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_round_sweep_multi<NARROW, WD>), dim3((p.R + p.rpb - 1) / p.rpb),
                           dim3(p.rpb << p.lshift), lds, s, p);
        return hipGetLastError();
    }
    const size_t lds = sweep_lds(p);
    hipError_t e = allow_lds(k_round_sweep<NARROW, WD>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_round_sweep<NARROW, WD>), dim3(p.R), dim3(p.block), lds, s, p);
    return hipGetLastError();
}

template <int NARROW, int WD>
static hipError_t persistent_t(const DevProblem &p, int64_t n_rounds, hipStream_t s, bool query_only,
                               int *max_blocks)
{
    const size_t lds = persistent_lds(p);
    auto kern = k_persistent<NARROW, WD>;
    if (query_only) {
        // a workgroup that does not fit the LDS cannot be resident at all
        int dev = 0, lds_max = 0;
        hipError_t q = hipGetDevice(&dev);
        if (q == hipSuccess) q = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (q != hipSuccess) return q;
        if (lds > (size_t)lds_max) {
            *max_blocks = 0;
            return hipSuccess;
        }
    }
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    if (query_only) {
        int per_cu = 0, dev = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, p.block, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        *max_blocks = per_cu * cus;
        return e;
    }
    DevProblem arg = p;
    void *args[] = {&arg, &n_rounds};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(p.R), dim3(p.block), args, lds, s);
}

// Narrow ELL widths are even (neighbours go in pairs); wide widths are any
// of 1..8, then 12, 16, 24, .., 48 for both; wider rows (multiples of 8) take
// the run-time-width instance WD = 0.  Packed general-constraint problems
// (NARROW = kPackedGen) have widths 2..8.
#define TDPT_DISPATCH(FN, ...)                                              \
    if (p.narrow && p.gen) {                                                \
        switch (p.wd) {                                                     \
        case 2: return FN<kPackedGen, 2>(__VA_ARGS__);                      \
        case 4: return FN<kPackedGen, 4>(__VA_ARGS__);                      \
        case 6: return FN<kPackedGen, 6>(__VA_ARGS__);                      \
        case 8: return FN<kPackedGen, 8>(__VA_ARGS__);                      \
        default: return hipErrorInvalidValue;                               \
        }                                                                   \
    }                                                                       \
    if (p.narrow) {                                                         \
        switch (p.wd) {                                                     \
        case 2: return FN<true, 2>(__VA_ARGS__);                            \
        case 4: return FN<true, 4>(__VA_ARGS__);                            \
        case 6: return FN<true, 6>(__VA_ARGS__);                            \
        case 8: return FN<true, 8>(__VA_ARGS__);                            \
        case 12: return FN<true, 12>(__VA_ARGS__);                          \
        case 16: return FN<true, 16>(__VA_ARGS__);                          \
        case 24: return FN<true, 24>(__VA_ARGS__);                          \
        case 32: return FN<true, 32>(__VA_ARGS__);                          \
        case 40: return FN<true, 40>(__VA_ARGS__);                          \
        case 48: return FN<true, 48>(__VA_ARGS__);                          \
        default:                                                            \
            if (p.wd > 48 && p.wd % 8 == 0) return FN<true, 0>(__VA_ARGS__);  \
            return hipErrorInvalidValue;                                    \
        }                                                                   \
    }                                                                       \
    switch (p.wd) {                                                         \
    case 1: return FN<false, 1>(__VA_ARGS__);                               \
    case 2: return FN<false, 2>(__VA_ARGS__);                               \
    case 3: return FN<false, 3>(__VA_ARGS__);                               \
    case 4: return FN<false, 4>(__VA_ARGS__);                               \
    case 5: return FN<false, 5>(__VA_ARGS__);                               \
    case 6: return FN<false, 6>(__VA_ARGS__);                               \
    case 7: return FN<false, 7>(__VA_ARGS__);                               \
    case 8: return FN<false, 8>(__VA_ARGS__);                               \
    case 12: return FN<false, 12>(__VA_ARGS__);                             \
    case 16: return FN<false, 16>(__VA_ARGS__);                             \
    case 24: return FN<false, 24>(__VA_ARGS__);                             \
    case 32: return FN<false, 32>(__VA_ARGS__);                             \
    case 40: return FN<false, 40>(__VA_ARGS__);                             \
    case 48: return FN<false, 48>(__VA_ARGS__);                             \
    default:                                                                \
        if (p.wd > 48 && p.wd % 8 == 0) return FN<false, 0>(__VA_ARGS__);   \
        return hipErrorInvalidValue;                                        \
    }

hipError_t launch_sweep(const DevProblem &p, hipStream_t s)
{
    if ((p.rpb > 1 || p.spin) &&
        (p.rpb < 1 || p.lshift < 0 || (p.rpb << p.lshift) > kMultiBlock || (p.spin && p.lshift < 2)))
        return hipErrorInvalidValue;
    TDPT_DISPATCH(round_sweep_t, p, s)
}

hipError_t launch_swap(const DevProblem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_track, dim3(1), dim3(kSmallBlock), 0, s, p);
    return hipGetLastError();
}

template <int NARROW, int WD>
static hipError_t batch_sweep_t(const DevProblem &p, const DevProblem *table, const int *first_block,
                                int count, int blocks, int block, size_t max_stride, int rpb, int lshift,
                                int spin, hipStream_t s)
{
    (void)p;
    if (rpb > 1 || spin) {
        const size_t lds = (size_t)rpb * max_stride + 16 * (size_t)rpb + 16;
        hipError_t e = allow_lds(k_batch_sweep_multi<NARROW, WD>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_batch_sweep_multi<NARROW, WD>), dim3(blocks), dim3(block), lds, s, table,
                           first_block, count, rpb, lshift, spin);
        return hipGetLastError();
    }
    const size_t lds = max_stride + 8 * (2 + 2 * (kMaxBlock / 64) + 3) + 16;
    hipError_t e = allow_lds(k_batch_sweep<NARROW, WD>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_batch_sweep<NARROW, WD>), dim3(blocks), dim3(block), lds, s, table,
                       first_block, count);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(const DevProblem &p, const DevProblem *table, const int *first_block,
                              int count, int blocks, int block, size_t max_stride, int rpb, int lshift,
                              int spin, hipStream_t s)
{
    if (rpb < 1 || ((rpb > 1 || spin) && (lshift < 0 || (rpb << lshift) != block || block > kMultiBlock)) ||
        (spin && lshift < 2))
        return hipErrorInvalidValue;
    TDPT_DISPATCH(batch_sweep_t, p, table, first_block, count, blocks, block, max_stride, rpb, lshift, spin, s)
}

static size_t bits_lds(int n_words)
{
    return (size_t)(n_words + 1) * 16 + 8 * 2 * kBitSlots * (kMaxBlock / 64) + 16;
}

template <bool TRACK, int WD, bool PAIR>
static hipError_t sweep_bits_t(const DevProblem &p, hipStream_t s)
{
    const size_t lds = bits_lds(p.n_words);
    hipError_t e = allow_lds(k_round_sweep_bits<WD, TRACK, PAIR>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_round_sweep_bits<WD, TRACK, PAIR>), dim3((p.R + kBitSlots - 1) / kBitSlots),
                       dim3(min(p.block, TRACK ? kBitsBlock : kBitsBlockScratch)), lds, s, p);
    return hipGetLastError();
}

template <bool TRACK, int WD, bool PAIR>
static hipError_t batch_sweep_bits_t(const DevProblem &p, const DevProblem *table, const int *first_block,
                                     int count, int blocks, int block, int max_words, hipStream_t s)
{
    (void)p;
    const size_t lds = bits_lds(max_words);
    hipError_t e = allow_lds(k_batch_sweep_bits<WD, TRACK, PAIR>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_batch_sweep_bits<WD, TRACK, PAIR>), dim3(blocks),
                       dim3(min(block, TRACK ? kBitsBlock : kBitsBlockScratch)), lds, s,
                       table, first_block, count);
    return hipGetLastError();
}

#define TDPT_BITS_CASE(FN, W, TR, PR, ...)                                              \
    case W:                                                                             \
        return (TR) ? ((PR) ? FN<true, W, true>(__VA_ARGS__) : FN<true, W, false>(__VA_ARGS__)) \
                    : ((PR) ? FN<false, W, true>(__VA_ARGS__) : FN<false, W, false>(__VA_ARGS__));
#define TDPT_DISPATCH_BITS(FN, TR, PR, ...)              \
    switch (p.wd) {                                      \
    TDPT_BITS_CASE(FN, 1, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 2, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 3, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 4, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 5, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 6, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 7, TR, PR, __VA_ARGS__)           \
    TDPT_BITS_CASE(FN, 8, TR, PR, __VA_ARGS__)           \
    default: return hipErrorInvalidValue;                \
    }

hipError_t launch_sweep_bits(const DevProblem &p, hipStream_t s)
{
    TDPT_DISPATCH_BITS(sweep_bits_t, track_updates(p.mcs), p.pair16 != 0, p, s)
}

hipError_t launch_batch_sweep_bits(const DevProblem &p, const DevProblem *table, const int *first_block,
                                   int count, int blocks, int block, int max_words, int min_mcs, hipStream_t s)
{
    TDPT_DISPATCH_BITS(batch_sweep_bits_t, track_updates(min_mcs), p.pair16 != 0, p, table, first_block, count,
                       blocks, block,
                       max_words, s)
}

hipError_t launch_batch_swap(const DevProblem *table, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_swap, dim3(count), dim3(kSmallBlock), 0, s, table);
    return hipGetLastError();
}

hipError_t persistent_max_blocks(const DevProblem &p, int *max_blocks)
{
    TDPT_DISPATCH(persistent_t, p, 0, nullptr, true, max_blocks)
}

hipError_t launch_persistent(const DevProblem &p, int64_t n_rounds, hipStream_t s)
{
    TDPT_DISPATCH(persistent_t, p, n_rounds, s, false, nullptr)
}

hipError_t launch_scratch_reset(const DevProblem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_scratch_reset, dim3((p.R + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevProblem &p, int64_t n_rounds, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kSmallBlock), 0, s, p, n_rounds);
    return hipGetLastError();
}

size_t persistent_lds_bytes(int stride, int I, int J)
{
    DevProblem q{};
    q.stride = stride;
    q.I = I;
    q.J = J;
    return persistent_lds(q);
}

template <int NARROW, int WD>
static hipError_t batch_persistent_t(const DevProblem &p, const DevProblem *table, const int *first_block,
                                     int count, int blocks, int block, size_t lds, int64_t n_rounds, hipStream_t s,
                                     int *max_blocks)
{
    (void)p;
    auto kern = k_batch_persistent<NARROW, WD>;
    if (max_blocks) {
        int dev = 0, lds_max = 0, per_cu = 0, cus = 0;
        hipError_t q = hipGetDevice(&dev);
        if (q == hipSuccess) q = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (q != hipSuccess) return q;
        if (lds > (size_t)lds_max) {
            *max_blocks = 0;
            return hipSuccess;
        }
        q = allow_lds(kern, lds);
        if (q == hipSuccess) q = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds);
        if (q == hipSuccess) q = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        *max_blocks = per_cu * cus;
        return q;
    }
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    void *args[] = {&table, &first_block, &count, &n_rounds};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(blocks), dim3(block), args, lds, s);
}

hipError_t batch_persistent_max_blocks(const DevProblem &p, int block, size_t lds, int *max_blocks)
{
    TDPT_DISPATCH(batch_persistent_t, p, nullptr, nullptr, 0, 0, block, lds, 0, nullptr, max_blocks)
}

hipError_t launch_batch_persistent(const DevProblem &p, const DevProblem *table, const int *first_block, int count,
                                   int blocks, int block, size_t lds, int64_t n_rounds, hipStream_t s)
{
    TDPT_DISPATCH(batch_persistent_t, p, table, first_block, count, blocks, block, lds, n_rounds, s, nullptr)
}

hipError_t launch_batch_scratch_reset(const DevProblem *table, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_scratch_reset, dim3(count), dim3(kSmallBlock), 0, s, table);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const DevProblem *table, int count, int64_t n_rounds, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_finalize, dim3(count), dim3(kSmallBlock), 0, s, table, n_rounds);
    return hipGetLastError();
}

}  // namespace tdpt
