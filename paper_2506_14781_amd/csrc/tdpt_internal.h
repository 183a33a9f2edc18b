// Internal layout shared by the host runtime and the gfx950 kernels of the
// 2D parallel tempering library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdpt {

constexpr int kMaxColors = 32;
constexpr int kMaxBlock = 1024;   // threads per sweep workgroup, at most
constexpr int kSmallBlock = 256;  // threads of the swap / energy kernels
constexpr int kMultiBlock = 256;  // threads per workgroup of the packed-slot sweeps, at most
constexpr int kRing = 8;          // rounds of partner mailboxes kept per position
constexpr int kBitSlots = 4;      // replicas per workgroup in the bit-packed layout
constexpr int kBitsBlock = 768;   // threads of a bit-packed sweep workgroup that follows f and g
                                  // update by update, at most
constexpr int kBitsBlockScratch = 1024;  // at most, when f and g are recomputed at the round's end
constexpr int kMaxHistVars = 20;  // logical variables of the per-round state histogram, at most

// Structure layouts of the byte-replica sweeps (their NARROW template
// argument): 32-bit rows; packed 16-bit index and coupling pairs with copy
// edges; packed problem rows with 32-bit general-constraint rows.
constexpr int kWide = 0;
constexpr int kPacked = 1;
constexpr int kPackedGen = 2;

// Header words of a problem's device state (int64 each).
enum HdrWord {
    kHdrRounds = 0,    // swap rounds completed
    kHdrFirstHit = 1,  // first sweep count with a target hit, -1 if none
    kHdrBestF = 2,     // best feasible bottom-right f_q, INT64_MAX if none
    kHdrBestSweep = 3, // sweep count of best_f, -1 if none
    kHdrError = 4,     // nonzero: a persistent launch gave up waiting for a partner
    kHdrWords = 8
};

// Best-state keys of the persistent driver: (f_q + 2^30) * 2^32 + sweep,
// ordered like (f_q, sweep).  Valid while |f_q| < 2^30 and sweeps < 2^32.
constexpr int64_t kKeyOffset = (int64_t)1 << 30;

// Everything a kernel needs about one problem, passed by value.
// Spins are numbered colour-major: class c occupies [cls_start[c],
// cls_live[c]) followed by dead padding up to cls_start[c+1] (a multiple of
// 4).  Index n_pad is a spin that is always 0; missing neighbours point there.
//
// Narrow structure (indices < 2^16, couplings in int16, fields < 2^22):
//   nbi[k2][n_pad]  neighbour indices 2*k2 and 2*k2+1 packed as 16+16 bits
//   nbj[k2][n_pad]  their couplings packed as int16 pairs
//   chp[n_pad]      the two copy neighbours packed as 16+16 bits
// Wide structure: nb_idx / nb_J [wd][n_pad] int32, ch_idx [2][n_pad] int32.
// Bit-packed layout (replicas too large for an int8 copy in LDS): spins are
// bits (1 = +1) in LDS; each colour class starts on a 32-bit boundary of the
// bit numbering (bit_start[c]), so spin rho of class c sits at bit
// b = rho - cls_start[c] + bit_start[c], and the kBitSlots replicas' bits
// b = 32 G .. 32 G + 31 fill the 16-byte word group G.  Within a group:
//   plain form: word r (byte 16 G + 4 r) holds bit b & 31 of replica r;
//     a position is stored as (G << 9) | (b & 31);
//   pair form (pair16): word 2 h + p (h = (b >> 4) & 1) holds bit b & 15 of
//     replica 2 p and, 16 places up, of replica 2 p + 1; a position is stored
//     as (G << 9) | (h << 8) | (b & 15).
// Either way a position shifted right by 5 is the LDS byte address of the
// words that hold the bit (the plain form's group, the pair form's word
// pair) and its low 5 bits are the bit's place in the word (of the replica
// pair's lower replica).  Structure:
//   nb_pos / nb_J [wd][n_pad] (missing neighbours: position 0, coupling 0),
//   nb_J2 [wd][n_pad] (pair form: 2 J as a 16-bit number in both halves),
//   ch_pos [2][n_pad] (a missing copy neighbour names bit 0 of an always-zero
//   word group n_words; row 0 also holds in bits 29..30 how many of the two
//   exist), h0 [n_pad] = b - sum_k J_k.
// The pair form sums the couplings of two replicas at once in 16-bit
// halves; the host chooses it when every spin's sum of 2 |J| over its
// problem neighbours is below 2^15, so the halves never overflow.
struct DevProblem {
    // structure (immutable)
    int32_t n_pad;      // padded spin count
    int32_t stride;     // bytes per replica slot (>= n_pad + 1, multiple of 16)
    int32_t n_colors;
    int32_t wd;         // problem-neighbour ELL width (even in the narrow layout)
    int32_t narrow;
    int32_t has_bias;   // any nonzero field
    int32_t block;      // threads per sweep workgroup
    int32_t rpb;        // per-round driver, int8: > 1 packs rpb slots per workgroup
    int32_t lshift;     // of 2^lshift lanes each (rpb << lshift threads)
    int32_t spin;       // packed sweep with one spin per lane (4 lanes per quad)
    int32_t bits;       // bit-packed layout
    int32_t pair16;     // its pair form
    int32_t n_words;    // 32-bit words per replica in the bit-packed layout
    int32_t bit_start[kMaxColors + 1];
    const int32_t *nb_pos; // bit-packed
    const int32_t *ch_pos; // bit-packed
    const int32_t *h0;     // bit-packed
    const uint32_t *nb_J2; // bit-packed, pair form
    int32_t cls_start[kMaxColors + 1];
    int32_t cls_live[kMaxColors];
    const uint32_t *nbi;   // narrow
    const uint32_t *nbj;   // narrow
    const uint32_t *chp;   // narrow
    const int32_t *nb_idx; // wide
    const int32_t *nb_J;   // wide
    const int32_t *ch_idx; // wide
    // General constraints (byte layout only): half the penalty field of spin
    // i is kh[i] + sum_k cn_w[k][i] s[cn_idx[k][i]] instead of the copy sum;
    // g = g0 - sum_i s_i (2 kh[i] + sum_k cn_w[k][i] s[cn_idx[k][i]]).
    int32_t gen;
    int32_t wcg;           // constraint ELL width, a multiple of 4
    const int32_t *cn_idx; // [wcg][n_pad] (padding: index n_pad, weight 0)
    const int32_t *cn_w;   // [wcg][n_pad]
    const int32_t *kh;     // [n_pad]
    int64_t g0;
    const int32_t *bias;   // [n_pad]
    const int32_t *orig;   // [n_pad] original spin index, -1 for padding
    // run configuration
    int32_t I, J, R;
    int32_t mcs;
    uint32_t key0, key1;
    uint32_t flags;
    int32_t has_target;
    int64_t f_target;
    int64_t trace_cap;
    const double *beta;   // [I]
    const int32_t *p_q;   // [J]
    // mutable state
    int64_t *hdr;         // [kHdrWords]
    int8_t *states;       // [R][stride]
    int64_t *f;           // [R] per slot
    int64_t *g;           // [R] per slot
    int32_t *slot_pos;    // [R]
    int32_t *pos_slot;    // [R]
    int64_t *p_att, *p_acc; // [I*(J-1)]
    int64_t *b_att, *b_acc; // [J*(I-1)]
    int8_t *best_state;   // [stride]
    int64_t *trace_f, *trace_g; // [trace_cap]
    // histogram of the bottom-right replica's logical state, one sample per
    // round after the swap step (hist_n = 0: off): bin sum_k [s > 0] 2^k over
    // the spins at colour-major positions hist_rank[0 .. hist_n)
    int32_t hist_n;
    const int32_t *hist_rank; // [hist_n]
    uint32_t *hist;           // [2^hist_n]
    // optional stage timestamps of the persistent driver (stage_cap = 0:
    // off): for rounds stage_round0 + 1 .. stage_round0 + stage_cap, per slot,
    // the 100 MHz real-time clock at the round's start, after its sweeps,
    // once the partner's (f, g) is in hand, and after the swap decision
    uint64_t *stage;          // [stage_cap][R][4], caller-owned device memory
    int32_t stage_cap;
    int64_t stage_round0;
    // persistent driver: workgroup b serves slot (b * slot_mul + slot_add) mod R
    // (1, 0 normally; gcd(slot_mul, R) = 1), so tests can vary which
    // workgroup, and so which compute unit and XCD, holds which slot
    int32_t slot_mul, slot_add;
    // scratch of the persistent driver (not part of checkpoints)
    uint64_t *mbox;       // [kRing][R][2] tagged (f, g) by grid position
    int64_t *slot_key;    // [R] best key per slot during a launch
    int8_t *slot_best;    // [R][stride] state behind slot_key
    int64_t *hit_min;     // [1] smallest sweep with a target hit during a launch
};

// Kernel launchers (tdpt_kernels.hip).  Return a hipError_t.
hipError_t launch_init_states(const DevProblem &p, hipStream_t s);
hipError_t launch_energy(const DevProblem &p, hipStream_t s);
hipError_t launch_sweep(const DevProblem &p, hipStream_t s);
hipError_t launch_swap(const DevProblem &p, hipStream_t s);
hipError_t persistent_max_blocks(const DevProblem &p, int *max_blocks);
hipError_t launch_persistent(const DevProblem &p, int64_t n_rounds, hipStream_t s);
hipError_t launch_scratch_reset(const DevProblem &p, hipStream_t s);
hipError_t launch_finalize(const DevProblem &p, int64_t n_rounds, hipStream_t s);
// Batched rounds over a device table of problems sharing p's layout (p is
// any member: it selects the kernel instance).  rpb slots per workgroup of
// `block` threads, 2^lshift lanes each (rpb << lshift == block) when rpb > 1
// or spin (one spin per lane, 2^lshift >= 4); first_block then counts
// ceil(R / rpb) workgroups per member.
hipError_t launch_batch_sweep(const DevProblem &p, const DevProblem *table, const int *first_block,
                              int count, int blocks, int block, size_t max_stride, int rpb, int lshift,
                              int spin, hipStream_t s);
hipError_t launch_batch_swap(const DevProblem *table, int count, hipStream_t s);
// Batched persistent driver over one layout group of count members whose
// block ranges (prefix sums in first_block) cover `blocks` workgroups; lds is
// the group's largest persistent_lds_bytes.  Cooperative: every workgroup
// must be resident at once (batch_persistent_max_blocks).
size_t persistent_lds_bytes(int stride, int I, int J);
hipError_t batch_persistent_max_blocks(const DevProblem &p, int block, size_t lds, int *max_blocks);
hipError_t launch_batch_persistent(const DevProblem &p, const DevProblem *table, const int *first_block, int count,
                                   int blocks, int block, size_t lds, int64_t n_rounds, hipStream_t s);
hipError_t launch_batch_scratch_reset(const DevProblem *table, int count, hipStream_t s);
hipError_t launch_batch_finalize(const DevProblem *table, int count, int64_t n_rounds, hipStream_t s);
// Readback into device buffers, in grid-position order and the caller's
// spin numbering (n physical spins): f and g [R]; states [R][n]; the best
// state [n].
hipError_t launch_gather_energies(const DevProblem &p, int64_t *f, int64_t *g, hipStream_t s);
hipError_t launch_gather_states(const DevProblem &p, int n, int8_t *out, hipStream_t s);
hipError_t launch_gather_best(const DevProblem &p, int8_t *out, hipStream_t s);
// [count][4] status words of a batch's members at out[order[i]] for table entry i.
hipError_t launch_batch_status(const DevProblem *table, int count, const int32_t *order, int64_t *out,
                               hipStream_t s);
// Bit-packed layout: one round of every slot (ceil(R / kBitSlots) blocks).
// Bit-packed sweeps of fewer than kScratchMcs per round follow f and g update
// by update; longer rounds recompute them from the round's final states
// (min_mcs: the fewest sweeps per round among a batch group's members).
constexpr int kScratchMcs = 4;
__host__ __device__ inline bool track_updates(int mcs) { return mcs < kScratchMcs; }
__host__ __device__ inline int bits_block_cap(int mcs) { return track_updates(mcs) ? kBitsBlock : kBitsBlockScratch; }
hipError_t launch_sweep_bits(const DevProblem &p, hipStream_t s);
hipError_t launch_batch_sweep_bits(const DevProblem &p, const DevProblem *table, const int *first_block,
                                   int count, int blocks, int block, int max_words, int min_mcs,
                                   hipStream_t s);

}  // namespace tdpt
