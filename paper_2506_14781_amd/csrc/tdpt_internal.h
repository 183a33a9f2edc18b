// Internal layout shared by the host runtime and the gfx950 kernels of the
// 2D parallel tempering library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdpt {

constexpr int kMaxColors = 32;
constexpr int kBlock = 256;       // threads per sweep workgroup (4 wave64)
constexpr int kMaxSlotsPerBlock = 4;

// Header words of a problem's device state (int64 each).
enum HdrWord {
    kHdrRounds = 0,    // swap rounds completed
    kHdrFirstHit = 1,  // first sweep count with a target hit, -1 if none
    kHdrBestF = 2,     // best feasible bottom-right f_q, INT64_MAX if none
    kHdrBestSweep = 3, // sweep count of best_f, -1 if none
    kHdrWords = 8
};

// Everything a kernel needs about one problem, passed by value.
// Spins are numbered colour-major: class c occupies [cls_start[c],
// cls_live[c]) followed by dead padding up to cls_start[c+1] (a multiple of
// 4).  Index n_pad is a spin that is always 0; missing neighbours point there.
struct DevProblem {
    // structure (immutable)
    int32_t n_pad;      // padded spin count
    int32_t stride;     // bytes per replica slot (>= n_pad + 1, multiple of 16)
    int32_t n_colors;
    int32_t wd;         // problem-neighbour ELL width
    int32_t wc;         // copy-neighbour ELL width
    int32_t narrow;     // nbp/chp packed 16+16 bit layout
    int32_t cls_start[kMaxColors + 1];
    int32_t cls_live[kMaxColors];
    const uint32_t *nbp;   // narrow: [wd][n_pad] idx | (J << 16)
    const int32_t *nb_idx; // wide: [wd][n_pad]
    const int32_t *nb_J;   // wide: [wd][n_pad]
    const uint32_t *chp;   // narrow (wc <= 2): [n_pad] c0 | (c1 << 16)
    const int32_t *ch_idx; // wide: [wc][n_pad]
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
};

// Kernel launchers (tdpt_kernels.hip).  Return a hipError_t.
hipError_t launch_init_states(const DevProblem &p, hipStream_t s);
hipError_t launch_energy(const DevProblem &p, hipStream_t s);
hipError_t launch_sweep(const DevProblem &p, int slots_per_block, hipStream_t s);
hipError_t launch_swap(const DevProblem &p, hipStream_t s);

}  // namespace tdpt
