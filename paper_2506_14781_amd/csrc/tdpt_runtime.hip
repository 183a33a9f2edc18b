// Host runtime of the 2D parallel tempering library: instance validation
// and colour-major re-layout, workspace layout, problem lifecycle, readback
// and checkpoints.  All sampling work runs in the kernels of
// tdpt_kernels.hip; this file only moves data and launches.
#include "tdpt.h"
#include "tdpt_internal.h"

#include <algorithm>
#include <functional>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof(buf), "%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
    g_err = buf;
    return TDPT_E_DEVICE;
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr size_t kMaxTimedLaunches = 4096;

// ELL widths the sweep kernels are instantiated for.
// ELL width (neighbour slots per spin) for a largest problem degree: the
// degree itself up to 8, then 12, then multiples of 8 up to kMaxWidth.
constexpr int kMaxWidth = 256;

int ell_width(int deg)
{
    if (deg <= 8) return std::max(deg, 1);
    if (deg <= 12) return 12;
    if (deg <= kMaxWidth) return (deg + 7) / 8 * 8;
    return -1;
}

}  // namespace

struct tdpt_instance {
    int32_t n = 0, n_pad = 0, n_colors = 0, wd = 0, narrow = 0, m = 0;
    int32_t max_deg = 0, max_copy_deg = 0;
    int64_t nnz = 0;
    std::vector<int32_t> rank;       // original -> colour-major
    std::vector<int32_t> orig;       // colour-major -> original (-1 padding)
    std::vector<int32_t> cls_start;  // [C+1]
    std::vector<int32_t> cls_live;   // [C]
    std::vector<int32_t> nb_idx, nb_J;  // [wd][n_pad]
    std::vector<int32_t> ch_idx;        // [2][n_pad]
    std::vector<int32_t> bias;          // [n_pad]
    int32_t has_bias = 0;
    int64_t max_field = 0;   // max_i sum_j |J_ij| + |b_i|
    int64_t max_abs_J = 0;   // max |J_ij|
    int64_t max_row_J = 0;   // max_i sum_j |J_ij|
    int64_t abs_f_bound = 0; // sum_{i<j} |J_ij| + sum_i |b_i|
    int32_t max_class_quads = 0;
    // The penalty field of spin i is 2 P c_i; c_i is the copy sum, or for
    // general constraints kh_i + sum_j Kh_ij s_j (constraint ELL cn_*).
    int32_t gen = 0;         // general constraint terms instead of copy edges
    int32_t n_terms = 0, max_cons_deg = 0;
    int32_t wcg = 0;         // constraint ELL width (multiple of 4)
    std::vector<int32_t> cn_idx, cn_w;  // [wcg][n_pad]
    std::vector<int32_t> kh;            // [n_pad]
    int64_t g0 = 0;          // constant of g
    int64_t max_cfield = 0;  // max_i |c_i|
    int64_t g_bound = 0;     // max |g|
    // logical variables (optional): variable k is read from its lowest-
    // numbered physical spin first_copy[k] (colour-major position first_rank[k])
    int32_t n_logical = 0;
    std::vector<int32_t> first_copy, first_rank;
};

struct tdpt_problem {
    tdpt::DevProblem dp{};
    hipStream_t stream = nullptr;
    tdpt_batch *batch = nullptr;  // the batch that holds it as a member, if any
    int32_t n_logical = 0;        // logical variables and their first copies
    std::vector<int32_t> first_copy;
    int32_t static_dev = -1;      // device whose static workspace it holds (-1: caller's memory)
    int32_t n = 0, I = 0, J = 0, R = 0, mcs = 1;
    std::vector<int32_t> rank;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0, mut_off = 0, mut_bytes = 0, mbox_off = 0, mbox_bytes = 0;
    int64_t trace_cap = 0;
    uint64_t fingerprint = 0;
    bool persistent = false;
    bool persistent_ok = false;  // the persistent driver may be used (layout, key range)
    int32_t min_block = 64;      // smallest sweep workgroup the per-phase bounds allow
    int32_t min_lanes = 1;       // fewest lanes per replica the per-phase bounds allow
    size_t stride_bytes = 0;     // bytes per replica slot
    int32_t max_class_quads = 0;
    int64_t rounds_host = 0;  // rounds done, as far as the host has enqueued them
    // rounds_host when the partner mailboxes were last valid (after a
    // persistent run, or cleared); rounds run since by per-round launches
    // leave them stale, and a stale entry 2^15 rounds old would carry a
    // matching round tag, so they are cleared before the next persistent run
    int64_t mbox_round = 0;
    // optional sweep-kernel timing (HIP events on the problem's stream)
    int32_t time_every = 0;
    int64_t sweep_launches = 0;
    int64_t timed_rounds = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    ~tdpt_problem()
    {
        for (auto &e : events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

namespace {

struct Layout {
    size_t hdr, states, f, g, slot_pos, pos_slot, p_att, p_acc, b_att, b_acc, best, trace_f,
        trace_g, hist, mut_end, mbox, slot_key, slot_best, hit_min, scratch_end;
    size_t beta, p_q, nbi, nbj, chp, nb_idx, nb_J, ch_idx, bias, orig, nb_pos, ch_pos, h0, nb_J2, cn_idx, cn_w, kh,
        hist_rank, total;
    int32_t stride, wd;
};

// Replicas whose int8 copy exceeds this many bytes of LDS use the bit-packed
// layout (kBitSlots replicas per workgroup as bits).
constexpr size_t kInt8StrideMax = 48 * 1024;

bool use_bits(const tdpt_instance *in)
{
    if (in->gen) return false;  // general constraints use the byte layout only
    if (const char *e = getenv("TDPT_LAYOUT")) {
        if (!strcmp(e, "bits")) return true;
        if (!strcmp(e, "bytes")) return false;
    }
    return align_up((size_t)in->n_pad + 1, 16) > kInt8StrideMax;
}

// The bit-packed layout's pair form sums 2 J_k b_k of two replicas in the
// 16-bit halves of one word: every spin's sum of 2 |J| must stay below 2^15.
bool use_pair16(const tdpt_instance *in)
{
    if (!use_bits(in)) return false;
    if (const char *e = getenv("TDPT_PAIR16"))
        if (!strcmp(e, "0")) return false;
    return 2 * in->max_row_J < ((int64_t)1 << 15);
}

// The packed structure (16-bit indices and coupling pairs) and the 16/24-bit
// arithmetic of the sweep need indices and couplings that fit 16 bits and
// every local field, penalty term and energy change below 2^22.  General
// constraints keep their rows 32-bit in either layout (packed only up to 8
// problem neighbours).
bool use_narrow(const tdpt_instance *in, const tdpt_run_cfg *cfg)
{
    const int64_t pmax = cfg->p_q[cfg->n_p - 1];
    return !use_bits(in) && in->narrow && (!in->gen || in->wd <= 8) &&
           in->max_field + 2 * pmax * in->max_cfield < ((int64_t)1 << 22) && in->max_cfield < ((int64_t)1 << 22);
}

Layout make_layout(const tdpt_instance *in, int32_t I, int32_t J, int64_t trace_cap, bool narrow,
                   int32_t hist_n)
{
    Layout L{};
    const size_t R = (size_t)I * J;
    L.stride = (int32_t)align_up((size_t)in->n_pad + 1, 16);
    L.wd = narrow ? (in->wd + 1) / 2 * 2 : in->wd;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.hdr = take(sizeof(int64_t) * tdpt::kHdrWords);
    L.states = take(R * (size_t)L.stride);
    L.f = take(R * 8);
    L.g = take(R * 8);
    L.slot_pos = take(R * 4);
    L.pos_slot = take(R * 4);
    const size_t np = (size_t)I * (J > 1 ? J - 1 : 0), nb = (size_t)J * (I > 1 ? I - 1 : 0);
    L.p_att = take(np * 8 + 8);
    L.p_acc = take(np * 8 + 8);
    L.b_att = take(nb * 8 + 8);
    L.b_acc = take(nb * 8 + 8);
    L.best = take((size_t)L.stride);
    L.trace_f = take((size_t)trace_cap * 8 + 8);
    L.trace_g = take((size_t)trace_cap * 8 + 8);
    L.hist = take(hist_n ? ((size_t)4 << hist_n) : 8);
    L.mut_end = o;
    L.mbox = take((size_t)tdpt::kRing * R * 16);
    L.slot_key = take(R * 8);
    L.slot_best = take(R * (size_t)L.stride);
    L.hit_min = take(8);
    L.scratch_end = o;
    L.beta = take((size_t)I * 8);
    L.p_q = take((size_t)J * 4);
    if (narrow) {
        const size_t rows = (size_t)(L.wd / 2) * in->n_pad * 4;
        L.nbi = take(rows);
        L.nbj = take(rows);
        L.nb_idx = L.nb_J = L.ch_idx = 0;
        if (in->gen) {
            const size_t cell = (size_t)in->wcg * in->n_pad * 4;
            L.cn_idx = take(cell);
            L.cn_w = take(cell);
            L.kh = take((size_t)in->n_pad * 4);
            L.chp = 0;
        } else {
            L.chp = take((size_t)in->n_pad * 4);
        }
    } else {
        const size_t ell = (size_t)L.wd * in->n_pad * 4;
        L.nb_idx = take(ell);
        L.nb_J = take(ell);
        L.nbi = L.nbj = L.chp = 0;
        if (in->gen) {
            const size_t cell = (size_t)in->wcg * in->n_pad * 4;
            L.cn_idx = take(cell);
            L.cn_w = take(cell);
            L.kh = take((size_t)in->n_pad * 4);
            L.ch_idx = 0;
        } else {
            L.ch_idx = take((size_t)2 * in->n_pad * 4);
        }
        if (use_bits(in)) {
            L.nb_pos = take(ell);
            L.ch_pos = take((size_t)2 * in->n_pad * 4);
            L.h0 = take((size_t)in->n_pad * 4);
            L.nb_J2 = take(ell);
        }
    }
    L.bias = take((size_t)in->n_pad * 4);
    L.orig = take((size_t)in->n_pad * 4);
    L.hist_rank = take((size_t)hist_n * 4 + 4);
    L.total = o;
    return L;
}

// Logical variables of the per-round state histogram a configuration asks
// for (0: none).
int hist_vars(const tdpt_instance *in, const tdpt_run_cfg *cfg, int32_t *nv)
{
    *nv = 0;
    if (!cfg->hist_logical) return TDPT_OK;
    if (in->n_logical < 1)
        return fail(TDPT_E_INVALID, "a logical-state histogram needs logical_of at instance creation");
    if (in->n_logical > tdpt::kMaxHistVars)
        return fail(TDPT_E_INVALID, "a logical-state histogram takes at most 20 logical variables");
    *nv = in->n_logical;
    return TDPT_OK;
}

int check_cfg(const tdpt_run_cfg *c)
{
    if (!c) return fail(TDPT_E_INVALID, "cfg is NULL");
    if (c->n_beta < 1 || !c->beta) return fail(TDPT_E_INVALID, "need n_beta >= 1 and a beta array");
    if (c->n_p < 1 || !c->p_q) return fail(TDPT_E_INVALID, "need n_p >= 1 and a p_q array");
    if ((int64_t)c->n_beta * c->n_p > (1 << 22)) return fail(TDPT_E_INVALID, "replica grid too large");
    for (int i = 0; i < c->n_beta; ++i) {
        if (!std::isfinite(c->beta[i]) || c->beta[i] <= 0.0)
            return fail(TDPT_E_INVALID, "beta must be finite and > 0");
        if (i && !(c->beta[i] > c->beta[i - 1]))
            return fail(TDPT_E_INVALID, "beta must be strictly ascending");
    }
    for (int j = 0; j < c->n_p; ++j) {
        if (c->p_q[j] < 0) return fail(TDPT_E_INVALID, "p_q must be >= 0");
        if (j && c->p_q[j] < c->p_q[j - 1]) return fail(TDPT_E_INVALID, "p_q must be non-decreasing");
    }
    if (c->mcs_per_swap < 1) return fail(TDPT_E_INVALID, "mcs_per_swap must be >= 1");
    if (c->trace_cap < 0) return fail(TDPT_E_INVALID, "trace_cap must be >= 0");
    if (c->flags & ~TDPT_NO_PSWAP) return fail(TDPT_E_INVALID, "unknown flag bits");
    return TDPT_OK;
}

// The fewest passes of a workgroup of at most `cap` threads over `quads`
// quads (one per lane per pass), then the fewest threads that keep that
// number of passes, in whole waves -- whole groups of four waves (one per
// SIMD of the compute unit) once a pass needs that many, since a compute
// unit whose SIMDs hold unequal wave counts waits for the fullest at every
// class barrier (at N=1000, one bit-packed workgroup per compute unit:
// 960 threads 33.5 ms per round, 1024 threads 31.6 ms).
int balanced_block(int quads, int cap)
{
    const int passes = std::max(1, (quads + cap - 1) / cap);
    const int need = (quads + passes - 1) / passes;
    const int g = need > 256 ? 256 : 64;
    const int b = (need + g - 1) / g * g;
    return std::min(std::max(b, 64), cap);
}

// Whether rpb slots of `stride` bytes fit the LDS a workgroup takes without
// giving up occupancy (64 KiB).
bool pack_fits(size_t stride, int rpb)
{
    return (size_t)rpb * (stride + 16) + 16 <= 65536;
}

// Default packing of an int8 replica for per-round sweeps: when its largest
// colour class takes under 64 lanes, one wave of 64 threads holds 64 / L
// slots, L the power of two (at least 4) covering that class and the lanes
// the per-phase bounds need; else one slot per workgroup (rpb = 1).
void default_pack(int max_quads, int min_lanes, size_t stride, int32_t *rpb, int32_t *lshift)
{
    *rpb = 1;
    *lshift = 0;
    int ls = 2;
    while ((1 << ls) < std::max(max_quads, min_lanes)) ++ls;
    if (ls >= 6 || !pack_fits(stride, 64 >> ls)) return;
    *rpb = 64 >> ls;
    *lshift = ls;
}

// Whether the packed sweep keeps a replica's structure in registers for a
// whole round (packed copy-edge layout, at most 4 problem neighbours, no
// fields, two colour classes of at most 2^lshift quads).  Then per-round
// launches beat the persistent driver once a round holds enough sweeps.
bool pack_hoists(bool narrow, bool gen, bool bits, bool has_bias, int wd, int n_colors, int max_quads,
                 int lshift)
{
    return narrow && !gen && !bits && !has_bias && wd <= 4 && n_colors == 2 && max_quads <= (1 << lshift);
}
bool pack_hoists(const tdpt::DevProblem &d, int max_quads, int lshift)
{
    return pack_hoists(d.narrow != 0, d.gen != 0, d.bits != 0, d.has_bias != 0, d.wd, d.n_colors, max_quads,
                       lshift);
}
constexpr int kPackRoundMcs = 16;  // sweeps per round from which packed per-round launches are preferred

// Shape of the packed sweep with one spin per lane (packed copy-edge layout,
// at most 8 problem neighbours): 2^lshift lanes, the power of two (>= 4,
// <= 256) covering the largest colour class's spins, so a lane takes one
// spin per phase; 64 / 2^lshift replicas per 64-thread workgroup below 64
// lanes, else one.  False when the replica does not qualify.
bool spin_shape(bool narrow, bool gen, bool bits, int wd, int max_quads, size_t stride, int32_t *rpb,
                int32_t *lshift)
{
    if (!narrow || gen || bits || wd > 8 || max_quads < 1 || 4 * max_quads > tdpt::kMultiBlock) return false;
    int ls = 2;
    while ((1 << ls) < 4 * max_quads) ++ls;
    const int r = std::max(1, 64 >> ls);
    if (!pack_fits(stride, r)) return false;
    *rpb = r;
    *lshift = ls;
    return true;
}

// Waves of one round of R replicas at rpb replicas per workgroup of
// rpb << lshift threads.
int64_t round_waves(int R, int rpb, int lshift)
{
    return (int64_t)((R + rpb - 1) / rpb) * std::max(1, (rpb << lshift) / 64);
}

// Up to this many waves per round (two per SIMD) the replicas' lanes are
// latency-bound and the spin-per-lane sweep is the default; beyond it the
// GPU is full and the quad-per-lane sweep, a quarter of the Philox work,
// is (N=12 batches, 50 sweeps per round: spin / quad 34 / 45 us per round
// at 32 problems = 1024 waves, 42 / 49 at 64, 53 / 50 at 96).
constexpr int64_t kSpinWaves = 2048;

// Fewest lanes per replica that keep every lane's per-phase sums of 2 |h|
// (f) and 2 |c| (g) over its quads below 2^31, for the largest penalty of
// the configuration (c is the half penalty field, which P = 0 leaves out of
// the field bound).
int32_t min_lanes_for(const tdpt_instance *in, int64_t pmax)
{
    const int64_t hmax = in->max_field + 2 * pmax * in->max_cfield;
    const int64_t hb = std::max(hmax, in->max_cfield);
    const int64_t q_allowed = std::max<int64_t>(1, (((int64_t)1 << 31) - 1) / (8 * std::max<int64_t>(hb, 1)));
    return (int32_t)std::max<int64_t>(1, (in->max_class_quads + q_allowed - 1) / q_allowed);
}

// Threads of a sweep workgroup: one lane per quad of the largest colour
// class, in balanced passes of at most `cap` threads (per-round driver), or
// one lane per two quads (persistent driver, whose two blocks per compute
// unit must both stay resident).
int sweep_block(const tdpt_instance *in, bool persistent, int cap = tdpt::kMaxBlock)
{
    const int quads = persistent ? (in->max_class_quads + 1) / 2 : in->max_class_quads;
    if (persistent) cap = tdpt::kMaxBlock / 2;
    int b = persistent ? (quads + 63) / 64 * 64 : balanced_block(quads, cap);
    if (const char *e = getenv("TDPT_BLOCK")) {
        const int v = atoi(e);
        if (v >= 64 && v <= cap && v % 64 == 0) b = v;
    }
    return std::min(std::max(b, 64), cap);
}

// Problem couplings: CSR shape, symmetry, no self loops or repeats; fills
// ent with each row's (col, J) sorted by col.
int check_csr(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
              const int32_t *b_q, const int32_t *color, std::vector<std::pair<int32_t, int32_t>> &ent)
{
    (void)b_q;
    if (n <= 0 || !row_ptr || !color) return fail(TDPT_E_INVALID, "need n > 0, row_ptr and color");
    if (row_ptr[0] != 0) return fail(TDPT_E_INVALID, "row_ptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return fail(TDPT_E_INVALID, "row_ptr must be non-decreasing");
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && (!col || !J_q)) return fail(TDPT_E_INVALID, "col and J_q are required");
    ent.assign((size_t)nnz, {0, 0});
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (j < 0 || j >= n) return fail(TDPT_E_INVALID, "col index out of range at row " + std::to_string(i));
            if (j == i) return fail(TDPT_E_INVALID, "self loop at spin " + std::to_string(i));
            ent[e] = {j, J_q[e]};
        }
        std::sort(ent.begin() + row_ptr[i], ent.begin() + row_ptr[i + 1]);
        for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e)
            if (ent[e].first == ent[e - 1].first)
                return fail(TDPT_E_INVALID, "repeated neighbour in row " + std::to_string(i));
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = ent[e].first;
            auto b = ent.begin() + row_ptr[j], en = ent.begin() + row_ptr[j + 1];
            auto it = std::lower_bound(b, en, std::make_pair(i, INT32_MIN));
            if (it == en || it->first != i || it->second != ent[e].second)
                return fail(TDPT_E_INVALID, "couplings are not symmetric at (" + std::to_string(i) + "," +
                                                std::to_string(j) + ")");
        }
    return TDPT_OK;
}

bool csr_has(const int32_t *row_ptr, const std::vector<std::pair<int32_t, int32_t>> &ent, int32_t i, int32_t j)
{
    auto b = ent.begin() + row_ptr[i], e = ent.begin() + row_ptr[i + 1];
    auto it = std::lower_bound(b, e, std::make_pair(j, INT32_MIN));
    return it != e && it->first == j;
}

// Colour classes: count (<= kMaxColors) and properness over the couplings.
int check_colors(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *color, int32_t &C)
{
    C = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (color[v] < 0) return fail(TDPT_E_INVALID, "negative colour");
        C = std::max(C, color[v] + 1);
    }
    if (C > tdpt::kMaxColors) return fail(TDPT_E_INVALID, "more than 32 colour classes");
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (color[i] == color[col[e]])
                return fail(TDPT_E_INVALID, "colouring is not proper on coupling (" + std::to_string(i) + "," +
                                                std::to_string(col[e]) + ")");
    return TDPT_OK;
}

// Colour-major numbering (classes padded to multiples of 4), the problem
// ELL and the fields of a validated instance.
int lay_out(tdpt_instance *in, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
            const int32_t *b_q, const int32_t *color, int32_t C)
{
    in->n = n;
    in->nnz = row_ptr[n];
    in->n_colors = C;
    std::vector<int32_t> size(C, 0);
    for (int32_t v = 0; v < n; ++v) size[color[v]]++;
    in->cls_start.assign(C + 1, 0);
    in->cls_live.assign(C, 0);
    for (int32_t c = 0; c < C; ++c) {
        in->cls_live[c] = in->cls_start[c] + size[c];
        in->cls_start[c + 1] = in->cls_start[c] + (size[c] + 3) / 4 * 4;
        in->max_class_quads = std::max(in->max_class_quads, (size[c] + 3) / 4);
    }
    const int32_t n_pad = in->cls_start[C];
    in->n_pad = n_pad;
    in->rank.assign(n, 0);
    in->orig.assign(n_pad, -1);
    {
        std::vector<int32_t> next(in->cls_start.begin(), in->cls_start.end() - 1);
        for (int32_t v = 0; v < n; ++v) {
            const int32_t r = next[color[v]]++;
            in->rank[v] = r;
            in->orig[r] = v;
        }
    }
    int32_t maxdeg = 0;
    for (int32_t i = 0; i < n; ++i) maxdeg = std::max(maxdeg, row_ptr[i + 1] - row_ptr[i]);
    in->max_deg = maxdeg;
    in->wd = ell_width(maxdeg);
    if (in->wd < 0) return fail(TDPT_E_INVALID, "a spin has more than 256 problem neighbours");
    const int32_t wd = in->wd;
    in->nb_idx.assign((size_t)wd * n_pad, n_pad);
    in->nb_J.assign((size_t)wd * n_pad, 0);
    in->bias.assign(n_pad, 0);
    bool narrow = (n_pad + 1 <= 65536);
    int64_t absf = 0;
    for (int32_t r = 0; r < n_pad; ++r) {
        const int32_t v = in->orig[r];
        if (v < 0) continue;
        int64_t field = b_q ? std::llabs((long long)b_q[v]) : 0, row_J = 0;
        int k = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e, ++k) {
            in->nb_idx[(size_t)k * n_pad + r] = in->rank[col[e]];
            in->nb_J[(size_t)k * n_pad + r] = J_q[e];
            field += std::llabs((long long)J_q[e]);
            row_J += std::llabs((long long)J_q[e]);
            in->max_abs_J = std::max(in->max_abs_J, (int64_t)std::llabs((long long)J_q[e]));
            if (J_q[e] < -32768 || J_q[e] > 32767) narrow = false;
            if (col[e] > v) absf += std::llabs((long long)J_q[e]);
        }
        if (b_q) {
            in->bias[r] = b_q[v];
            absf += std::llabs((long long)b_q[v]);
            if (b_q[v] != 0) in->has_bias = 1;
        }
        in->max_field = std::max(in->max_field, field);
        in->max_row_J = std::max(in->max_row_J, row_J);
    }
    in->abs_f_bound = absf;
    in->narrow = narrow ? 1 : 0;
    return TDPT_OK;
}

// Wall time (ms) of n rounds enqueued by `enqueue` on `stream`.
int time_rounds(hipStream_t stream, const std::function<int()> &enqueue, double &ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    int rc = TDPT_OK;
    e = hipEventRecord(a, stream);
    if (e == hipSuccess) {
        rc = enqueue();
        if (rc == TDPT_OK) e = hipEventRecord(b, stream);
    }
    if (rc == TDPT_OK && e == hipSuccess) e = hipEventSynchronize(b);
    float f = 0.f;
    if (rc == TDPT_OK && e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    ms = f;
    return TDPT_OK;
}

}  // namespace

extern "C" {

const char *tdpt_last_error(void) { return g_err.c_str(); }

// The logical variable of every physical spin (values 0 .. N-1, each used):
// variable k is read from its lowest-numbered spin.
static int set_logical(tdpt_instance *in, const int32_t *logical_of)
{
    if (!logical_of) return TDPT_OK;
    const int32_t n = in->n;
    int32_t N = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (logical_of[v] < 0 || logical_of[v] >= n)
            return fail(TDPT_E_INVALID, "logical_of[" + std::to_string(v) + "] out of range");
        N = std::max(N, logical_of[v] + 1);
    }
    in->first_copy.assign(N, -1);
    for (int32_t v = n - 1; v >= 0; --v) in->first_copy[logical_of[v]] = v;
    for (int32_t k = 0; k < N; ++k)
        if (in->first_copy[k] < 0)
            return fail(TDPT_E_INVALID, "logical variable " + std::to_string(k) + " has no spin");
    in->first_rank.resize(N);
    for (int32_t k = 0; k < N; ++k) in->first_rank[k] = in->rank[in->first_copy[k]];
    in->n_logical = N;
    return TDPT_OK;
}

int tdpt_instance_create(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
                         const int32_t *b_q, int32_t m, const int32_t *copy_a,
                         const int32_t *copy_b, const int32_t *color, const int32_t *logical_of,
                         tdpt_instance **out)
{
    if (!out) return fail(TDPT_E_INVALID, "out is NULL");
    *out = nullptr;
    std::vector<std::pair<int32_t, int32_t>> ent;
    int rc = check_csr(n, row_ptr, col, J_q, b_q, color, ent);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!copy_a || !copy_b))) return fail(TDPT_E_INVALID, "bad copy-edge arrays");
    // copy edges
    std::vector<int32_t> cdeg(n, 0);
    std::vector<std::pair<int32_t, int32_t>> cpairs((size_t)m);
    for (int32_t e = 0; e < m; ++e) {
        const int32_t a = copy_a[e], b = copy_b[e];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b)
            return fail(TDPT_E_INVALID, "bad copy edge " + std::to_string(e));
        if (csr_has(row_ptr, ent, a, b))
            return fail(TDPT_E_INVALID, "copy edge " + std::to_string(e) + " is also a coupling");
        cpairs[e] = {std::min(a, b), std::max(a, b)};
        if (++cdeg[a] > 2 || ++cdeg[b] > 2)
            return fail(TDPT_E_INVALID, "copy constraints must form chains (at most 2 copy edges per spin)");
    }
    std::sort(cpairs.begin(), cpairs.end());
    for (int32_t e = 1; e < m; ++e)
        if (cpairs[e] == cpairs[e - 1]) return fail(TDPT_E_INVALID, "repeated copy edge");
    int32_t C = 0;
    rc = check_colors(n, row_ptr, col, color, C);
    if (rc) return rc;
    for (int32_t e = 0; e < m; ++e)
        if (color[copy_a[e]] == color[copy_b[e]])
            return fail(TDPT_E_INVALID, "colouring is not proper on copy edge " + std::to_string(e));

    auto *in = new (std::nothrow) tdpt_instance();
    if (!in) return fail(TDPT_E_NOMEM, "host allocation failed");
    rc = lay_out(in, n, row_ptr, col, J_q, b_q, color, C);
    if (rc) {
        delete in;
        return rc;
    }
    in->m = m;
    in->max_copy_deg = 0;
    for (int32_t v = 0; v < n; ++v) in->max_copy_deg = std::max(in->max_copy_deg, cdeg[v]);
    const int32_t n_pad = in->n_pad;
    in->ch_idx.assign((size_t)2 * n_pad, n_pad);
    for (int32_t e = 0; e < m; ++e) {
        const int32_t a = in->rank[copy_a[e]], b = in->rank[copy_b[e]];
        int32_t *sa = (in->ch_idx[a] == n_pad) ? &in->ch_idx[a] : &in->ch_idx[(size_t)n_pad + a];
        *sa = b;
        int32_t *sb = (in->ch_idx[b] == n_pad) ? &in->ch_idx[b] : &in->ch_idx[(size_t)n_pad + b];
        *sb = a;
    }
    // half the penalty field is the copy sum (|.| <= 2); g <= 4 m
    in->max_cfield = 2;
    in->g_bound = 4 * (int64_t)m;
    rc = set_logical(in, logical_of);
    if (rc) {
        delete in;
        return rc;
    }
    *out = in;
    return TDPT_OK;
}

int tdpt_instance_create_terms(int32_t n, const int32_t *row_ptr, const int32_t *col,
                               const int32_t *J_q, const int32_t *b_q, int32_t n_terms,
                               const int32_t *term_ptr, const int32_t *term_idx,
                               const int32_t *term_coef, const int32_t *term_const,
                               const int32_t *color, const int32_t *logical_of, tdpt_instance **out)
{
    if (!out) return fail(TDPT_E_INVALID, "out is NULL");
    *out = nullptr;
    std::vector<std::pair<int32_t, int32_t>> ent;
    int rc = check_csr(n, row_ptr, col, J_q, b_q, color, ent);
    if (rc) return rc;
    if (n_terms < 0 || (n_terms > 0 && (!term_ptr || !term_idx || !term_coef || !term_const)))
        return fail(TDPT_E_INVALID, "bad constraint-term arrays");
    if (n_terms > 0 && term_ptr[0] != 0) return fail(TDPT_E_INVALID, "term_ptr[0] must be 0");
    for (int32_t t = 0; t < n_terms; ++t)
        if (term_ptr[t + 1] < term_ptr[t]) return fail(TDPT_E_INVALID, "term_ptr must be non-decreasing");
    // g = sum_t (sum_e a_e s_e + d_t)^2 = g0 - 2 sum_i kh_i s_i - 2 sum_{i<j} Kh_ij s_i s_j
    // with Kh_ij = -sum_t a_ti a_tj, kh_i = -sum_t a_ti d_t, g0 = sum_t (sum_e a_e^2 + d_t^2)
    std::vector<int32_t> seen(n, -1);
    std::vector<std::vector<std::pair<int32_t, int64_t>>> kh_pairs(n);
    std::vector<int64_t> kh(n, 0);
    __int128 g0 = 0;
    const __int128 kBig = (__int128)1 << 62;
    for (int32_t t = 0; t < n_terms; ++t) {
        const int32_t e0 = term_ptr[t], e1 = term_ptr[t + 1];
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t v = term_idx[e];
            if (v < 0 || v >= n) return fail(TDPT_E_INVALID, "term index out of range in term " + std::to_string(t));
            if (seen[v] == t) return fail(TDPT_E_INVALID, "spin repeated in term " + std::to_string(t));
            seen[v] = t;
            const int64_t a = term_coef[e];
            kh[v] -= a * (int64_t)term_const[t];
            g0 += (__int128)a * a;
            for (int32_t e2 = e0; e2 < e1; ++e2)
                if (e2 != e) kh_pairs[v].push_back({term_idx[e2], -a * (int64_t)term_coef[e2]});
            if (std::llabs((long long)kh[v]) >= ((int64_t)1 << 40))
                return fail(TDPT_E_RANGE, "constraint coefficients too large");
        }
        g0 += (__int128)term_const[t] * term_const[t];
        if (g0 >= kBig) return fail(TDPT_E_RANGE, "constant of g reaches 2^62");
    }
    // merge repeated pairs, drop zero weights
    int64_t max_cfield = 0, g_bound = (int64_t)g0;
    int32_t wcg = 0;
    for (int32_t v = 0; v < n; ++v) {
        auto &L = kh_pairs[v];
        std::sort(L.begin(), L.end());
        size_t w = 0;
        for (size_t i = 0; i < L.size();) {
            size_t j = i;
            int64_t sum = 0;
            while (j < L.size() && L[j].first == L[i].first) sum += L[j++].second;
            if (sum != 0) L[w++] = {L[i].first, sum};
            i = j;
        }
        L.resize(w);
        int64_t cf = std::llabs((long long)kh[v]);
        for (auto &pr : L) {
            if (pr.second < INT32_MIN || pr.second > INT32_MAX)
                return fail(TDPT_E_RANGE, "a pair weight of g exceeds int32");
            cf += std::llabs((long long)pr.second);
        }
        if (kh[v] < INT32_MIN || kh[v] > INT32_MAX) return fail(TDPT_E_RANGE, "a linear weight of g exceeds int32");
        if (cf >= ((int64_t)1 << 31)) return fail(TDPT_E_RANGE, "a penalty field can reach 2^31");
        max_cfield = std::max(max_cfield, cf);
        g_bound += 2 * cf;  // 2|kh_v| + sum_j 2|Kh_vj|: every pair counted from both ends
        if (g_bound >= ((int64_t)1 << 62)) return fail(TDPT_E_RANGE, "g can reach 2^62");
        wcg = std::max(wcg, (int32_t)L.size());
    }
    if (wcg > 1024) return fail(TDPT_E_INVALID, "a spin shares constraint terms with more than 1024 others");
    int32_t C = 0;
    rc = check_colors(n, row_ptr, col, color, C);
    if (rc) return rc;
    for (int32_t v = 0; v < n; ++v)
        for (auto &pr : kh_pairs[v])
            if (color[v] == color[pr.first])
                return fail(TDPT_E_INVALID, "colouring is not proper on the constraint pair (" + std::to_string(v) +
                                                "," + std::to_string(pr.first) + ")");

    auto *in = new (std::nothrow) tdpt_instance();
    if (!in) return fail(TDPT_E_NOMEM, "host allocation failed");
    rc = lay_out(in, n, row_ptr, col, J_q, b_q, color, C);
    if (rc) {
        delete in;
        return rc;
    }
    const int32_t n_pad = in->n_pad;
    in->gen = 1;
    in->n_terms = n_terms;
    in->max_cons_deg = wcg;
    in->wcg = std::max(4, (wcg + 3) / 4 * 4);
    in->cn_idx.assign((size_t)in->wcg * n_pad, n_pad);
    in->cn_w.assign((size_t)in->wcg * n_pad, 0);
    in->kh.assign(n_pad, 0);
    for (int32_t r = 0; r < n_pad; ++r) {
        const int32_t v = in->orig[r];
        if (v < 0) continue;
        auto L = kh_pairs[v];
        for (auto &pr : L) pr.first = in->rank[pr.first];
        std::sort(L.begin(), L.end());
        for (size_t k = 0; k < L.size(); ++k) {
            in->cn_idx[k * n_pad + r] = L[k].first;
            in->cn_w[k * n_pad + r] = (int32_t)L[k].second;
        }
        in->kh[r] = (int32_t)kh[v];
    }
    in->g0 = (int64_t)g0;
    in->max_cfield = max_cfield;
    in->g_bound = g_bound;
    if (int rc2 = set_logical(in, logical_of)) {
        delete in;
        return rc2;
    }
    *out = in;
    return TDPT_OK;
}

int tdpt_instance_info_get(const tdpt_instance *in, tdpt_instance_info *out)
{
    if (!in || !out) return fail(TDPT_E_INVALID, "NULL argument");
    out->n = in->n;
    out->n_pad = in->n_pad;
    out->n_colors = in->n_colors;
    out->max_degree = in->max_deg;
    out->max_copy_degree = in->max_copy_deg;
    out->narrow = in->narrow;
    out->nnz = in->nnz;
    out->m = in->m;
    out->n_terms = in->n_terms;
    out->max_constraint_degree = in->max_cons_deg;
    out->n_logical = in->n_logical;
    return TDPT_OK;
}

void tdpt_instance_destroy(tdpt_instance *in) { delete in; }

int tdpt_workspace_bytes(const tdpt_instance *in, const tdpt_run_cfg *cfg, size_t *bytes)
{
    if (!in || !bytes) return fail(TDPT_E_INVALID, "NULL argument");
    int rc = check_cfg(cfg);
    if (rc) return rc;
    int32_t hist_n = 0;
    rc = hist_vars(in, cfg, &hist_n);
    if (rc) return rc;
    *bytes = make_layout(in, cfg->n_beta, cfg->n_p, cfg->trace_cap, use_narrow(in, cfg), hist_n).total;
    return TDPT_OK;
}

int tdpt_problem_create(const tdpt_instance *in, const tdpt_run_cfg *cfg, void *dev_ws,
                        size_t ws_bytes, void *stream, tdpt_problem **out)
{
    if (!out) return fail(TDPT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!in) return fail(TDPT_E_INVALID, "instance is NULL");
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!dev_ws) return fail(TDPT_E_INVALID, "workspace is NULL");
    if (((uintptr_t)dev_ws) % 256) return fail(TDPT_E_INVALID, "workspace must be 256-byte aligned");
    const int32_t I = cfg->n_beta, J = cfg->n_p, R = I * J;
    const bool narrow = use_narrow(in, cfg);
    int32_t hist_n = 0;
    rc = hist_vars(in, cfg, &hist_n);
    if (rc) return rc;
    const Layout L = make_layout(in, I, J, cfg->trace_cap, narrow, hist_n);
    if (ws_bytes < L.total)
        return fail(TDPT_E_NOMEM, "workspace holds " + std::to_string(ws_bytes) + " bytes, needs " +
                                      std::to_string(L.total));
    // fixed-point bounds
    const int64_t pmax = cfg->p_q[J - 1];
    const int64_t hmax = in->max_field + 2 * pmax * in->max_cfield;  // |h| bound
    if (in->max_cfield > 0 && 2 * pmax > (((int64_t)1 << 31) / in->max_cfield))
        return fail(TDPT_E_RANGE, "local field can reach 2^31");
    if (hmax >= ((int64_t)1 << 31))
        return fail(TDPT_E_RANGE, "local field can reach 2^31");
    const bool bits = use_bits(in);
    const int64_t blk = bits ? sweep_block(in, false, tdpt::bits_block_cap(cfg->mcs_per_swap))
                             : std::min(sweep_block(in, false), sweep_block(in, true));
    // a lane's per-phase sums: of 2 |h| (f) and of 2 |c| (g) per spin, c the
    // half penalty field, which P = 0 leaves out of hmax
    const int64_t hb = std::max(hmax, in->max_cfield);
    const int64_t quads_per_thread = (in->max_class_quads + blk - 1) / blk;
    if (quads_per_thread * 4 * 2 * hb >= ((int64_t)1 << 31))
        return fail(TDPT_E_RANGE, "per-phase energy change can reach 2^31");
    // smallest workgroup (multiple of 64) keeping every lane's per-phase sums below 2^31
    const int32_t min_lanes = min_lanes_for(in, pmax);
    const int32_t min_block = std::max<int32_t>(64, (min_lanes + 63) / 64 * 64);
    if (in->g_bound > 0 && pmax > (((int64_t)1 << 51) / in->g_bound))
        return fail(TDPT_E_RANGE, "energy differences can reach 2^52");
    const int64_t ebound = in->abs_f_bound + pmax * in->g_bound;
    if (ebound >= ((int64_t)1 << 51)) return fail(TDPT_E_RANGE, "energy differences can reach 2^52");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
            "hipDeviceGetAttribute");
    const size_t lds_limit = std::max((size_t)lds_max, (size_t)65536) - 1024;
    int32_t bit_start[tdpt::kMaxColors + 1];
    bit_start[0] = 0;
    for (int c = 0; c < in->n_colors; ++c)
        bit_start[c + 1] = (int32_t)align_up((size_t)bit_start[c] + (in->cls_live[c] - in->cls_start[c]), 32);
    const int32_t n_words = bit_start[in->n_colors] / 32;
    if (bits && in->max_deg > 8)
        return fail(TDPT_E_INVALID, "the bit-packed layout takes at most 8 problem neighbours per spin");
    if (bits && in->max_abs_J >= ((int64_t)1 << 23))
        return fail(TDPT_E_RANGE, "the bit-packed layout takes couplings |J_q| < 2^23");
    if (bits && pmax >= ((int64_t)1 << 22))
        return fail(TDPT_E_RANGE, "the bit-packed layout takes penalties P_q < 2^22");
    if (bits ? (size_t)(n_words + 1) * 16 + 4096 > lds_limit : (size_t)L.stride > lds_limit)
        return fail(TDPT_E_INVALID, "a replica (" + std::to_string(in->n_pad) +
                                        " spins) does not fit the LDS of one workgroup");

    auto *p = new (std::nothrow) tdpt_problem();
    if (!p) return fail(TDPT_E_NOMEM, "host allocation failed");
    p->stream = (hipStream_t)stream;
    p->n = in->n;
    p->I = I;
    p->J = J;
    p->R = R;
    p->mcs = cfg->mcs_per_swap;
    p->rank = in->rank;
    p->min_block = min_block;
    p->min_lanes = min_lanes;
    p->stride_bytes = L.stride;
    p->max_class_quads = in->max_class_quads;
    p->ws = (uint8_t *)dev_ws;
    p->ws_bytes = ws_bytes;
    p->mut_off = 0;
    p->mut_bytes = L.mut_end;
    p->mbox_off = L.mbox;
    p->mbox_bytes = L.slot_key - L.mbox;
    p->trace_cap = cfg->trace_cap;
    p->fingerprint = ((uint64_t)in->n_pad << 40) ^ ((uint64_t)R << 20) ^ (uint64_t)L.total;

    tdpt::DevProblem &d = p->dp;
    uint8_t *ws = p->ws;
    d.n_pad = in->n_pad;
    d.stride = L.stride;
    d.n_colors = in->n_colors;
    d.wd = L.wd;
    d.narrow = narrow ? 1 : 0;
    d.has_bias = in->has_bias;
    d.block = bits ? sweep_block(in, false, tdpt::bits_block_cap(cfg->mcs_per_swap)) : sweep_block(in, false);
    d.rpb = 1;
    d.lshift = 0;
    d.spin = 0;
    if (!bits) default_pack(in->max_class_quads, p->min_lanes, L.stride, &d.rpb, &d.lshift);
    {
        // a problem alone is latency-bound unless its replicas fill the GPU
        int32_t r = 1, ls = 0;
        const char *es = getenv("TDPT_SPIN");
        if (!(es && es[0] == '0') &&
            spin_shape(narrow, in->gen != 0, bits, L.wd, in->max_class_quads, L.stride, &r, &ls) &&
            (round_waves(R, r, ls) <= kSpinWaves || (es && es[0] == '1'))) {
            d.rpb = r;
            d.lshift = ls;
            d.spin = 1;
        }
    }
    d.bits = bits ? 1 : 0;
    d.pair16 = use_pair16(in) ? 1 : 0;
    d.n_words = n_words;
    for (int c = 0; c <= in->n_colors; ++c) d.bit_start[c] = bit_start[c];
    d.nb_pos = bits ? (const int32_t *)(ws + L.nb_pos) : nullptr;
    d.ch_pos = bits ? (const int32_t *)(ws + L.ch_pos) : nullptr;
    d.h0 = bits ? (const int32_t *)(ws + L.h0) : nullptr;
    d.nb_J2 = bits ? (const uint32_t *)(ws + L.nb_J2) : nullptr;
    for (int c = 0; c <= in->n_colors; ++c) d.cls_start[c] = in->cls_start[c];
    for (int c = 0; c < in->n_colors; ++c) d.cls_live[c] = in->cls_live[c];
    d.nbi = narrow ? (const uint32_t *)(ws + L.nbi) : nullptr;
    d.nbj = narrow ? (const uint32_t *)(ws + L.nbj) : nullptr;
    d.chp = (narrow && !in->gen) ? (const uint32_t *)(ws + L.chp) : nullptr;
    d.nb_idx = narrow ? nullptr : (const int32_t *)(ws + L.nb_idx);
    d.nb_J = narrow ? nullptr : (const int32_t *)(ws + L.nb_J);
    d.ch_idx = (narrow || in->gen) ? nullptr : (const int32_t *)(ws + L.ch_idx);
    d.gen = in->gen;
    d.wcg = in->wcg;
    d.cn_idx = in->gen ? (const int32_t *)(ws + L.cn_idx) : nullptr;
    d.cn_w = in->gen ? (const int32_t *)(ws + L.cn_w) : nullptr;
    d.kh = in->gen ? (const int32_t *)(ws + L.kh) : nullptr;
    d.g0 = in->g0;
    d.bias = (const int32_t *)(ws + L.bias);
    d.orig = (const int32_t *)(ws + L.orig);
    d.I = I;
    d.J = J;
    d.R = R;
    d.mcs = cfg->mcs_per_swap;
    d.key0 = (uint32_t)cfg->seed;
    d.key1 = (uint32_t)(cfg->seed >> 32);
    d.flags = cfg->flags;
    d.has_target = cfg->has_target ? 1 : 0;
    d.f_target = cfg->f_target_q;
    d.trace_cap = cfg->trace_cap;
    d.beta = (const double *)(ws + L.beta);
    d.p_q = (const int32_t *)(ws + L.p_q);
    d.hdr = (int64_t *)(ws + L.hdr);
    d.states = (int8_t *)(ws + L.states);
    d.f = (int64_t *)(ws + L.f);
    d.g = (int64_t *)(ws + L.g);
    d.slot_pos = (int32_t *)(ws + L.slot_pos);
    d.pos_slot = (int32_t *)(ws + L.pos_slot);
    d.p_att = (int64_t *)(ws + L.p_att);
    d.p_acc = (int64_t *)(ws + L.p_acc);
    d.b_att = (int64_t *)(ws + L.b_att);
    d.b_acc = (int64_t *)(ws + L.b_acc);
    d.best_state = (int8_t *)(ws + L.best);
    d.trace_f = (int64_t *)(ws + L.trace_f);
    d.trace_g = (int64_t *)(ws + L.trace_g);
    d.mbox = (uint64_t *)(ws + L.mbox);
    d.slot_key = (int64_t *)(ws + L.slot_key);
    d.slot_best = (int8_t *)(ws + L.slot_best);
    d.hit_min = (int64_t *)(ws + L.hit_min);
    d.slot_mul = 1;
    d.slot_add = 0;
    if (const char *e = getenv("TDPT_SLOT_ORDER")) {
        // test hook "mul,add": another assignment of slots to persistent workgroups
        long a = 1, b = 0;
        if (sscanf(e, "%ld,%ld", &a, &b) == 2 && a >= 1 && b >= 0 && b < R && std::gcd((long)R, a) == 1) {
            d.slot_mul = (int32_t)(a % R == 0 ? 1 : a % R);
            d.slot_add = (int32_t)b;
        }
    }
    d.hist_n = hist_n;
    d.hist_rank = (const int32_t *)(ws + L.hist_rank);
    d.hist = (uint32_t *)(ws + L.hist);
    p->n_logical = in->n_logical;
    p->first_copy = in->first_copy;

    hipStream_t s = p->stream;
    auto cleanup = [&](int code) {
        delete p;
        return code;
    };
    // immutable structure
    hipError_t e = hipSuccess;
#define UP(dst, src, bytes)                                                        \
    do {                                                                           \
        e = hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, s);       \
        if (e == hipSuccess) e = hipStreamSynchronize(s);                          \
        if (e != hipSuccess) return cleanup(hip_fail(e, "upload"));                \
    } while (0)
    UP(ws + L.beta, cfg->beta, (size_t)I * 8);
    UP(ws + L.p_q, cfg->p_q, (size_t)J * 4);
    if (hist_n) UP(ws + L.hist_rank, in->first_rank.data(), (size_t)hist_n * 4);
    if (narrow) {
        // neighbour pairs (2k, 2k+1): indices as 16+16 bits, couplings as int16 pairs
        const int32_t n_pad = in->n_pad, wd = in->wd, pairs = L.wd / 2;
        auto idx_at = [&](int k, int32_t r) { return k < wd ? in->nb_idx[(size_t)k * n_pad + r] : n_pad; };
        auto j_at = [&](int k, int32_t r) { return k < wd ? in->nb_J[(size_t)k * n_pad + r] : 0; };
        std::vector<uint32_t> A((size_t)pairs * n_pad), B((size_t)pairs * n_pad);
        for (int k2 = 0; k2 < pairs; ++k2)
            for (int32_t r = 0; r < n_pad; ++r) {
                A[(size_t)k2 * n_pad + r] = ((uint32_t)idx_at(2 * k2, r) & 0xffffu) |
                                            ((uint32_t)idx_at(2 * k2 + 1, r) << 16);
                B[(size_t)k2 * n_pad + r] = ((uint32_t)j_at(2 * k2, r) & 0xffffu) |
                                            ((uint32_t)(j_at(2 * k2 + 1, r) & 0xffff) << 16);
            }
        UP(ws + L.nbi, A.data(), A.size() * 4);
        UP(ws + L.nbj, B.data(), B.size() * 4);
        if (in->gen) {
            UP(ws + L.cn_idx, in->cn_idx.data(), in->cn_idx.size() * 4);
            UP(ws + L.cn_w, in->cn_w.data(), in->cn_w.size() * 4);
            UP(ws + L.kh, in->kh.data(), in->kh.size() * 4);
        } else {
            std::vector<uint32_t> ch((size_t)n_pad);
            for (int32_t r = 0; r < n_pad; ++r)
                ch[r] = ((uint32_t)in->ch_idx[r] & 0xffffu) | ((uint32_t)in->ch_idx[(size_t)n_pad + r] << 16);
            UP(ws + L.chp, ch.data(), ch.size() * 4);
        }
    } else {
        UP(ws + L.nb_idx, in->nb_idx.data(), in->nb_idx.size() * 4);
        UP(ws + L.nb_J, in->nb_J.data(), in->nb_J.size() * 4);
        if (in->gen) {
            UP(ws + L.cn_idx, in->cn_idx.data(), in->cn_idx.size() * 4);
            UP(ws + L.cn_w, in->cn_w.data(), in->cn_w.size() * 4);
            UP(ws + L.kh, in->kh.data(), in->kh.size() * 4);
        } else {
            UP(ws + L.ch_idx, in->ch_idx.data(), in->ch_idx.size() * 4);
        }
        if (bits) {
            // structure in bit positions: spin rho of class c sits at
            // rho - cls_start[c] + bit_start[c]
            const int32_t n_pad = in->n_pad;
            std::vector<int32_t> cls_of(n_pad, 0);
            for (int c = 0; c < in->n_colors; ++c)
                for (int32_t r = in->cls_start[c]; r < in->cls_start[c + 1]; ++r) cls_of[r] = c;
            // a bit position b is stored as 512 (b >> 5) + (b & 31) (plain
            // form) or 512 (b >> 5) + 256 ((b >> 4) & 1) + (b & 15) (pair
            // form): shifted right by 5 it is the LDS byte address of the
            // word group, or of the word pair, that holds the bit
            const bool pair = d.pair16 != 0;
            auto bitpos = [&](int32_t r) {
                const int32_t b = r - in->cls_start[cls_of[r]] + bit_start[cls_of[r]];
                return pair ? ((b >> 5) << 9) | (((b >> 4) & 1) << 8) | (b & 15) : ((b >> 5) << 9) | (b & 31);
            };
            std::vector<int32_t> pos(in->nb_idx.size()), chp(in->ch_idx.size()), h0(n_pad, 0);
            for (int k = 0; k < in->wd; ++k)
                for (int32_t r = 0; r < n_pad; ++r) {
                    const int32_t nb = in->nb_idx[(size_t)k * n_pad + r];
                    pos[(size_t)k * n_pad + r] = (nb == n_pad) ? 0 : bitpos(nb);
                    h0[r] -= in->nb_J[(size_t)k * n_pad + r];
                }
            for (int32_t r = 0; r < n_pad; ++r) h0[r] += in->bias[r];
            // copy neighbours: a missing one names bit 0 of the always-zero
            // word group n_words; row 0 also carries, in bits 29..30, how
            // many of the spin's two copy neighbours exist
            const int32_t zero_pos = n_words << 9;
            for (size_t i = 0; i < chp.size(); ++i)
                chp[i] = (in->ch_idx[i] == n_pad) ? zero_pos : bitpos(in->ch_idx[i]);
            for (int32_t r = 0; r < n_pad; ++r) {
                const int32_t kc = (in->ch_idx[r] != n_pad) + (in->ch_idx[(size_t)n_pad + r] != n_pad);
                chp[r] |= kc << 29;
            }
            // pair form: 2 J as a 16-bit number in both halves
            std::vector<uint32_t> j2(in->nb_J.size());
            for (size_t i = 0; i < j2.size(); ++i) j2[i] = ((uint32_t)(2 * in->nb_J[i]) & 0xffffu) * 0x10001u;
            UP(ws + L.nb_pos, pos.data(), pos.size() * 4);
            UP(ws + L.ch_pos, chp.data(), chp.size() * 4);
            UP(ws + L.h0, h0.data(), h0.size() * 4);
            UP(ws + L.nb_J2, j2.data(), j2.size() * 4);
        }
    }
    UP(ws + L.bias, in->bias.data(), in->bias.size() * 4);
    UP(ws + L.orig, in->orig.data(), in->orig.size() * 4);
    // mutable state: cleared on the device (states and best-state copies
    // are most of the workspace), then the few words that start non-zero
    {
        if (cfg->s0)
            for (size_t i = 0; i < (size_t)R * in->n; ++i)
                if (cfg->s0[i] != 1 && cfg->s0[i] != -1) return cleanup(fail(TDPT_E_INVALID, "s0 must be +-1"));
        e = hipMemsetAsync(ws, 0, L.scratch_end, s);
        if (e != hipSuccess) return cleanup(hip_fail(e, "clear workspace"));
        std::vector<int64_t> hdr(tdpt::kHdrWords, 0);
        hdr[tdpt::kHdrRounds] = 0;
        hdr[tdpt::kHdrFirstHit] = -1;
        hdr[tdpt::kHdrBestF] = INT64_MAX;
        hdr[tdpt::kHdrBestSweep] = -1;
        UP(ws + L.hdr, hdr.data(), hdr.size() * 8);
        std::vector<int32_t> ids(R);
        for (int32_t r = 0; r < R; ++r) ids[r] = r;
        UP(ws + L.slot_pos, ids.data(), ids.size() * 4);
        UP(ws + L.pos_slot, ids.data(), ids.size() * 4);
        if (cfg->s0) {
            // about 16 MB of replicas per upload (padding bytes stay zero)
            const int32_t per = (int32_t)std::max<size_t>(1, ((size_t)16 << 20) / (size_t)L.stride);
            std::vector<int8_t> st((size_t)std::min(per, R) * L.stride, 0);
            for (int32_t r0 = 0; r0 < R; r0 += per) {
                const int32_t nr = std::min(per, R - r0);
                for (int32_t r = 0; r < nr; ++r) {
                    const int8_t *src = cfg->s0 + (size_t)(r0 + r) * in->n;
                    int8_t *dst = st.data() + (size_t)r * L.stride;
                    for (int32_t v = 0; v < in->n; ++v) dst[in->rank[v]] = src[v];
                }
                UP(ws + L.states + (size_t)r0 * L.stride, st.data(), (size_t)nr * L.stride);
            }
        }
    }
#undef UP
    if (!cfg->s0) {
        e = tdpt::launch_init_states(d, s);
        if (e != hipSuccess) return cleanup(hip_fail(e, "init states"));
    }
    e = tdpt::launch_energy(d, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "initial energies"));
    // the persistent driver needs every slot's block resident at once
    p->persistent = false;
    const char *pe = getenv("TDPT_PERSISTENT");
    // its best-state keys need |f| < 2^30, its mailboxes carry f and g in 48 bits
    p->persistent_ok = !(pe && pe[0] == '0') && !bits && in->abs_f_bound < tdpt::kKeyOffset &&
                       in->g_bound < ((int64_t)1 << 47);
    // small bipartite replicas whose structure the packed per-round sweep
    // holds in registers run that driver when rounds are long enough
    // (TDPT_PERSISTENT=1 asks for the persistent driver wherever it fits)
    const bool prefer_round = ((d.spin && d.n_colors <= 4) || (d.rpb > 1 && pack_hoists(d, in->max_class_quads, d.lshift))) &&
                              cfg->mcs_per_swap >= kPackRoundMcs && !(pe && pe[0] == '1');
    if (p->persistent_ok && !prefer_round) {
        tdpt::DevProblem dq = d;
        dq.block = sweep_block(in, true);
        int max_blocks = 0;
        e = tdpt::persistent_max_blocks(dq, &max_blocks);
        if (e != hipSuccess) return cleanup(hip_fail(e, "occupancy query"));
        if (max_blocks >= R) {
            p->persistent = true;
            d.block = dq.block;
        }
    }
    *out = p;
    return TDPT_OK;
}

// Structure layout of a problem, which selects its sweep kernel instance:
// problems of one batch group share it.
struct GroupKey {
    int bits, narrow, packed_gen, wd, pair16;
    bool operator==(const GroupKey &o) const
    {
        return bits == o.bits && narrow == o.narrow && packed_gen == o.packed_gen && wd == o.wd &&
               pair16 == o.pair16;
    }
    // batch order: int8 before bit-packed, packed before wide, copy edges
    // before general constraints, narrower rows first
    bool operator<(const GroupKey &o) const
    {
        if (bits != o.bits) return bits < o.bits;
        if (narrow != o.narrow) return narrow > o.narrow;
        if (packed_gen != o.packed_gen) return packed_gen < o.packed_gen;
        if (wd != o.wd) return wd < o.wd;
        return pair16 > o.pair16;
    }
    int32_t code() const { return bits | narrow << 1 | packed_gen << 2 | wd << 3 | pair16 << 12; }
};

static GroupKey group_key(const tdpt::DevProblem &d)
{
    return GroupKey{d.bits ? 1 : 0, d.narrow ? 1 : 0, (d.narrow && d.gen) ? 1 : 0, d.wd, d.pair16 ? 1 : 0};
}

// Membership of problems in batches (defined with the batches below).
static int member_busy(tdpt_problem *p);
static void leave_batch(tdpt_problem *p);

// Record a timing event pair around the next launch if it is sampled.
static int timing_begin(tdpt_problem *p, std::pair<hipEvent_t, hipEvent_t> &ev, bool &timed)
{
    timed = p->time_every > 0 && p->sweep_launches % p->time_every == 0 &&
            p->events.size() < kMaxTimedLaunches;
    if (!timed) return TDPT_OK;
    HIP_TRY(hipEventCreate(&ev.first), "hipEventCreate");
    HIP_TRY(hipEventCreate(&ev.second), "hipEventCreate");
    p->events.push_back(ev);
    HIP_TRY(hipEventRecord(ev.first, p->stream), "hipEventRecord");
    return TDPT_OK;
}

int tdpt_problem_run(tdpt_problem *p, int64_t n_rounds)
{
    if (!p) return fail(TDPT_E_INVALID, "problem is NULL");
    if (n_rounds < 0) return fail(TDPT_E_INVALID, "n_rounds must be >= 0");
    if (int rc = member_busy(p)) return rc;
    // the sweep index is a 32-bit Philox counter word
    if ((p->rounds_host + n_rounds) * (int64_t)p->mcs > ((int64_t)1 << 32))
        return fail(TDPT_E_RANGE, "a problem runs at most 2^32 sweeps");
    if (n_rounds == 0) return TDPT_OK;
    if (p->persistent) {
        if (p->mbox_round != p->rounds_host)
            HIP_TRY(hipMemsetAsync(p->ws + p->mbox_off, 0, p->mbox_bytes, p->stream), "clear mailboxes");
        HIP_TRY(tdpt::launch_scratch_reset(p->dp, p->stream), "launch scratch reset");
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        bool timed;
        int rc = timing_begin(p, ev, timed);
        if (rc) return rc;
        hipError_t e = tdpt::launch_persistent(p->dp, n_rounds, p->stream);
        if (e != hipSuccess) return hip_fail(e, "launch persistent");
        if (timed) {
            HIP_TRY(hipEventRecord(ev.second, p->stream), "hipEventRecord");
            p->timed_rounds += n_rounds;
        }
        ++p->sweep_launches;
        HIP_TRY(tdpt::launch_finalize(p->dp, n_rounds, p->stream), "launch finalize");
        p->rounds_host += n_rounds;
        p->mbox_round = p->rounds_host;
        return TDPT_OK;
    }
    for (int64_t r = 0; r < n_rounds; ++r) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        bool timed;
        int rc = timing_begin(p, ev, timed);
        if (rc) return rc;
        hipError_t e = p->dp.bits ? tdpt::launch_sweep_bits(p->dp, p->stream)
                                  : tdpt::launch_sweep(p->dp, p->stream);
        if (e != hipSuccess) return hip_fail(e, "launch sweep");
        if (timed) {
            HIP_TRY(hipEventRecord(ev.second, p->stream), "hipEventRecord");
            p->timed_rounds += 1;
        }
        ++p->sweep_launches;
        e = tdpt::launch_swap(p->dp, p->stream);
        if (e != hipSuccess) return hip_fail(e, "launch swap");
    }
    p->rounds_host += n_rounds;
    return TDPT_OK;
}

int tdpt_problem_set_timing(tdpt_problem *p, int32_t every)
{
    if (!p || every < 0) return fail(TDPT_E_INVALID, "bad argument");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    p->events.clear();
    p->time_every = every;
    p->sweep_launches = 0;
    p->timed_rounds = 0;
    return TDPT_OK;
}

int tdpt_problem_read_timing(tdpt_problem *p, double *total_ms, int64_t *launches, int64_t *rounds)
{
    if (!p || !total_ms || !launches || !rounds) return fail(TDPT_E_INVALID, "NULL argument");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    double total = 0.0;
    for (auto &e : p->events) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
        total += ms;
    }
    *launches = (int64_t)p->events.size();
    *total_ms = total;
    *rounds = p->timed_rounds;
    return TDPT_OK;
}

int tdpt_problem_autotune(tdpt_problem *p, int32_t rounds_per_trial, tdpt_tune_report *out)
{
    if (!p || !out) return fail(TDPT_E_INVALID, "NULL argument");
    if (rounds_per_trial < 1) return fail(TDPT_E_INVALID, "rounds_per_trial must be >= 1");
    if (int rc = member_busy(p)) return rc;
    constexpr int kMaxTrials = 32;
    // the trials run (temporarily) up to kMaxTrials * (1 + rounds_per_trial) rounds
    if ((p->rounds_host + kMaxTrials * (1 + (int64_t)rounds_per_trial)) * (int64_t)p->mcs > ((int64_t)1 << 32))
        return fail(TDPT_E_RANGE, "a problem runs at most 2^32 sweeps");
    // candidates: (driver, threads per workgroup, slots per workgroup, log2
    // of lanes per slot)
    struct Cand {
        int first, second, rpb, lshift, spin;
    };
    std::vector<Cand> cand;
    const int cap = p->dp.bits ? tdpt::bits_block_cap(p->mcs) : tdpt::kMaxBlock;
    const int quads = p->max_class_quads;
    // a spread of sizes plus the balanced one (its last pass over a class
    // nearly full)
    std::vector<int> per_round = {64, 128, 192, 256, 384, 512, 640, 768, 1024};
    const int bal = balanced_block(quads, cap);
    if (std::find(per_round.begin(), per_round.end(), bal) == per_round.end()) per_round.push_back(bal);
    std::sort(per_round.begin(), per_round.end());
    for (int b : per_round)
        if (b >= p->min_block && b <= cap && b <= std::max(64, (quads + 63) / 64 * 64)) cand.push_back({0, b, 1, 0, 0});
    // int8 replicas of a small largest class: several per workgroup of 64,
    // 128 or 256 threads, one to four passes over the class
    if (!p->dp.bits)
        for (int ls = 0; ls <= 5; ++ls) {
            const int lanes = 1 << ls;
            if (lanes < p->min_lanes || 4 * lanes < quads || (ls > 0 && lanes / 2 >= quads)) continue;
            for (int blk : {64, 128, 256})
                if (pack_fits(p->stride_bytes, blk >> ls)) cand.push_back({0, blk, blk >> ls, ls, 0});
        }
    // one spin per lane: one or two passes over the largest class
    if (p->dp.narrow && !p->dp.gen && !p->dp.bits && p->dp.wd <= 8)
        for (int ls = 2; ls <= 8; ++ls) {
            const int lanes = 1 << ls;
            if (lanes < 2 * quads || (ls > 2 && lanes / 2 >= 4 * quads)) continue;
            const int blk = std::max(64, lanes);
            if (blk <= tdpt::kMultiBlock && pack_fits(p->stride_bytes, blk >> ls)) cand.push_back({0, blk, blk >> ls, ls, 1});
        }
    if (p->persistent_ok) {
        for (int b = 64; b <= tdpt::kMaxBlock / 2; b += 64) {
            if (b < p->min_block || b > std::max(64, (quads + 63) / 64 * 64)) continue;
            tdpt::DevProblem dq = p->dp;
            dq.block = b;
            int max_blocks = 0;
            HIP_TRY(tdpt::persistent_max_blocks(dq, &max_blocks), "occupancy query");
            if (max_blocks >= p->R) cand.push_back({1, b, 1, 0, 0});
        }
    }
    if (cand.empty()) return fail(TDPT_E_INVALID, "no launch shape satisfies the problem's bounds");
    if (cand.size() > (size_t)kMaxTrials) cand.resize(kMaxTrials);
    // keep the state: every trial round is undone afterwards
    size_t bytes = 0;
    int rc = tdpt_problem_save(p, nullptr, &bytes);
    if (rc) return rc;
    std::vector<uint8_t> saved(bytes);
    rc = tdpt_problem_save(p, saved.data(), &bytes);
    if (rc) return rc;
    const bool old_persistent = p->persistent;
    const int old_block = p->dp.block, old_rpb = p->dp.rpb, old_lshift = p->dp.lshift, old_spin = p->dp.spin;
    const int32_t old_every = p->time_every;
    p->time_every = 0;
    memset(out, 0, sizeof(*out));
    double best = 1e300;
    int best_i = -1;
    for (size_t i = 0; i < cand.size() && rc == TDPT_OK; ++i) {
        p->persistent = cand[i].first == 1;
        p->dp.block = cand[i].rpb > 1 || cand[i].spin ? old_block : cand[i].second;
        p->dp.rpb = cand[i].rpb;
        p->dp.lshift = cand[i].lshift;
        p->dp.spin = cand[i].spin;
        rc = tdpt_problem_run(p, 1);  // warm-up
        double ms = 0.0;
        if (rc == TDPT_OK)
            rc = time_rounds(p->stream, [&] { return tdpt_problem_run(p, rounds_per_trial); }, ms);
        if (rc) break;
        const double per = ms / rounds_per_trial;
        out->trial_driver[i] = cand[i].first;
        out->trial_block[i] = cand[i].second;
        out->trial_slots[i] = cand[i].rpb;
        out->trial_spin[i] = cand[i].spin;
        out->trial_ms_per_round[i] = per;
        out->n_trials = (int32_t)i + 1;
        if (per < best) {
            best = per;
            best_i = (int)i;
        }
    }
    p->time_every = old_every;
    if (rc || best_i < 0) {
        p->persistent = old_persistent;
        p->dp.block = old_block;
        p->dp.rpb = old_rpb;
        p->dp.lshift = old_lshift;
        p->dp.spin = old_spin;
        (void)tdpt_problem_load(p, saved.data(), saved.size());
        return rc ? rc : fail(TDPT_E_DEVICE, "autotune timed nothing");
    }
    p->persistent = cand[best_i].first == 1;
    p->dp.block = cand[best_i].rpb > 1 || cand[best_i].spin ? old_block : cand[best_i].second;
    p->dp.rpb = cand[best_i].rpb;
    p->dp.lshift = cand[best_i].lshift;
    p->dp.spin = cand[best_i].spin;
    out->driver = cand[best_i].first;
    out->block = cand[best_i].second;
    out->slots = cand[best_i].rpb;
    out->spin = cand[best_i].spin;
    out->ms_per_round = best;
    return tdpt_problem_load(p, saved.data(), saved.size());
}

static int d2h(tdpt_problem *p, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "readback");
    return TDPT_OK;
}

int tdpt_problem_query(tdpt_problem *p, tdpt_status *out)
{
    if (!p || !out) return fail(TDPT_E_INVALID, "NULL argument");
    int64_t h[tdpt::kHdrWords];
    int rc = d2h(p, h, p->dp.hdr, sizeof(h));
    if (rc) return rc;
    if (h[tdpt::kHdrError] == 2)
        return fail(TDPT_E_DEVICE, "a sweep kernel found its LDS replica away from address 0 and did not run");
    if (h[tdpt::kHdrError] == 3)
        return fail(TDPT_E_DEVICE, "a bit-packed sweep kernel of the other form was launched and did not run");
    if (h[tdpt::kHdrError])
        return fail(TDPT_E_DEVICE, "a persistent launch gave up after 2 s waiting for a swap partner's "
                                   "mailbox (blocks not co-resident, or partners disagreeing on a swap)");
    out->rounds_done = h[tdpt::kHdrRounds];
    out->driver = p->persistent ? 1 : 0;
    out->slots = p->persistent ? 1 : std::max(p->dp.rpb, 1);
    out->spin = p->persistent ? 0 : p->dp.spin;
    out->sweeps_done = h[tdpt::kHdrRounds] * p->mcs;
    out->first_hit_sweep = h[tdpt::kHdrFirstHit];
    out->best_f_q = h[tdpt::kHdrBestF];
    out->best_sweep = h[tdpt::kHdrBestSweep];
    return TDPT_OK;
}

int tdpt_problem_read_perm(tdpt_problem *p, int32_t *pos_to_slot)
{
    if (!p || !pos_to_slot) return fail(TDPT_E_INVALID, "NULL argument");
    return d2h(p, pos_to_slot, p->dp.pos_slot, (size_t)p->R * 4);
}

int tdpt_problem_read_energies(tdpt_problem *p, int64_t *f_q, int64_t *g)
{
    if (!p) return fail(TDPT_E_INVALID, "NULL argument");
    std::vector<int32_t> ps(p->R);
    std::vector<int64_t> fs(p->R), gs(p->R);
    int rc = d2h(p, ps.data(), p->dp.pos_slot, (size_t)p->R * 4);
    if (!rc) rc = d2h(p, fs.data(), p->dp.f, (size_t)p->R * 8);
    if (!rc) rc = d2h(p, gs.data(), p->dp.g, (size_t)p->R * 8);
    if (rc) return rc;
    for (int32_t q = 0; q < p->R; ++q) {
        if (f_q) f_q[q] = fs[ps[q]];
        if (g) g[q] = gs[ps[q]];
    }
    return TDPT_OK;
}

int tdpt_problem_read_states(tdpt_problem *p, int8_t *s)
{
    if (!p || !s) return fail(TDPT_E_INVALID, "NULL argument");
    const size_t stride = (size_t)p->dp.stride;
    std::vector<int32_t> ps(p->R);
    std::vector<int8_t> st((size_t)p->R * stride);
    int rc = d2h(p, ps.data(), p->dp.pos_slot, (size_t)p->R * 4);
    if (!rc) rc = d2h(p, st.data(), p->dp.states, st.size());
    if (rc) return rc;
    for (int32_t q = 0; q < p->R; ++q) {
        const int8_t *src = st.data() + (size_t)ps[q] * stride;
        int8_t *dst = s + (size_t)q * p->n;
        for (int32_t v = 0; v < p->n; ++v) dst[v] = src[p->rank[v]];
    }
    return TDPT_OK;
}

int tdpt_problem_read_best(tdpt_problem *p, int8_t *s, int64_t *f_q, int64_t *sweep)
{
    if (!p) return fail(TDPT_E_INVALID, "NULL argument");
    int64_t h[tdpt::kHdrWords];
    int rc = d2h(p, h, p->dp.hdr, sizeof(h));
    if (rc) return rc;
    if (f_q) *f_q = h[tdpt::kHdrBestF];
    if (sweep) *sweep = h[tdpt::kHdrBestSweep];
    if (s) {
        std::vector<int8_t> st((size_t)p->dp.stride);
        rc = d2h(p, st.data(), p->dp.best_state, st.size());
        if (rc) return rc;
        for (int32_t v = 0; v < p->n; ++v) s[v] = st[p->rank[v]];
    }
    return TDPT_OK;
}

int tdpt_problem_read_counters(tdpt_problem *p, int64_t *p_att, int64_t *p_acc, int64_t *b_att,
                               int64_t *b_acc)
{
    if (!p) return fail(TDPT_E_INVALID, "NULL argument");
    const size_t np = (size_t)p->I * (p->J - 1), nb = (size_t)p->J * (p->I - 1);
    int rc = TDPT_OK;
    if (p_att && np) rc = d2h(p, p_att, p->dp.p_att, np * 8);
    if (!rc && p_acc && np) rc = d2h(p, p_acc, p->dp.p_acc, np * 8);
    if (!rc && b_att && nb) rc = d2h(p, b_att, p->dp.b_att, nb * 8);
    if (!rc && b_acc && nb) rc = d2h(p, b_acc, p->dp.b_acc, nb * 8);
    return rc;
}

int tdpt_problem_read_trace(tdpt_problem *p, int64_t *f_q, int64_t *g, int64_t *count)
{
    if (!p || !count) return fail(TDPT_E_INVALID, "NULL argument");
    int64_t h[tdpt::kHdrWords];
    int rc = d2h(p, h, p->dp.hdr, sizeof(h));
    if (rc) return rc;
    const int64_t c = std::min(h[tdpt::kHdrRounds], p->trace_cap);
    *count = c;
    if (c > 0 && f_q) rc = d2h(p, f_q, p->dp.trace_f, (size_t)c * 8);
    if (!rc && c > 0 && g) rc = d2h(p, g, p->dp.trace_g, (size_t)c * 8);
    return rc;
}

int tdpt_problem_set_stage_trace(tdpt_problem *p, uint64_t *dev_buf, int32_t rounds)
{
    if (!p) return fail(TDPT_E_INVALID, "problem is NULL");
    if (rounds < 0 || (rounds > 0 && !dev_buf)) return fail(TDPT_E_INVALID, "need a buffer for rounds > 0");
    if (int rc = member_busy(p)) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    p->dp.stage = rounds ? dev_buf : nullptr;
    p->dp.stage_cap = rounds;
    p->dp.stage_round0 = p->rounds_host;
    return TDPT_OK;
}

int tdpt_problem_read_best_logical(tdpt_problem *p, int8_t *x, int64_t *f_q, int64_t *sweep)
{
    if (!p) return fail(TDPT_E_INVALID, "NULL argument");
    if (x && p->n_logical == 0)
        return fail(TDPT_E_STATE, "the instance was created without logical_of");
    std::vector<int8_t> s(x ? (size_t)p->n : 0);
    int rc = tdpt_problem_read_best(p, x ? s.data() : nullptr, f_q, sweep);
    if (rc) return rc;
    if (x)
        for (int32_t k = 0; k < p->n_logical; ++k) x[k] = s[p->first_copy[k]];
    return TDPT_OK;
}

int tdpt_problem_read_histogram(tdpt_problem *p, uint32_t *counts, int64_t *samples)
{
    if (!p || !counts) return fail(TDPT_E_INVALID, "NULL argument");
    if (!p->dp.hist_n) return fail(TDPT_E_STATE, "the run configuration asked for no histogram");
    int64_t h[tdpt::kHdrWords];
    int rc = d2h(p, h, p->dp.hdr, sizeof(h));
    if (!rc) rc = d2h(p, counts, p->dp.hist, (size_t)4 << p->dp.hist_n);
    if (!rc && samples) *samples = h[tdpt::kHdrRounds];
    return rc;
}

int tdpt_problem_read_energies_async(tdpt_problem *p, int64_t *dev_f_q, int64_t *dev_g)
{
    if (!p || (!dev_f_q && !dev_g)) return fail(TDPT_E_INVALID, "NULL argument");
    HIP_TRY(tdpt::launch_gather_energies(p->dp, dev_f_q, dev_g, p->stream), "launch gather");
    return TDPT_OK;
}

int tdpt_problem_read_states_async(tdpt_problem *p, int8_t *dev_s)
{
    if (!p || !dev_s) return fail(TDPT_E_INVALID, "NULL argument");
    HIP_TRY(tdpt::launch_gather_states(p->dp, p->n, dev_s, p->stream), "launch gather");
    return TDPT_OK;
}

int tdpt_problem_read_best_async(tdpt_problem *p, int8_t *dev_s, int64_t *dev_f_sweep)
{
    if (!p || (!dev_s && !dev_f_sweep)) return fail(TDPT_E_INVALID, "NULL argument");
    if (dev_s) HIP_TRY(tdpt::launch_gather_best(p->dp, dev_s, p->stream), "launch gather");
    if (dev_f_sweep)
        HIP_TRY(hipMemcpyAsync(dev_f_sweep, p->dp.hdr + tdpt::kHdrBestF, 2 * sizeof(int64_t),
                               hipMemcpyDeviceToDevice, p->stream), "copy best");
    return TDPT_OK;
}

int tdpt_problem_query_async(tdpt_problem *p, int64_t *dev_words)
{
    if (!p || !dev_words) return fail(TDPT_E_INVALID, "NULL argument");
    static_assert(tdpt::kHdrRounds == 0 && tdpt::kHdrFirstHit == 1 && tdpt::kHdrBestF == 2 &&
                      tdpt::kHdrBestSweep == 3, "header word order");
    HIP_TRY(hipMemcpyAsync(dev_words, p->dp.hdr, 4 * sizeof(int64_t), hipMemcpyDeviceToDevice, p->stream),
            "copy status");
    return TDPT_OK;
}

int tdpt_layout_get(const tdpt_instance *in, const tdpt_run_cfg *cfg, tdpt_layout *out)
{
    if (!in || !out) return fail(TDPT_E_INVALID, "NULL argument");
    int rc = check_cfg(cfg);
    if (rc) return rc;
    const bool narrow = use_narrow(in, cfg);
    const Layout L = make_layout(in, cfg->n_beta, cfg->n_p, cfg->trace_cap, narrow, 0);
    out->bits = use_bits(in) ? 1 : 0;
    out->narrow = narrow ? 1 : 0;
    out->general = in->gen ? 1 : 0;
    out->ell_width = L.wd;
    out->pair16 = use_pair16(in) ? 1 : 0;
    out->group_key = GroupKey{out->bits, out->narrow, (narrow && in->gen) ? 1 : 0, L.wd, out->pair16}.code();
    // the per-round sweep's default shape, as tdpt_problem_create sets it
    // (without its environment overrides)
    int32_t rpb = 1, lshift = 0, srpb = 1, sls = 0;
    if (!out->bits)
        default_pack(in->max_class_quads, min_lanes_for(in, cfg->p_q[cfg->n_p - 1]), L.stride, &rpb, &lshift);
    const int R = cfg->n_beta * cfg->n_p;
    out->spin = spin_shape(narrow, in->gen != 0, out->bits != 0, L.wd, in->max_class_quads, L.stride, &srpb, &sls) &&
                        round_waves(R, srpb, sls) <= kSpinWaves
                    ? 1
                    : 0;
    if (out->spin) {
        rpb = srpb;
        lshift = sls;
    }
    out->slots = rpb;
    out->lanes = rpb > 1 || out->spin ? 1 << lshift : 0;
    out->held = (out->spin && in->n_colors <= 4) ||
                        (!out->spin && rpb > 1 &&
                         pack_hoists(narrow, in->gen != 0, out->bits != 0, in->has_bias != 0, L.wd, in->n_colors,
                                     in->max_class_quads, lshift))
                    ? 1
                    : 0;
    out->per_round = out->held && cfg->mcs_per_swap >= kPackRoundMcs ? 1 : 0;
    return TDPT_OK;
}

static const uint64_t kCkptMagic = 0x3154504454324454ull;  // "TD2TDPT1"

int tdpt_problem_save(tdpt_problem *p, void *host, size_t *bytes)
{
    if (!p || !bytes) return fail(TDPT_E_INVALID, "NULL argument");
    const size_t need = 16 + p->mut_bytes;
    if (!host) {
        *bytes = need;
        return TDPT_OK;
    }
    if (*bytes < need) return fail(TDPT_E_NOMEM, "checkpoint buffer too small");
    uint64_t head[2] = {kCkptMagic, p->fingerprint};
    memcpy(host, head, 16);
    *bytes = need;
    return d2h(p, (uint8_t *)host + 16, p->ws + p->mut_off, p->mut_bytes);
}

int tdpt_problem_load(tdpt_problem *p, const void *host, size_t bytes)
{
    if (!p || !host) return fail(TDPT_E_INVALID, "NULL argument");
    if (int rc = member_busy(p)) return rc;
    if (bytes != 16 + p->mut_bytes) return fail(TDPT_E_INVALID, "checkpoint size does not match the problem");
    uint64_t head[2];
    memcpy(head, host, 16);
    if (head[0] != kCkptMagic || head[1] != p->fingerprint)
        return fail(TDPT_E_INVALID, "checkpoint belongs to a different problem shape");
    hipError_t e = hipMemcpyAsync(p->ws + p->mut_off, (const uint8_t *)host + 16, p->mut_bytes,
                                  hipMemcpyHostToDevice, p->stream);
    // stale partner mailboxes of the rounds being replaced must not match
    if (e == hipSuccess) e = hipMemsetAsync(p->ws + p->mbox_off, 0, p->mbox_bytes, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint load");
    int64_t rounds = 0;
    memcpy(&rounds, (const uint8_t *)host + 16 + sizeof(int64_t) * tdpt::kHdrRounds, sizeof(rounds));
    p->rounds_host = rounds;
    p->mbox_round = rounds;
    return TDPT_OK;
}

// ------------------------------------------------ static workspace
// One workspace per GPU in a static device array, for callers that cannot
// allocate device memory.  Host code never passes the array's name to a
// kernel or copy: on the host it is only a stand-in for the symbol, and its
// device address (one per GPU) comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[TDPT_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];            // device address of `scratch` on each GPU
tdpt_problem *g_static_owner[kMaxDevices];  // the live problem holding it, if any
}  // namespace

int tdpt_problem_create_static(const tdpt_instance *in, const tdpt_run_cfg *cfg, void *stream,
                               tdpt_problem **out)
{
    if (!out) return fail(TDPT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!in) return fail(TDPT_E_INVALID, "instance is NULL");
    size_t need = 0;
    int rc = tdpt_workspace_bytes(in, cfg, &need);
    if (rc) return rc;
    if (need > (size_t)TDPT_STATIC_WORKSPACE_BYTES)
        return fail(TDPT_E_NOMEM, "the problem needs " + std::to_string(need) +
                                      " bytes of workspace; the static workspace holds " +
                                      std::to_string((size_t)TDPT_STATIC_WORKSPACE_BYTES));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TDPT_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr) % 256) return fail(TDPT_E_DEVICE, "static workspace address unusable");
        g_static_ptr[dev] = ptr;
    }
    if (g_static_owner[dev])
        return fail(TDPT_E_BUSY, "another problem holds this GPU's static workspace (destroy it first)");
    rc = tdpt_problem_create(in, cfg, g_static_ptr[dev], (size_t)TDPT_STATIC_WORKSPACE_BYTES, stream, out);
    if (rc) return rc;
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
    return TDPT_OK;
}

void tdpt_problem_destroy(tdpt_problem *p)
{
    if (!p) return;
    leave_batch(p);
    if (p->static_dev >= 0) {
        // the next holder clears the array on its own stream: let this one's work end first
        (void)hipStreamSynchronize(p->stream);
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[p->static_dev] == p) g_static_owner[p->static_dev] = nullptr;
    }
    delete p;
}

// ------------------------------------------------------------------ batches

struct tdpt_batch {
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    int32_t cap = 0;
    int block = 256;
    std::vector<tdpt_problem *> members;  // in table order
    struct Group {
        int first_member, count, blocks, prefix_off;
        size_t max_stride;
        int max_words;
        int block;      // threads per sweep workgroup of this group
        int min_block;  // smallest the members' per-phase bounds allow
        size_t plds;    // LDS of a persistent workgroup (largest member)
        int min_mcs;    // fewest sweeps per round among the members
        // per-round driver, int8 layouts: rpb > 1 packs rpb slots into one
        // workgroup of rpb << lshift threads (block then applies to the
        // persistent driver only)
        int rpb = 1, lshift = 0;
        int spin = 0;       // packed sweep with one spin per lane (rpb may then be 1)
        int replicas = 0;   // slots of all members (workgroups of the persistent driver)
        int max_quads = 0;  // largest colour class of any member, in quads
        int min_lanes = 1;  // fewest lanes per slot the members' per-phase bounds allow
    };
    std::vector<Group> groups;
    hipEvent_t done = nullptr;
    // HIP graph of graph_rounds rounds (0: launch every round directly),
    // captured on cap_stream and replayed on stream; rebuilt after any change
    // of members or launch shapes.
    int32_t graph_rounds = 0;
    // persistent driver: one cooperative launch per group runs many rounds
    // (every member's workgroups resident at once); else one launch pair per
    // round.  driver_mode -1 picks the persistent driver when it fits.
    int32_t driver_mode = -1;
    bool persistent = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    // per-round driver: the sweeps of different layout groups run side by
    // side on auxiliary streams (fork and join through events each round)
    static constexpr int kAux = 7;
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr, join[kAux] = {};
    // a member was destroyed or moved to another batch: the device table
    // names it, so runs wait for tdpt_batch_set_members
    bool stale = false;
    // the autotuner chose packed slots for some group: per-round launches
    // until the next tdpt_batch_set_members
    bool tuned_per_round = false;
    // workgroup prefix sums as last uploaded (they depend on the driver and
    // on the groups' slots per workgroup)
    std::vector<int32_t> prefix_host;
    void drop_graph()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    ~tdpt_batch()
    {
        if (done) (void)hipEventSynchronize(done);
        for (auto *p : members) p->batch = nullptr;
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (int k = 0; k < kAux; ++k) {
            if (aux[k]) (void)hipStreamDestroy(aux[k]);
            if (join[k]) (void)hipEventDestroy(join[k]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (done) (void)hipEventDestroy(done);
    }
};

static size_t batch_table_bytes(int32_t cap) { return align_up((size_t)cap * sizeof(tdpt::DevProblem), 256); }
// Batch workspace: the descriptor table, the members' block prefix sums, the
// caller's index of every table entry, and [cap][4] int64 status words.
static size_t batch_prefix_bytes(int32_t cap) { return align_up((size_t)(2 * cap + 1) * 4, 256); }
static size_t batch_order_off(int32_t cap) { return batch_table_bytes(cap) + batch_prefix_bytes(cap); }
static size_t batch_status_off(int32_t cap) { return batch_order_off(cap) + align_up((size_t)cap * 4, 256); }
static size_t batch_ws_bytes(int32_t cap) { return batch_status_off(cap) + align_up((size_t)cap * 32, 256); }

// TDPT_E_BUSY while the last run of the batch holding p has not finished.
static int member_busy(tdpt_problem *p)
{
    if (!p->batch) return TDPT_OK;
    const hipError_t e = hipEventQuery(p->batch->done);
    if (e == hipErrorNotReady)
        return fail(TDPT_E_BUSY, "the problem's batch has a run in flight (wait with a read or query call)");
    if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    return TDPT_OK;
}

// Take p out of its batch (after the batch's work in flight): the batch's
// device table still names p, so the batch needs new members before it runs.
static void leave_batch(tdpt_problem *p)
{
    tdpt_batch *b = p->batch;
    if (!b) return;
    (void)hipEventSynchronize(b->done);
    b->members.erase(std::remove(b->members.begin(), b->members.end(), p), b->members.end());
    b->stale = true;
    b->drop_graph();
    p->batch = nullptr;
}


// Workgroup prefix sums of every group for the current driver: per member
// its first workgroup within the group (bit-packed: 4 slots per workgroup;
// int8: one slot each, or rpb under packed per-round launches).
static std::vector<int32_t> batch_prefix(tdpt_batch *b)
{
    std::vector<int32_t> prefix;
    for (auto &g : b->groups) {
        g.prefix_off = (int)prefix.size();
        const int rpb = b->persistent ? 1 : g.rpb;
        int blocks = 0;
        for (int k = g.first_member; k < g.first_member + g.count; ++k) {
            const tdpt_problem *p = b->members[k];
            prefix.push_back(blocks);
            blocks += p->dp.bits ? (p->R + tdpt::kBitSlots - 1) / tdpt::kBitSlots : (p->R + rpb - 1) / rpb;
        }
        g.blocks = blocks;
    }
    return prefix;
}

// Recompute the prefix sums and upload them if they changed (after the
// batch's work in flight); a captured graph names the old launch shapes.
static int batch_sync_prefix(tdpt_batch *b)
{
    std::vector<int32_t> prefix = batch_prefix(b);
    if (prefix == b->prefix_host || prefix.empty()) {
        b->prefix_host.swap(prefix);
        return TDPT_OK;
    }
    b->drop_graph();
    b->prefix_host.clear();
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    HIP_TRY(hipMemcpyAsync(b->ws + batch_table_bytes(b->cap), prefix.data(), prefix.size() * 4,
                           hipMemcpyHostToDevice, b->stream),
            "upload batch prefix");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    b->prefix_host.swap(prefix);
    return TDPT_OK;
}

// Whether the persistent driver runs this batch: every member allows it, no
// group is bit-packed, the autotuner did not choose packed per-round
// launches, and each group's workgroups fit the GPU at once.  Then the
// prefix sums follow the choice.
static int batch_decide_mode(tdpt_batch *b)
{
    b->persistent = false;
    // every group packed with its structure in registers, every member's
    // rounds long enough: per-round launches (as for one such problem)
    bool prefer_round = !b->groups.empty();
    for (const auto &g : b->groups) {
        prefer_round = prefer_round && (g.rpb > 1 || g.spin) && g.min_mcs >= kPackRoundMcs;
        for (int k = g.first_member; prefer_round && k < g.first_member + g.count; ++k)
            prefer_round = g.spin ? b->members[k]->dp.n_colors <= 4 && 4 * b->members[k]->max_class_quads <= (1 << g.lshift)
                                  : pack_hoists(b->members[k]->dp, b->members[k]->max_class_quads, g.lshift);
    }
    const char *pe = getenv("TDPT_PERSISTENT");
    if (pe && pe[0] == '1') prefer_round = false;
    bool fits = !b->members.empty() && b->driver_mode != 0 && !b->tuned_per_round && !prefer_round;
    for (auto *p : b->members) fits = fits && p->persistent_ok;
    for (size_t gi = 0; fits && gi < b->groups.size(); ++gi) {
        const auto &g = b->groups[gi];
        const tdpt::DevProblem &d0 = b->members[g.first_member]->dp;
        if (d0.bits || g.block > tdpt::kMaxBlock / 2 || g.block < g.min_block) {
            fits = false;
            break;
        }
        int max_blocks = 0;
        HIP_TRY(tdpt::batch_persistent_max_blocks(d0, g.block, g.plds, &max_blocks), "occupancy query");
        fits = max_blocks >= g.replicas;
    }
    b->persistent = fits;
    return batch_sync_prefix(b);
}

// Default slots per workgroup of an int8 group under per-round launches:
// when its largest colour class takes under 64 lanes, one wave of 64 holds
// 64 / L slots, L the power of two covering that class (and the members'
// per-phase bounds); larger replicas keep one slot per workgroup.
// Default shape of a group's per-round sweep: one spin per lane while the
// whole batch's round stays within kSpinWaves waves (latency-bound), else
// several replicas per workgroup at one quad per lane (default_pack).
static void batch_default_pack(tdpt_batch *b, tdpt_batch::Group &g)
{
    const tdpt::DevProblem &d0 = b->members[g.first_member]->dp;
    g.rpb = 1;
    g.lshift = 0;
    g.spin = 0;
    if (d0.bits) return;
    const char *es = getenv("TDPT_BATCH_SPIN");
    const bool spin_ok = !(es && es[0] == '0') && d0.narrow && !d0.gen && d0.wd <= 8;
    if (const char *e = getenv("TDPT_BATCH_LANES")) {
        // test hook: lanes per slot (a power of two); the workgroup then holds
        // max(block, lanes) / lanes slots, block from TDPT_BATCH_BLOCK or 64;
        // TDPT_BATCH_SPIN=1 makes it one spin per lane (lanes >= 4)
        const int v = atoi(e);
        int ls = 0;
        while ((1 << ls) < v) ++ls;
        const bool spin = es && es[0] == '1' && spin_ok;
        const int need = spin ? std::max(4, 4 * g.min_lanes) : g.min_lanes;
        if (v >= 1 && (1 << ls) == v && v >= need && v <= tdpt::kMultiBlock) {
            const char *eb = getenv("TDPT_BATCH_BLOCK");
            const int blk = std::max(eb ? atoi(eb) : 64, v);
            const int r = blk / v;
            if (blk % v == 0 && (r >= 2 || spin) && blk <= tdpt::kMultiBlock && pack_fits(g.max_stride, r)) {
                g.rpb = r;
                g.lshift = ls;
                g.spin = spin ? 1 : 0;
            }
        }
        return;
    }
    default_pack(g.max_quads, g.min_lanes, g.max_stride, &g.rpb, &g.lshift);
    int32_t r = 1, ls = 0;
    if (spin_ok && spin_shape(true, false, false, d0.wd, g.max_quads, g.max_stride, &r, &ls)) {
        int64_t waves = 0;
        for (const auto *m : b->members) waves += round_waves(m->R, r, ls);
        if (waves <= kSpinWaves) {
            g.rpb = r;
            g.lshift = ls;
            g.spin = 1;
        }
    }
}

// n_rounds rounds of every member through the persistent driver.
static int enqueue_batch_persistent(tdpt_batch *b, int64_t n_rounds)
{
    const tdpt::DevProblem *table = (const tdpt::DevProblem *)b->ws;
    const int *prefix = (const int *)(b->ws + batch_table_bytes(b->cap));
    for (auto *p : b->members)
        if (p->mbox_round != p->rounds_host)
            HIP_TRY(hipMemsetAsync(p->ws + p->mbox_off, 0, p->mbox_bytes, b->stream), "clear mailboxes");
    for (const auto &g : b->groups) {
        const tdpt::DevProblem &d0 = b->members[g.first_member]->dp;
        hipError_t e = tdpt::launch_batch_scratch_reset(table + g.first_member, g.count, b->stream);
        if (e == hipSuccess)
            e = tdpt::launch_batch_persistent(d0, table + g.first_member, prefix + g.prefix_off, g.count, g.blocks,
                                              g.block, g.plds, n_rounds, b->stream);
        if (e == hipSuccess) e = tdpt::launch_batch_finalize(table + g.first_member, g.count, n_rounds, b->stream);
        if (e != hipSuccess) return hip_fail(e, "launch batch persistent");
    }
    return TDPT_OK;
}

// One round of every member: the sweep launch of each layout group, then the
// swap-and-track launch.
// Auxiliary streams and events for the groups' side-by-side sweeps.
static int batch_aux_init(tdpt_batch *b)
{
    const int n_aux = std::min((int)b->groups.size() - 1, tdpt_batch::kAux);
    if (n_aux <= 0) return TDPT_OK;
    if (!b->fork) HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
    for (int k = 0; k < n_aux; ++k) {
        if (!b->aux[k]) HIP_TRY(hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking), "hipStreamCreate");
        if (!b->join[k]) HIP_TRY(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming), "hipEventCreate");
    }
    return TDPT_OK;
}

static int enqueue_batch_round(tdpt_batch *b, hipStream_t s)
{
    const tdpt::DevProblem *table = (const tdpt::DevProblem *)b->ws;
    const int *prefix = (const int *)(b->ws + batch_table_bytes(b->cap));
    const int n_groups = (int)b->groups.size();
    const int n_aux = std::min(n_groups - 1, tdpt_batch::kAux);
    if (n_aux > 0) {
        int rc = batch_aux_init(b);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->fork, s), "hipEventRecord");
        for (int k = 0; k < n_aux; ++k) HIP_TRY(hipStreamWaitEvent(b->aux[k], b->fork, 0), "hipStreamWaitEvent");
    }
    // group 0 on the batch's stream, group g > 0 on auxiliary stream (g-1) mod kAux
    for (int gi = 0; gi < n_groups; ++gi) {
        const auto &g = b->groups[gi];
        hipStream_t gs = gi == 0 ? s : b->aux[(gi - 1) % tdpt_batch::kAux];
        const tdpt::DevProblem &d0 = b->members[g.first_member]->dp;
        hipError_t e = d0.bits ? tdpt::launch_batch_sweep_bits(d0, table + g.first_member, prefix + g.prefix_off,
                                                               g.count, g.blocks, g.block, g.max_words, g.min_mcs, gs)
                               : tdpt::launch_batch_sweep(d0, table + g.first_member, prefix + g.prefix_off,
                                                          g.count, g.blocks,
                                                          g.rpb > 1 || g.spin ? g.rpb << g.lshift : g.block,
                                                          g.max_stride, g.rpb, g.lshift, g.spin, gs);
        if (e != hipSuccess) return hip_fail(e, "launch batch sweep");
    }
    for (int k = 0; k < n_aux; ++k) {
        HIP_TRY(hipEventRecord(b->join[k], b->aux[k]), "hipEventRecord");
        HIP_TRY(hipStreamWaitEvent(s, b->join[k], 0), "hipStreamWaitEvent");
    }
    hipError_t e = tdpt::launch_batch_swap(table, (int)b->members.size(), s);
    if (e != hipSuccess) return hip_fail(e, "launch batch swap");
    return TDPT_OK;
}

// Capture graph_rounds rounds into b->graph (kernel launches only).
static int capture_batch_graph(tdpt_batch *b)
{
    b->drop_graph();
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    {
        int rc = batch_aux_init(b);
        if (rc) return rc;
    }
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    int rc = TDPT_OK;
    for (int32_t r = 0; r < b->graph_rounds && rc == TDPT_OK; ++r) rc = enqueue_batch_round(b, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return TDPT_OK;
}


int tdpt_batch_workspace_bytes(int32_t max_members, size_t *bytes)
{
    if (max_members < 1 || !bytes) return fail(TDPT_E_INVALID, "need max_members >= 1");
    *bytes = batch_ws_bytes(max_members);
    return TDPT_OK;
}

int tdpt_batch_create(int32_t max_members, void *dev_ws, size_t ws_bytes, void *stream, tdpt_batch **out)
{
    if (!out) return fail(TDPT_E_INVALID, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = tdpt_batch_workspace_bytes(max_members, &need);
    if (rc) return rc;
    if (!dev_ws || ((uintptr_t)dev_ws) % 256) return fail(TDPT_E_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(TDPT_E_NOMEM, "batch workspace too small");
    auto *b = new (std::nothrow) tdpt_batch();
    if (!b) return fail(TDPT_E_NOMEM, "host allocation failed");
    b->stream = (hipStream_t)stream;
    b->ws = (uint8_t *)dev_ws;
    b->cap = max_members;
    if (const char *e = getenv("TDPT_BATCH_BLOCK")) {
        const int v = atoi(e);
        if (v >= 64 && v <= tdpt::kMaxBlock && v % 64 == 0) b->block = v;
    }
    hipError_t e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipEventCreate");
    }
    *out = b;
    return TDPT_OK;
}

int tdpt_batch_set_members(tdpt_batch *b, tdpt_problem *const *probs, int32_t count)
{
    if (!b) return fail(TDPT_E_INVALID, "batch is NULL");
    if (count < 0 || count > b->cap || (count > 0 && !probs))
        return fail(TDPT_E_INVALID, "member count out of range");
    std::vector<tdpt_problem *> m(probs, probs + count);
    for (auto *p : m)
        if (!p) return fail(TDPT_E_INVALID, "NULL member");
    std::vector<tdpt_problem *> caller(m);
    {
        std::vector<tdpt_problem *> chk = m;
        std::sort(chk.begin(), chk.end());
        if (std::adjacent_find(chk.begin(), chk.end()) != chk.end())
            return fail(TDPT_E_INVALID, "a problem appears twice in the batch");
    }
    for (auto *p : m) HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    // On any failure below the batch is left empty (and its old members
    // released), never half replaced.
    auto empty_batch = [&]() {
        for (auto *p : b->members) p->batch = nullptr;
        b->members.clear();
        b->groups.clear();
        b->persistent = false;
        b->stale = false;
    };
    // group by structure layout (the sweep kernel instance), largest
    // replicas first
    std::stable_sort(m.begin(), m.end(), [&](const tdpt_problem *x, const tdpt_problem *y) {
        const GroupKey kx = group_key(x->dp), ky = group_key(y->dp);
        if (!(kx == ky)) return kx < ky;
        return x->dp.stride > y->dp.stride;
    });
    b->drop_graph();
    empty_batch();
    std::vector<tdpt_batch::Group> groups;
    std::vector<tdpt::DevProblem> table(m.size());
    for (size_t i = 0; i < m.size(); ++i) {
        table[i] = m[i]->dp;
        if (groups.empty() || !(group_key(m[i]->dp) == group_key(m[i - 1]->dp))) {
            tdpt_batch::Group g{(int)i, 0, 0, 0, 0, 0, 0, 64, 0, INT_MAX};
            groups.push_back(g);
        }
        auto &g = groups.back();
        g.min_block = std::max(g.min_block, m[i]->min_block);
        g.min_lanes = std::max(g.min_lanes, m[i]->min_lanes);
        g.max_quads = std::max(g.max_quads, m[i]->max_class_quads);
        g.replicas += m[i]->R;
        g.count += 1;
        g.max_stride = std::max(g.max_stride, (size_t)m[i]->dp.stride);
        g.max_words = std::max(g.max_words, m[i]->dp.n_words);
        g.plds = std::max(g.plds, tdpt::persistent_lds_bytes(m[i]->dp.stride, m[i]->I, m[i]->J));
        g.min_mcs = std::min(g.min_mcs, m[i]->mcs);
    }
    // every group runs one kernel instance over its members' descriptors:
    // refuse a group whose members would need different instances
    for (auto &g : groups)
        for (int k = g.first_member + 1; k < g.first_member + g.count; ++k)
            if (!(group_key(m[k]->dp) == group_key(m[g.first_member]->dp)))
                return fail(TDPT_E_INVALID, "internal: a batch group mixes structure layouts");
    for (auto &g : groups) {
        const int cap = m[g.first_member]->dp.bits ? tdpt::bits_block_cap(g.min_mcs) : tdpt::kMaxBlock;
        if (g.min_block > cap)
            return fail(TDPT_E_RANGE, "a member's per-phase energy bounds need a larger workgroup than "
                                      "the batched sweep allows");
        // per-round default: the batch's workgroup size for byte layouts; for
        // bit-packed groups the members' own (their sweep wants every thread
        // a compute unit can hold next to one 4-replica workgroup)
        int def = b->block;
        if (m[g.first_member]->dp.bits) {
            def = 64;
            for (int k = g.first_member; k < g.first_member + g.count; ++k) def = std::max(def, m[k]->dp.block);
        }
        g.block = std::min(std::max(def, g.min_block), cap);
    }
    // members that move here from another batch leave it first
    for (auto *p : m)
        if (p->batch && p->batch != b) leave_batch(p);
    b->members = m;
    b->groups = groups;
    b->tuned_per_round = false;
    b->prefix_host.clear();
    for (auto &g : b->groups) batch_default_pack(b, g);
    // the persistent driver when every group fits at once (with the members'
    // own workgroup sizes), else per-round launches with the batch default
    {
        std::vector<int> per_round_blocks;
        for (auto &g : b->groups) {
            per_round_blocks.push_back(g.block);
            int want = g.min_block;
            for (int k = g.first_member; k < g.first_member + g.count; ++k)
                want = std::max(want, b->members[k]->dp.block);
            g.block = std::min(want, tdpt::kMaxBlock / 2);
        }
        int rc = batch_decide_mode(b);
        if (rc == TDPT_OK && !b->persistent)
            for (size_t gi = 0; gi < b->groups.size(); ++gi) b->groups[gi].block = per_round_blocks[gi];
        if (rc) {
            b->members.clear();
            b->groups.clear();
            b->persistent = false;
            b->prefix_host.clear();
            return rc;
        }
    }
    if (!m.empty()) {
        // the caller's index of every table entry (for status reads in the caller's order)
        std::vector<int32_t> order(m.size());
        for (size_t i = 0; i < m.size(); ++i)
            order[i] = (int32_t)(std::find(caller.begin(), caller.end(), m[i]) - caller.begin());
        hipError_t e = hipMemcpyAsync(b->ws, table.data(), table.size() * sizeof(tdpt::DevProblem),
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->ws + batch_order_off(b->cap), order.data(), order.size() * 4,
                               hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) {
            b->members.clear();
            b->groups.clear();
            b->persistent = false;
            b->prefix_host.clear();
            return hip_fail(e, "upload batch table");
        }
    }
    for (auto *p : m) p->batch = b;
    return TDPT_OK;
}

int tdpt_batch_run(tdpt_batch *b, int64_t n_rounds)
{
    if (!b) return fail(TDPT_E_INVALID, "batch is NULL");
    if (n_rounds < 0) return fail(TDPT_E_INVALID, "n_rounds must be >= 0");
    if (b->stale)
        return fail(TDPT_E_STATE, "a member was destroyed or joined another batch: set the members again");
    if (n_rounds == 0 || b->members.empty()) return TDPT_OK;
    for (auto *p : b->members)
        if ((p->rounds_host + n_rounds) * (int64_t)p->mcs > ((int64_t)1 << 32))
            return fail(TDPT_E_RANGE, "a problem runs at most 2^32 sweeps");
    int64_t r = 0;
    if (b->persistent) {
        int rc = enqueue_batch_persistent(b, n_rounds);
        if (rc) return rc;
        r = n_rounds;
    }
    if (r < n_rounds && b->graph_rounds > 0 && n_rounds >= b->graph_rounds) {
        if (!b->graph) {
            int rc = capture_batch_graph(b);
            if (rc) return rc;
        }
        for (; r + b->graph_rounds <= n_rounds; r += b->graph_rounds)
            HIP_TRY(hipGraphLaunch(b->graph, b->stream), "hipGraphLaunch");
    }
    for (; r < n_rounds; ++r) {
        int rc = enqueue_batch_round(b, b->stream);
        if (rc) return rc;
    }
    HIP_TRY(hipEventRecord(b->done, b->stream), "hipEventRecord");
    for (auto *p : b->members) {
        HIP_TRY(hipStreamWaitEvent(p->stream, b->done, 0), "hipStreamWaitEvent");
        p->rounds_host += n_rounds;
        if (b->persistent) p->mbox_round = p->rounds_host;
    }
    return TDPT_OK;
}

int tdpt_batch_autotune(tdpt_batch *b, int32_t rounds_per_trial, tdpt_batch_tune_report *out)
{
    if (!b || !out) return fail(TDPT_E_INVALID, "NULL argument");
    if (rounds_per_trial < 1) return fail(TDPT_E_INVALID, "rounds_per_trial must be >= 1");
    memset(out, 0, sizeof(*out));
    if (b->members.empty()) return TDPT_OK;
    if (b->groups.size() > 32) return fail(TDPT_E_INVALID, "more than 32 layout groups");
    // keep every member's state: the trial rounds are undone afterwards
    std::vector<std::vector<uint8_t>> saved(b->members.size());
    for (size_t i = 0; i < b->members.size(); ++i) {
        size_t bytes = 0;
        int rc = tdpt_problem_save(b->members[i], nullptr, &bytes);
        if (rc) return rc;
        saved[i].resize(bytes);
        rc = tdpt_problem_save(b->members[i], saved[i].data(), &bytes);
        if (rc) return rc;
    }
    auto restore = [&]() {
        int rc = TDPT_OK;
        for (size_t i = 0; i < b->members.size() && rc == TDPT_OK; ++i) {
            HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
            rc = tdpt_problem_load(b->members[i], saved[i].data(), saved[i].size());
        }
        return rc;
    };
    const int sizes[] = {64, 128, 256, 512, 1024};
    int rc = TDPT_OK;
    const int32_t graph_rounds = b->graph_rounds;
    b->graph_rounds = 0;  // trials launch directly
    b->drop_graph();
    out->n_groups = (int32_t)b->groups.size();
    // candidates: one slot per workgroup of `block` threads (run by the
    // persistent driver when it fits), or, for int8 groups, rpb slots of
    // 2^lshift lanes in per-round workgroups of 64, 128 or 256 threads, from
    // 4 passes over the largest class down to one
    struct Cand {
        int block, rpb, lshift, spin;
    };
    std::vector<bool> packed(b->groups.size(), false);
    auto any_packed = [&]() { return std::find(packed.begin(), packed.end(), true) != packed.end(); };
    for (size_t gi = 0; gi < b->groups.size() && rc == TDPT_OK; ++gi) {
        auto &g = b->groups[gi];
        const bool bits = b->members[g.first_member]->dp.bits != 0;
        const int cap = bits ? tdpt::bits_block_cap(g.min_mcs) : tdpt::kMaxBlock;
        std::vector<Cand> cands;
        for (int sz : sizes)
            if (sz >= g.min_block && sz <= cap) cands.push_back({sz, 1, 0, 0});
        if (!bits)
            for (int ls = 0; ls <= 5; ++ls) {
                const int lanes = 1 << ls;
                if (lanes < g.min_lanes || 4 * lanes < g.max_quads || (ls > 0 && lanes / 2 >= g.max_quads)) continue;
                for (int blk : {64, 128, 256})
                    if (pack_fits(g.max_stride, blk >> ls)) cands.push_back({blk, blk >> ls, ls, 0});
            }
        // one spin per lane: one or two passes over the largest class
        const tdpt::DevProblem &d0 = b->members[g.first_member]->dp;
        if (!bits && d0.narrow && !d0.gen && d0.wd <= 8)
            for (int ls = 2; ls <= 8; ++ls) {
                const int lanes = 1 << ls;
                if (lanes < 2 * g.max_quads || lanes < 4 * g.min_lanes || (ls > 2 && lanes / 2 >= 4 * g.max_quads))
                    continue;
                const int blk = std::max(64, lanes);
                if (blk <= tdpt::kMultiBlock && pack_fits(g.max_stride, blk >> ls)) cands.push_back({blk, blk >> ls, ls, 1});
            }
        double best = 1e300;
        Cand best_c{g.block, g.rpb, g.lshift, g.spin};
        bool best_packed = packed[gi];
        const int keep_block = g.block;
        for (const Cand &c : cands) {
            if (out->n_trials >= 128) break;
            g.block = c.rpb > 1 || c.spin ? keep_block : c.block;
            g.rpb = c.rpb;
            g.lshift = c.lshift;
            g.spin = c.spin;
            packed[gi] = c.rpb > 1 || c.spin;
            b->tuned_per_round = any_packed();
            rc = batch_decide_mode(b);
            if (rc) break;
            rc = tdpt_batch_run(b, 1);  // warm-up
            double ms = 0.0;
            if (rc == TDPT_OK)
                rc = time_rounds(b->stream, [&] { return tdpt_batch_run(b, rounds_per_trial); }, ms);
            if (rc) break;
            const double per = ms / rounds_per_trial;
            const int t = out->n_trials++;
            out->trial_group[t] = (int32_t)gi;
            out->trial_block[t] = c.block;
            out->trial_slots[t] = c.rpb;
            out->trial_spin[t] = c.spin;
            out->trial_ms_per_round[t] = per;
            if (per < best) {
                best = per;
                best_c = c;
                best_packed = c.rpb > 1 || c.spin;
            }
        }
        g.block = best_packed ? keep_block : best_c.block;
        g.rpb = best_c.rpb;
        g.lshift = best_c.lshift;
        g.spin = best_c.spin;
        packed[gi] = best_packed;
        out->group_block[gi] = best_c.block;
        out->group_slots[gi] = best_c.rpb;
        out->group_spin[gi] = best_c.spin;
        out->group_ms_per_round[gi] = best;
    }
    b->tuned_per_round = any_packed();
    {
        const int rc1 = batch_decide_mode(b);
        if (rc == TDPT_OK) rc = rc1;
    }
    out->persistent = b->persistent ? 1 : 0;
    b->graph_rounds = graph_rounds;
    const int rc2 = restore();
    return rc ? rc : rc2;
}

int tdpt_batch_query_async(tdpt_batch *b, int64_t *dev_words)
{
    if (!b || !dev_words) return fail(TDPT_E_INVALID, "NULL argument");
    if (b->stale)
        return fail(TDPT_E_STATE, "a member was destroyed or joined another batch: set the members again");
    if (b->members.empty()) return TDPT_OK;
    HIP_TRY(tdpt::launch_batch_status((const tdpt::DevProblem *)b->ws, (int)b->members.size(),
                                      (const int32_t *)(b->ws + batch_order_off(b->cap)), dev_words, b->stream),
            "launch batch status");
    return TDPT_OK;
}

int tdpt_batch_query(tdpt_batch *b, int64_t *words)
{
    if (!b || !words) return fail(TDPT_E_INVALID, "NULL argument");
    if (b->members.empty() && !b->stale) return TDPT_OK;
    int64_t *dev = (int64_t *)(b->ws + batch_status_off(b->cap));
    int rc = tdpt_batch_query_async(b, dev);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(words, dev, b->members.size() * 32, hipMemcpyDeviceToHost, b->stream), "readback");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return TDPT_OK;
}

int tdpt_batch_set_driver(tdpt_batch *b, int32_t driver)
{
    if (!b) return fail(TDPT_E_INVALID, "batch is NULL");
    if (driver != -1 && driver != 0) return fail(TDPT_E_INVALID, "driver must be -1 (automatic) or 0 (per round)");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    b->driver_mode = driver;
    return batch_decide_mode(b);
}

int tdpt_batch_query_driver(tdpt_batch *b, int32_t *driver)
{
    if (!b || !driver) return fail(TDPT_E_INVALID, "NULL argument");
    *driver = b->persistent ? 1 : 0;
    return TDPT_OK;
}

int tdpt_batch_set_graph(tdpt_batch *b, int32_t rounds_per_graph)
{
    if (!b) return fail(TDPT_E_INVALID, "batch is NULL");
    if (rounds_per_graph < 0 || rounds_per_graph > 4096)
        return fail(TDPT_E_INVALID, "rounds_per_graph must be in [0, 4096]");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    b->drop_graph();
    b->graph_rounds = rounds_per_graph;
    return TDPT_OK;
}

void tdpt_batch_destroy(tdpt_batch *b) { delete b; }

}  // extern "C"
