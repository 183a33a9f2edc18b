// gfx950 kernels of the 2D parallel tempering library.
//
// Round structure (Algorithm 1): every replica performs mcs sweeps, f and g
// of its final state are known, one swap step runs, the bottom-right replica
// is recorded.  Replica configurations never move: a swap exchanges the
// position labels of two replica slots (pos_slot / slot_pos), which is the
// same as exchanging the configurations.
//
// Sweep layout: one workgroup owns RB replica slots and keeps their int8
// spins in LDS for the whole round.  Spins are numbered colour-major; a lane
// takes a quad of 4 consecutive spins of the current colour class, which
// share one Philox4x32-10 call and one 16-byte load per neighbour slot of
// the ELL structure.  Same-colour spins have no coupling between them, so
// updating a whole class in parallel equals updating it one spin at a time
// (chromatic Gibbs), and the workgroup barrier between classes keeps the
// sweep order.
#include "tdpt_internal.h"

#include <math.h>

namespace tdpt {

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
        const uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)m1;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ------------------------------------------------------- heat-bath decision
// The decision is the double-precision expression
//   +1  iff  (double)u < ldexp(1 / (1 + exp(-ldexp(beta * h, -11))), 32)
// i.e. P(+1) = sigma(2 beta h) with h in Q12.  The float path below decides
// exactly the same way whenever u is more than 2^16 away from the threshold
// (its error is below 2^15 on the 2^32 scale, see DESIGN notes on the
// margin), and defers to the double expression otherwise (probability about
// 2^-15 per update).
__device__ __attribute__((noinline)) int heat_bath_exact(double beta, int h, uint32_t u)
{
    const double x = ldexp(beta * (double)h, -11);
    const double p = 1.0 / (1.0 + exp(-x));
    return ((double)u < ldexp(p, 32)) ? 1 : -1;
}

__device__ __forceinline__ int heat_bath(int h, float cb, double beta, uint32_t u)
{
    const float y = (float)h * cb;  // x * log2(e), x = 2 beta h / 4096
    if (y > 46.0f) return 1;        // x > 31.8: threshold above 2^32 - 1
    if (y < -46.0f) return (u == 0u) ? heat_bath_exact(beta, h, u) : -1;
    const float e = __builtin_amdgcn_exp2f(-y);
    const float X = __builtin_amdgcn_rcpf(1.0f + e) * 4294967296.0f;
    const float uf = (float)u;
    if (uf < X - 65536.0f) return 1;
    if (uf >= X + 65536.0f) return -1;
    return heat_bath_exact(beta, h, u);
}

// ----------------------------------------------------------- block helpers
__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------ sweep kernel
template <bool NARROW, int WD, int RB>
__device__ __forceinline__ void sweep_quad(const DevProblem &P, int8_t *lds, int q, int live,
                                           uint32_t t, const uint32_t (&pos)[RB],
                                           const double (&beta)[RB], const float (&cb)[RB],
                                           const int (&twoP)[RB], int ns, int (&dfa)[RB],
                                           int (&dga)[RB])
{
    const int r0 = q * 4;
    int idx[WD][4];
    int jv[WD][4];
    int c0[4], c1[4];
    if constexpr (NARROW) {
#pragma unroll
        for (int k = 0; k < WD; ++k) {
            const uint4 e = reinterpret_cast<const uint4 *>(P.nbp + (size_t)k * P.n_pad)[q];
            idx[k][0] = e.x & 0xffff; jv[k][0] = (int)e.x >> 16;
            idx[k][1] = e.y & 0xffff; jv[k][1] = (int)e.y >> 16;
            idx[k][2] = e.z & 0xffff; jv[k][2] = (int)e.z >> 16;
            idx[k][3] = e.w & 0xffff; jv[k][3] = (int)e.w >> 16;
        }
        const uint4 c = reinterpret_cast<const uint4 *>(P.chp)[q];
        c0[0] = c.x & 0xffff; c1[0] = c.x >> 16;
        c0[1] = c.y & 0xffff; c1[1] = c.y >> 16;
        c0[2] = c.z & 0xffff; c1[2] = c.z >> 16;
        c0[3] = c.w & 0xffff; c1[3] = c.w >> 16;
    } else {
#pragma unroll
        for (int k = 0; k < WD; ++k) {
            const int4 a = reinterpret_cast<const int4 *>(P.nb_idx + (size_t)k * P.n_pad)[q];
            const int4 b = reinterpret_cast<const int4 *>(P.nb_J + (size_t)k * P.n_pad)[q];
            idx[k][0] = a.x; idx[k][1] = a.y; idx[k][2] = a.z; idx[k][3] = a.w;
            jv[k][0] = b.x; jv[k][1] = b.y; jv[k][2] = b.z; jv[k][3] = b.w;
        }
        const int4 a = reinterpret_cast<const int4 *>(P.ch_idx)[q];
        const int4 b = reinterpret_cast<const int4 *>(P.ch_idx + P.n_pad)[q];
        c0[0] = a.x; c0[1] = a.y; c0[2] = a.z; c0[3] = a.w;
        c1[0] = b.x; c1[1] = b.y; c1[2] = b.z; c1[3] = b.w;
    }
    const int4 bb = reinterpret_cast<const int4 *>(P.bias)[q];
    const int bias[4] = {bb.x, bb.y, bb.z, bb.w};

#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (r >= ns) break;
        int8_t *s = lds + r * P.stride;
        uint32_t u0 = (uint32_t)q, u1 = t, u2 = pos[r], u3 = 0u;
        philox10(u0, u1, u2, u3, P.key0, P.key1);
        const uint32_t u[4] = {u0, u1, u2, u3};
        const char4 old = *reinterpret_cast<const char4 *>(s + r0);
        const int so[4] = {old.x, old.y, old.z, old.w};
        int sn[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (r0 + j < live) {
                int hp = bias[j];
#pragma unroll
                for (int k = 0; k < WD; ++k) hp += jv[k][j] * (int)s[idx[k][j]];
                const int cs = (int)s[c0[j]] + (int)s[c1[j]];
                const int h = hp + twoP[r] * cs;
                sn[j] = heat_bath(h, cb[r], beta[r], u[j]);
                const int ds = sn[j] - so[j];
                dfa[r] -= ds * hp;
                dga[r] -= 2 * ds * cs;
            } else {
                sn[j] = so[j];
            }
        }
        *reinterpret_cast<char4 *>(s + r0) =
            make_char4((char)sn[0], (char)sn[1], (char)sn[2], (char)sn[3]);
    }
}

template <bool NARROW, int WD, int RB>
__global__ __launch_bounds__(kBlock) void k_round_sweep(DevProblem P)
{
    extern __shared__ __align__(16) int8_t lds[];
    __shared__ int64_t red[kBlock / 64][RB][2];
    const int tid = threadIdx.x;
    const int slot0 = blockIdx.x * RB;
    const int ns = min(RB, P.R - slot0);

    const int nvec = P.stride >> 4;
    for (int r = 0; r < ns; ++r) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.states + (size_t)(slot0 + r) * P.stride);
        uint4 *dst = reinterpret_cast<uint4 *>(lds + r * P.stride);
        for (int v = tid; v < nvec; v += kBlock) dst[v] = src[v];
    }
    const int64_t n_round = P.hdr[kHdrRounds] + 1;
    uint32_t pos[RB];
    double beta[RB];
    float cb[RB];
    int twoP[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int p = (r < ns) ? P.slot_pos[slot0 + r] : 0;
        const int i = p / P.J, j = p - (p / P.J) * P.J;
        pos[r] = (uint32_t)p;
        beta[r] = P.beta[i];
        cb[r] = (float)(beta[r] * (1.4426950408889634 / 2048.0));
        twoP[r] = 2 * P.p_q[j];
    }
    __syncthreads();

    int64_t df[RB], dg[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) { df[r] = 0; dg[r] = 0; }

    for (int k = 0; k < P.mcs; ++k) {
        const uint32_t t = (uint32_t)((n_round - 1) * P.mcs + k);
        for (int c = 0; c < P.n_colors; ++c) {
            const int q0 = P.cls_start[c] >> 2, q1 = P.cls_start[c + 1] >> 2;
            const int live = P.cls_live[c];
            int dfa[RB], dga[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) { dfa[r] = 0; dga[r] = 0; }
            for (int q = q0 + tid; q < q1; q += kBlock)
                sweep_quad<NARROW, WD, RB>(P, lds, q, live, t, pos, beta, cb, twoP, ns, dfa, dga);
#pragma unroll
            for (int r = 0; r < RB; ++r) { df[r] += dfa[r]; dg[r] += dga[r]; }
            __syncthreads();
        }
    }

    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int64_t a = wave_sum64(df[r]);
        const int64_t b = wave_sum64(dg[r]);
        if (lane == 0) { red[wave][r][0] = a; red[wave][r][1] = b; }
    }
    __syncthreads();
    if (tid < ns) {
        int64_t a = 0, b = 0;
        for (int w = 0; w < kBlock / 64; ++w) { a += red[w][tid][0]; b += red[w][tid][1]; }
        P.f[slot0 + tid] += a;
        P.g[slot0 + tid] += b;
    }
    for (int r = 0; r < ns; ++r) {
        uint4 *dst = reinterpret_cast<uint4 *>(P.states + (size_t)(slot0 + r) * P.stride);
        const uint4 *src = reinterpret_cast<const uint4 *>(lds + r * P.stride);
        for (int v = tid; v < nvec; v += kBlock) dst[v] = src[v];
    }
}

// -------------------------------------------------------------- swap kernel
__device__ __forceinline__ double philox_u53(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1)
{
    philox10(c0, c1, c2, c3, k0, k1);
    return ((double)(c0 >> 5) * 67108864.0 + (double)(c1 >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ bool metropolis(double x, double u)
{
    return x >= 0.0 || u <= exp(x);
}

// One swap step of Algorithm 1 plus bottom-right tracking; one workgroup.
__global__ __launch_bounds__(kBlock) void k_swap_track(DevProblem P)
{
    __shared__ int improved;
    __shared__ int br_slot;
    const int tid = threadIdx.x;
    const int64_t n = P.hdr[kHdrRounds] + 1;
    const int first = (n % 2 == 0) ? 1 : 0;
    const bool dir_beta = (P.flags & 1u) ? true : (((n - 1) / 2) % 2 == 1);
    if (!dir_beta) {
        const int per = (P.J - first) / 2;
        const int total = P.I * per;
        for (int w = tid; w < total; w += kBlock) {
            const int i = w / per, k = first + 2 * (w - (w / per) * per);
            const int a = i * P.J + k, b = a + 1;
            const int sa = P.pos_slot[a], sb = P.pos_slot[b];
            const int64_t dpg = ((int64_t)P.p_q[k + 1] - P.p_q[k]) * (P.g[sb] - P.g[sa]);
            const double x = ldexp(P.beta[i] * (double)dpg, -12);
            const double u = philox_u53((uint32_t)k, (uint32_t)n, (uint32_t)i, 1u, P.key0, P.key1);
            const int ci = i * (P.J - 1) + k;
            P.p_att[ci] += 1;
            if (metropolis(x, u)) {
                P.p_acc[ci] += 1;
                P.pos_slot[a] = sb; P.pos_slot[b] = sa;
                P.slot_pos[sb] = a; P.slot_pos[sa] = b;
            }
        }
    } else {
        const int per = (P.I - first) / 2;
        const int total = P.J * per;
        for (int w = tid; w < total; w += kBlock) {
            const int j = w / per, k = first + 2 * (w - (w / per) * per);
            const int a = k * P.J + j, b = a + P.J;
            const int sa = P.pos_slot[a], sb = P.pos_slot[b];
            const int64_t ea = P.f[sa] + (int64_t)P.p_q[j] * P.g[sa];
            const int64_t eb = P.f[sb] + (int64_t)P.p_q[j] * P.g[sb];
            const double dbeta = P.beta[k + 1] - P.beta[k];
            const double x = ldexp(dbeta * (double)(eb - ea), -12);
            const double u = philox_u53((uint32_t)k, (uint32_t)n, (uint32_t)j, 2u, P.key0, P.key1);
            const int ci = j * (P.I - 1) + k;
            P.b_att[ci] += 1;
            if (metropolis(x, u)) {
                P.b_acc[ci] += 1;
                P.pos_slot[a] = sb; P.pos_slot[b] = sa;
                P.slot_pos[sb] = a; P.slot_pos[sa] = b;
            }
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
    if (improved) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.states + (size_t)br_slot * P.stride);
        uint4 *dst = reinterpret_cast<uint4 *>(P.best_state);
        for (int v = tid; v < (P.stride >> 4); v += kBlock) dst[v] = src[v];
    }
    __syncthreads();
    if (tid == 0) P.hdr[kHdrRounds] = n;
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

// f = -sum_{i<j} J s_i s_j - sum b s and g = sum_copy (s_a - s_b)^2 of every
// slot, from scratch (one workgroup per slot).
__global__ __launch_bounds__(kBlock) void k_energy(DevProblem P)
{
    __shared__ int64_t red[kBlock / 64][2];
    const int slot = blockIdx.x;
    const int8_t *s = P.states + (size_t)slot * P.stride;
    int64_t f2 = 0, g2 = 0;
    for (int r = threadIdx.x; r < P.n_pad; r += blockDim.x) {
        const int si = s[r];
        if (si == 0) continue;
        int64_t hp = 0;
        for (int k = 0; k < P.wd; ++k) {
            int id, jv;
            if (P.narrow) {
                const uint32_t e = P.nbp[(size_t)k * P.n_pad + r];
                id = e & 0xffff; jv = (int)e >> 16;
            } else {
                id = P.nb_idx[(size_t)k * P.n_pad + r];
                jv = P.nb_J[(size_t)k * P.n_pad + r];
            }
            hp += (int64_t)jv * s[id];
        }
        f2 -= si * hp + 2 * (int64_t)P.bias[r] * si;
        int ca, cb;
        if (P.narrow) {
            const uint32_t c = P.chp[r];
            ca = c & 0xffff; cb = c >> 16;
        } else {
            ca = P.ch_idx[r]; cb = P.ch_idx[P.n_pad + r];
        }
        if (ca != P.n_pad) { const int d = si - s[ca]; g2 += d * d; }
        if (cb != P.n_pad) { const int d = si - s[cb]; g2 += d * d; }
    }
    const int64_t a = wave_sum64(f2), b = wave_sum64(g2);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[wave][0] = a; red[wave][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t fa = 0, ga = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { fa += red[w][0]; ga += red[w][1]; }
        P.f[slot] = fa / 2;
        P.g[slot] = ga / 2;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_init_states(const DevProblem &p, hipStream_t s)
{
    dim3 grid((p.stride + 255) / 256, p.R);
    hipLaunchKernelGGL(k_init_states, grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_energy(const DevProblem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(p.R), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

template <bool NARROW, int WD, int RB>
static hipError_t launch_sweep_t(const DevProblem &p, hipStream_t s)
{
    const size_t lds = (size_t)RB * p.stride;
    static bool attr_set = false;
    if (!attr_set && lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)k_round_sweep<NARROW, WD, RB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int blocks = (p.R + RB - 1) / RB;
    hipLaunchKernelGGL((k_round_sweep<NARROW, WD, RB>), dim3(blocks), dim3(kBlock), lds, s, p);
    return hipGetLastError();
}

template <bool NARROW, int RB>
static hipError_t launch_sweep_w(const DevProblem &p, hipStream_t s)
{
    switch (p.wd) {
    case 1: return launch_sweep_t<NARROW, 1, RB>(p, s);
    case 2: return launch_sweep_t<NARROW, 2, RB>(p, s);
    case 3: return launch_sweep_t<NARROW, 3, RB>(p, s);
    case 4: return launch_sweep_t<NARROW, 4, RB>(p, s);
    case 5: return launch_sweep_t<NARROW, 5, RB>(p, s);
    case 6: return launch_sweep_t<NARROW, 6, RB>(p, s);
    case 7: return launch_sweep_t<NARROW, 7, RB>(p, s);
    case 8: return launch_sweep_t<NARROW, 8, RB>(p, s);
    case 12: return launch_sweep_t<NARROW, 12, RB>(p, s);
    case 16: return launch_sweep_t<NARROW, 16, RB>(p, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(const DevProblem &p, int rb, hipStream_t s)
{
    if (p.narrow)
        return (rb == 1) ? launch_sweep_w<true, 1>(p, s)
             : (rb == 2) ? launch_sweep_w<true, 2>(p, s) : launch_sweep_w<true, 4>(p, s);
    return (rb == 1) ? launch_sweep_w<false, 1>(p, s)
         : (rb == 2) ? launch_sweep_w<false, 2>(p, s) : launch_sweep_w<false, 4>(p, s);
}

hipError_t launch_swap(const DevProblem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_track, dim3(1), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

}  // namespace tdpt
