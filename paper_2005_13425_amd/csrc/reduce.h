// Deterministic workgroup and grid reductions for gfx950 (wave64).
//
// A grid reduction writes one partial per workgroup.  Workgroups are grouped
// by RED_GROUP; the workgroup that takes the last ticket of its group sums the
// group's partials in index order, and the workgroup that finishes the last
// group sums the group sums (and any partials left by an earlier launch) in
// index order.  A grid of at most RED_ONE_LEVEL workgroups uses one level:
// the workgroup that takes the last ticket sums all partials in index order.  The order of every sum is fixed by the launch shape, so the
// result is bitwise reproducible.  Every counter sits on a cache line of its
// own: atomics on one line are serialised, and with the counters packed the
// reduction at the end of a 2048-workgroup launch took 3 us longer; groups of
// 16 rather than 32 took off another 0.5 us.
#pragma once

#include <hip/hip_runtime.h>

#include "addrspace.h"

namespace nek {

constexpr int RED_GROUP = 16;          // workgroups per first-level ticket
constexpr int RED_MAX_BLOCKS = 2048;   // grid cap of the reduction kernels
constexpr int RED_MAX_GROUPS = RED_MAX_BLOCKS / RED_GROUP;
constexpr int RED_TICKET_STRIDE = 32;  // counters 128 bytes apart
// grids of at most this many workgroups take one ticket level: the second
// level's store, ticket and loads cost more than the contention of every
// workgroup on one counter there (the assemble-update at N = 9: 1.0-1.1 us
// less with 80 to 280 workgroups, 1.1 us more with 528, 7 us more with 1016)
#ifndef NEK_RED_ONE_LEVEL
#define NEK_RED_ONE_LEVEL 384
#endif
constexpr unsigned int RED_ONE_LEVEL = NEK_RED_ONE_LEVEL;
constexpr int RED_TICKETS = (1 + RED_MAX_GROUPS) * RED_TICKET_STRIDE;   // words per reduction site

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a workgroup of NT threads (multiple of 64); valid in thread 0.
// lds must hold NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += lds[q];
    }
    __syncthreads();
    return s;
}

// Sum over the NT threads [base, base + NT) of a workgroup that holds several
// independent parts (NT and base multiples of 64); valid in thread base.  lds
// must hold one double per wave of the whole workgroup, and every thread of
// the workgroup calls it (two barriers).  For base = 0 in a workgroup of NT
// threads it is block_sum<NT>, operation for operation.
template <int NT>
__device__ __forceinline__ double seg_sum(double v, double *lds, int base) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x == base) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += lds[base / 64 + q];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ double load_coherent(gptr<const double> p) {
    unsigned long long bits =
        __hip_atomic_load((gptr<const unsigned long long>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)bits);
}

__device__ __forceinline__ void store_coherent(gptr<double> p, double v) {
    __hip_atomic_store((gptr<unsigned long long>)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Agent-scope ticket: the caller's coherent stores have completed first.
__device__ __forceinline__ unsigned int take_ticket(gptr<unsigned int> t) {
    __builtin_amdgcn_s_waitcnt(0);
    return __hip_atomic_fetch_add(t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Storage of one reduction site (all device memory), for up to RED_MAX_SUMS
// sums reduced together (component c of workgroup lb at part[lb*K + c]):
//   part[K * gridDim.x]   per-workgroup partials
//   gpart[K * groups]     per-group sums
//   tk[RED_TICKETS]       zero-initialised counters, RED_TICKET_STRIDE words
//                         apart (reset after use)
//   extra[nextra]         partials written by an earlier launch, added last
//                         to the first sum
constexpr int RED_MAX_SUMS = 2;

struct RedSite {
    double *part;
    double *gpart;
    unsigned int *tk;
    const double *extra;
    long nextra;
};

// Publish K sums s[0..K) (valid in thread 0).  Returns true in every thread of
// the one workgroup that completes the reduction; thread 0 of it has the
// totals in out[0..K).
//
// Partials go out with agent-scope atomic stores (through the per-XCD L2 to
// the device-coherent level) and each thread waits for its stores before it
// takes a ticket; readers use agent-scope atomic loads.  No agent-scope fence
// is used: on gfx950 such a fence writes back the whole L2 of the XCD.
//
// lb / nb: this workgroup's index and the number of workgroups taking part
// (blockIdx.x / gridDim.x for a plain launch, the slot-local values in a
// launch that serves several solves).  Every component is summed in the same
// fixed order, so K = 1 and the first component of K = 2 agree bitwise.
template <int NT, int K>
__device__ bool grid_finish_k(const double *s, const RedSite &r, double *out, double *lds,
                              unsigned int lb, unsigned int nb) {
    static_assert(K >= 1 && K <= RED_MAX_SUMS, "at most RED_MAX_SUMS sums per site");
    static_assert(NT >= RED_GROUP, "one thread per partial of a group");
    __shared__ int stage;   // 0: not last, 1: last of its group, 2: last overall
    const gptr<double> part = (gptr<double>)r.part;
    const gptr<double> gpart = (gptr<double>)r.gpart;
    const gptr<unsigned int> tk = (gptr<unsigned int>)r.tk;
    const gptr<const double> extra = (gptr<const double>)r.extra;
    if (nb <= RED_ONE_LEVEL) {
        // one level: every workgroup takes a ticket on the top counter, the
        // last sums all partials in index order
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < K; ++c) store_coherent(part + (size_t)lb * K + c, s[c]);
            const unsigned int t = take_ticket(tk);
            stage = (t == nb - 1u) ? 2 : 0;
        }
        __syncthreads();
        if (stage != 2) return false;
        double e = 0.0;
        for (long q = threadIdx.x; q < r.nextra; q += NT) e += load_coherent(extra + q);
        e = block_sum<NT>(e, lds);
        double u[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            u[c] = 0.0;
            for (long q = threadIdx.x; q < (long)nb; q += NT) u[c] += load_coherent(part + q * K + c);
            u[c] = block_sum<NT>(u[c], lds);
        }
        if (threadIdx.x == 0) {
            tk[0] = 0u;
            out[0] = e + u[0];
#pragma unroll
            for (int c = 1; c < K; ++c) out[c] = u[c];
        }
        return true;
    }
    const unsigned int grp = lb / RED_GROUP;
    const unsigned int ngroups = (nb + RED_GROUP - 1) / RED_GROUP;
    const unsigned int gsize = (grp + 1 == ngroups) ? nb - grp * RED_GROUP : RED_GROUP;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c) store_coherent(part + (size_t)lb * K + c, s[c]);
        const unsigned int t = take_ticket(tk + (size_t)(1 + grp) * RED_TICKET_STRIDE);
        stage = (t == gsize - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (stage == 0) return false;
    // last workgroup of the group: ordered group sums
    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        v[c] = 0.0;
        if (threadIdx.x < gsize)
            v[c] = load_coherent(part + ((size_t)grp * RED_GROUP + threadIdx.x) * K + c);
        v[c] = block_sum<NT>(v[c], lds);
    }
    if (threadIdx.x == 0) {
        tk[(size_t)(1 + grp) * RED_TICKET_STRIDE] = 0u;
#pragma unroll
        for (int c = 0; c < K; ++c) store_coherent(gpart + (size_t)grp * K + c, v[c]);
        const unsigned int t = take_ticket(tk);
        stage = (t == ngroups - 1u) ? 2 : 0;
    }
    __syncthreads();
    if (stage != 2) return false;
    // last group: ordered sums of the group sums, then the extra partials
    double e = 0.0;
    for (long q = threadIdx.x; q < r.nextra; q += NT) e += load_coherent(extra + q);
    e = block_sum<NT>(e, lds);
    double u[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        u[c] = 0.0;
        for (long q = threadIdx.x; q < (long)ngroups; q += NT) u[c] += load_coherent(gpart + q * K + c);
        u[c] = block_sum<NT>(u[c], lds);
    }
    if (threadIdx.x == 0) {
        tk[0] = 0u;
        out[0] = e + u[0];
#pragma unroll
        for (int c = 1; c < K; ++c) out[c] = u[c];
    }
    return true;
}

template <int NT>
__device__ __forceinline__ bool grid_finish(double s, const RedSite &r, double *out, double *lds,
                                            unsigned int lb, unsigned int nb) {
    return grid_finish_k<NT, 1>(&s, r, out, lds, lb, nb);
}

template <int NT>
__device__ __forceinline__ bool grid_finish(double s, const RedSite &r, double *out, double *lds) {
    return grid_finish<NT>(s, r, out, lds, blockIdx.x, gridDim.x);
}

}  // namespace nek
