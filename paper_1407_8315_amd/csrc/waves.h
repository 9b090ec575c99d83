// Wave-level list appends and counters shared by the decoders.
#pragma once

#include "common.h"

namespace sft {

// Append to a list shared by many lanes with one atomic per wavefront: every
// lane of the wave that is still running must call this (pred may be false);
// returns the slot of a lane with pred set.
__device__ inline int wave_append(int* counter, bool pred) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// Add n (0 <= n < 8) to *addr for every running lane of the wave and return
// each lane's previous value plus the sum over lower running lanes with the
// same address: one atomic per wave when all lanes share the address (the
// common case: a wave's bins belong to one signal), one per lane otherwise.
// The prefix sums come from one ballot per bit of n, so any subset of the
// wave's lanes may be running.
__device__ inline int wave_add(int* addr, int n) {
    const unsigned long long run = __ballot(true);
    const int lane = __lane_id();
    const int leader = __ffsll((long long)run) - 1;
    const unsigned long long a_lead = __shfl((unsigned long long)addr, leader);
    if (__ballot((unsigned long long)addr != a_lead) != 0ull) return atomicAdd(addr, n);
    const unsigned long long lt = (1ull << lane) - 1ull;
    const unsigned long long b0 = __ballot(n & 1), b1 = __ballot(n & 2), b2 = __ballot(n & 4);
    const int before = __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
    const int total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
    int base = 0;
    if (lane == leader && total > 0) base = atomicAdd(addr, total);
    base = __shfl(base, leader);
    return base + before;
}

// Count pred over the wave into *addr: one atomic per wave when every running
// lane has the same address, one per lane otherwise.
__device__ inline void wave_count(int* addr, bool pred) {
    const unsigned long long run = __ballot(true);
    const unsigned long long m = __ballot(pred);
    const int leader = __ffsll((long long)run) - 1;
    const unsigned long long a_lead = __shfl((unsigned long long)addr, leader);
    if (__ballot((unsigned long long)addr != a_lead) != 0ull) {
        if (pred) atomicAdd(addr, 1);
        return;
    }
    if (__lane_id() == leader && m != 0ull) atomicAdd(addr, __popcll(m));
}

}  // namespace sft
