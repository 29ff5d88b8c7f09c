// Device-side sorted-set primitives for gfx950 (64-lane wavefronts).
//
// Every candidate set is an ascending int32 array (a CSR neighbor list or a
// buffer built from lists). Intersections cost O(|A| + |B|) in the paper's
// model (Section IV-C, "Measurement of c_i and l_i"; Section IV-E: sorted
// contiguous lists). Here a group of G lanes intersects cooperatively: each
// lane takes one element of the smaller list and binary-searches it in the
// larger one; ballot + popcount compact the hits in order. Single lanes use a
// branch-free merge or a galloping search, whichever the sizes favour. When
// the larger operand is a hub's list, membership is one bit test in the hub's
// dense bitmap instead of a binary search (one cache line instead of ~log2 n).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpdev {

struct Set {
    const int32_t* p;
    int32_t n;
    // Dense membership bitmap of the whole (uncut) neighbor list when the
    // list belongs to a hub, else null. A bit test replaces the binary search
    // for values inside the range the set was cut to.
    const uint32_t* bits;
};

// First index i in [0, n) with a[i] >= x (n if none).
__device__ __forceinline__ int32_t lower_bound(const int32_t* a, int32_t n, int32_t x) {
    int32_t base = 0;
    while (n > 0) {
        int32_t half = n >> 1;
        if (a[base + half] < x) {
            base += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return base;
}

__device__ __forceinline__ bool contains(const int32_t* a, int32_t n, int32_t x) {
    int32_t i = lower_bound(a, n, x);
    return i < n && a[i] == x;
}

// Restrict a sorted set to values in [lo, hi).
__device__ __forceinline__ Set trim(Set s, int32_t lo, int32_t hi) {
    int32_t b = lo > 0 ? lower_bound(s.p, s.n, lo) : 0;
    int32_t e = hi < 0x7fffffff ? lower_bound(s.p, s.n, hi) : s.n;
    if (e < b) e = b;
    return Set{s.p + b, e - b, s.bits};
}

// x in s, for an x inside the value range that s was cut to.
__device__ __forceinline__ bool member(const Set& s, int32_t x) {
    if (s.bits) return (s.bits[x >> 5] >> (x & 31)) & 1u;
    return contains(s.p, s.n, x);
}

// |{x in A : bit x of bits set}| by one lane, not counting x with skip(x).
// A must lie inside the value range the bitmap's set was cut to. Four
// independent loads are kept in flight per lane.
template <typename Skip>
__device__ __forceinline__ uint32_t count_bits(Set a, const uint32_t* bits, Skip skip) {
    uint32_t c = 0;
    int32_t i = 0;
    for (; i + 4 <= a.n; i += 4) {
        const int32_t x0 = a.p[i], x1 = a.p[i + 1], x2 = a.p[i + 2], x3 = a.p[i + 3];
        const uint32_t w0 = bits[x0 >> 5], w1 = bits[x1 >> 5], w2 = bits[x2 >> 5], w3 = bits[x3 >> 5];
        if ((w0 >> (x0 & 31)) & 1u) c += !skip(x0);
        if ((w1 >> (x1 & 31)) & 1u) c += !skip(x1);
        if ((w2 >> (x2 & 31)) & 1u) c += !skip(x2);
        if ((w3 >> (x3 & 31)) & 1u) c += !skip(x3);
    }
    for (; i < a.n; ++i) {
        const int32_t x = a.p[i];
        if ((bits[x >> 5] >> (x & 31)) & 1u) c += !skip(x);
    }
    return c;
}

// The same for a short list A not yet cut to [lo, hi): every element is
// loaded and range-tested. Independent loads instead of the two dependent
// chains of binary searches that cutting would take.
constexpr int32_t kShortList = 32;

template <typename Skip>
__device__ __forceinline__ uint32_t count_bits_range(Set a, int32_t lo, int32_t hi, const uint32_t* bits,
                                                     Skip skip) {
    uint32_t c = 0;
    int32_t i = 0;
    for (; i + 4 <= a.n; i += 4) {
        const int32_t x0 = a.p[i], x1 = a.p[i + 1], x2 = a.p[i + 2], x3 = a.p[i + 3];
        if (x0 >= hi) break;
        const uint32_t w0 = bits[x0 >> 5], w1 = bits[x1 >> 5], w2 = bits[x2 >> 5], w3 = bits[x3 >> 5];
        if (x0 >= lo && ((w0 >> (x0 & 31)) & 1u)) c += !skip(x0);
        if (x1 >= lo && x1 < hi && ((w1 >> (x1 & 31)) & 1u)) c += !skip(x1);
        if (x2 >= lo && x2 < hi && ((w2 >> (x2 & 31)) & 1u)) c += !skip(x2);
        if (x3 >= lo && x3 < hi && ((w3 >> (x3 & 31)) & 1u)) c += !skip(x3);
    }
    for (; i < a.n; ++i) {
        const int32_t x = a.p[i];
        if (x >= hi) break;
        if (x >= lo && ((bits[x >> 5] >> (x & 31)) & 1u)) c += !skip(x);
    }
    return c;
}

// |A ∩ B| by one lane, not counting elements x with skip(x).
template <typename Skip>
__device__ __forceinline__ uint32_t intersect_count_serial(Set a, Set b, Skip skip) {
    if (a.n > b.n) {
        Set t = a;
        a = b;
        b = t;
    }
    if (a.n == 0) return 0;
    uint32_t c = 0;
    if (b.bits) return count_bits(a, b.bits, skip);
    if (a.n * 16 < b.n) {
        // galloping: each element of the small set searched in the rest of the large one
        const int32_t* p = b.p;
        int32_t n = b.n;
        for (int32_t i = 0; i < a.n && n > 0; ++i) {
            int32_t x = a.p[i];
            int32_t j = lower_bound(p, n, x);
            if (j < n && p[j] == x) {
                c += !skip(x);
                ++j;
            }
            p += j;
            n -= j;
        }
        return c;
    }
    int32_t i = 0, j = 0;
    while (i < a.n && j < b.n) {
        int32_t x = a.p[i], y = b.p[j];
        if (x == y) c += !skip(x);
        i += (x <= y);
        j += (y <= x);
    }
    return c;
}

__device__ __forceinline__ uint32_t intersect_count_serial(Set a, Set b) {
    return intersect_count_serial(a, b, [](int32_t) { return false; });
}

// A group of G consecutive lanes of one wavefront acting together.
template <int G>
struct Group {
    static_assert(G == 64 || G == 32 || G == 16 || G == 8, "group size");
    int lane;   // lane in the wavefront
    int gl;     // lane in the group
    int gbase;  // first lane of the group

    __device__ __forceinline__ Group() {
        lane = __lane_id();
        gl = lane & (G - 1);
        gbase = lane & ~(G - 1);
    }
    __device__ __forceinline__ uint64_t ballot(bool pred) const {
        uint64_t m = __ballot(pred);
        if (G == 64) return m;
        return (m >> gbase) & ((uint64_t(1) << G) - 1);
    }
    __device__ __forceinline__ uint32_t below_mask_count(uint64_t m) const {
        return __popcll(m & ((uint64_t(1) << gl) - 1));
    }
    template <typename T>
    __device__ __forceinline__ T bcast(T v, int src) const {
        return __shfl(v, src, G);
    }
    __device__ __forceinline__ uint64_t sum(uint64_t v) const {
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
        return v;
    }
};

// Group-cooperative dst = A ∩ B (both already cut to the wanted range).
// Returns the number of elements written (the same in every lane).
template <int G>
__device__ __forceinline__ int32_t intersect_into(const Group<G>& g, Set a, Set b, int32_t* dst) {
    if (a.n > b.n) {
        Set t = a;
        a = b;
        b = t;
    }
    int32_t out = 0;
    for (int32_t base = 0; base < a.n; base += G) {
        int32_t i = base + g.gl;
        bool found = false;
        int32_t x = 0;
        if (i < a.n) {
            x = a.p[i];
            found = member(b, x);
        }
        uint64_t m = g.ballot(found);
        if (found) dst[out + (int32_t)g.below_mask_count(m)] = x;
        out += (int32_t)__popcll(m);
    }
    return out;
}

// Group-cooperative |A ∩ B| not counting x with skip(x) (same value in every lane).
template <int G, typename Skip>
__device__ __forceinline__ uint32_t intersect_count_group(const Group<G>& g, Set a, Set b, Skip skip) {
    if (a.n > b.n) {
        Set t = a;
        a = b;
        b = t;
    }
    uint32_t out = 0;
    for (int32_t base = 0; base < a.n; base += G) {
        int32_t i = base + g.gl;
        bool found = false;
        if (i < a.n) {
            int32_t x = a.p[i];
            found = member(b, x) && !skip(x);
        }
        out += (uint32_t)__popcll(g.ballot(found));
    }
    return out;
}

}  // namespace gpdev
