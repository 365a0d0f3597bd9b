// Batched evaluation: many populations (of one or several jobs, each with
// its own matrix, archive and parameters) in one kernel launch.
//
// A workgroup takes one individual and splits its rows into items of 4096
// rows (or a few such chunks), one wave each; individuals of all jobs form
// one flat index space, so a single launch covers the whole batch,
// individuals of uneven length included. With a pair table a lane tests 64
// rows at once: each step of the series is one 64-bit load of the pair's
// bitmap, and the rows' steps against each trend are counted bit-sliced in
// a counter that starts at 2^P - (t+1) and so carries out of its top plane
// on the (t+1)-th such step; a sticky carry flag per trend then decides the
// row, with no compares. Without a table the item runs the gather form
// (lane = row) over its 64-row blocks. The last wave of the workgroup to
// finish reduces the individual: the count, the rows shared with each
// archive member, and the FP64 fitness. The paper sends the whole
// population to the GPU at once (Sec. 2.4, step 2); here several
// populations share the launch.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device.h"
#include "internal.h"

namespace ebic {

struct DevJob {
    const uint16_t *ranks;
    const uint64_t *pairs;
    const uint64_t *pairs_strict;  // strict pair table or NULL
    int32_t rows, cols, rows_pad, w32, w64;
    int32_t pstride;  // words per pair in the pair table
    int32_t mode;     // 1 = pair table, 0 = gather
    int32_t nchunks;  // 4096-row chunks per individual
    int32_t cpi;      // chunks per item (one wave walks them WPL at a time)
    int32_t ipi;      // items (waves) per individual = ceil(nchunks / cpi)
    int32_t pop_size, pop_len;
    int64_t ind_begin;   // first individual of this job in the batch
    const int32_t *pop_off;
    const uint16_t *pop_cols;
    const int32_t *order;
    int32_t arch_size, arch_len;
    const uint64_t *arch_support;
    const int32_t *arch_off;
    const uint16_t *arch_cols;
    int32_t approx_permille, negative_trends, overlap_permille, min_rows, k_score_min, tie_rule;
    double *fitness;
    int32_t *count;
    uint64_t *support;
    int32_t *overlap;
};

namespace {

constexpr int kMaxWaves = 16;     // waves per workgroup: items per individual
constexpr int kMixedWaves = 4;    // the same, for jobs sharing a launch with smaller ones
constexpr int kItemRows = 4096;   // 64 lanes x 64 rows, or 64 blocks x 64 rows
// pair-bitmap loads in flight per wave (KB) and words per lane (WPL) are
// template parameters, picked per batch by the autotuner
constexpr int kGGroup = 8;        // archive members whose columns one pass loads (no LDS copy)
constexpr int kHGroup = 4;        // archive members whose shared rows one pass counts
constexpr int kHWords = 3;        // support words per lane and pass when counting them
constexpr int kArchLdsCols = 8192;  // largest archive whose columns are copied to LDS (16 KB)
constexpr int kSchedBatch = 4;   // schedule phases loaded together
constexpr int kSupLdsWords = 2048;  // longest support kept in LDS for the reduction (16 KB)
// Individuals per workgroup: as many as keep the workgroup at kGroupWaves
// waves or fewer (at most kMaxIpw) and its LDS at kGroupLds bytes or fewer.
// A workgroup's individuals are slots a grid apart (g, g + G, ...): on the
// 10,000-row workload (two waves per individual) pairing slot g with slot
// g + 2,048 took a launch from 22.5 to 20.5 us, while pairing neighbours
// (g, g + 1) made it 0.4 us slower and pairing g with the mirror slot 2G-1-g
// 1.7 us slower; workgroups of eight waves were slower still.
constexpr int kGroupWaves = 4;
constexpr int kMaxIpw = 4;  // 1, 2 or 4 (ceil(total / ipw) by shifts in the kernel)
constexpr size_t kGroupLds = 65536;

// Segment of a flat index (a job's individuals, a phase of the item
// schedule): count the segment starts after the first at or below it. The
// starts sit in a compact array, so the loads are independent scalar loads.
__device__ inline int find_segment(const int64_t *__restrict__ begins, int njobs, int64_t x) {
    int j = 0;
    for (int q = 1; q < njobs; q++) j += begins[q] <= x;
    return j;
}

// Bit-sliced sum of KB one-bit inputs into PSUM_BITS(KB) planes.
template <int KB>
struct PartialSum {
    static constexpr int B = KB == 1 ? 1 : KB == 2 ? 2 : 3;
    static_assert(KB == 1 || KB == 2 || KB == 4, "groups of 1, 2 or 4 steps");
    __device__ __forceinline__ static void sum(const uint64_t *v, uint64_t *s) {
        if constexpr (KB == 1) {
            s[0] = v[0];
        } else if constexpr (KB == 2) {
            s[0] = v[0] ^ v[1];
            s[1] = v[0] & v[1];
        } else {
            const uint64_t a0 = v[0] ^ v[1] ^ v[2];
            const uint64_t a1 = (v[0] & v[1]) | (v[2] & (v[0] ^ v[1]));
            const uint64_t c = a0 & v[3];
            s[0] = a0 ^ v[3];
            s[1] = a1 ^ c;
            s[2] = a1 & c;
        }
    }
};

// C (P planes) += S (B planes), ripple carry; the carry out of the top plane
// and any bit of S at or above plane P set the sticky flag ov.
template <int P, int B>
__device__ __forceinline__ void add_sticky(uint64_t *C, const uint64_t *S, uint64_t &ov) {
    uint64_t c = 0;
#pragma unroll
    for (int p = 0; p < P; p++) {
        if (p < B) {
            const uint64_t a = C[p], x = a ^ S[p];
            C[p] = x ^ c;
            c = (a & S[p]) | (c & x);
        } else {
            const uint64_t a = C[p];
            C[p] = a ^ c;
            c = a & c;
        }
    }
#pragma unroll
    for (int p = P; p < B; p++) c |= S[p];
    ov |= c;
}

// Steps against the increasing trend (downs) and against the decreasing
// trend (ups) of the 64 rows of each of this lane's WPL words (w, w + 64,
// ...), counted bit-sliced over P planes from the start value 2^P - (t+1)
// (2^P >= t+1), so that the count passes 2^P - 1 exactly on the (t+1)-th
// step against the trend; that carry is kept in a sticky flag per trend
// (dov, uov). A row fits the increasing trend while dov is clear, the
// decreasing one while uov is clear. Each group of KB steps is loaded
// together, summed into a small partial count and added to the counters
// once; after each group the wave stops once every row has failed both
// trends. Writes the fit words to fit[].
template <int P, bool NEG, int KB, int WPL, bool TWO>
__device__ __forceinline__ void pairs_count_two(const uint64_t *__restrict__ pairs,
                                            const uint64_t *__restrict__ strict, bool loose,
                                            int64_t pstride, int wlim, const int32_t *s_pd, int k,
                                            int t, int w, uint64_t *fit) {
    constexpr int NP = P > 0 ? P : 1;
    constexpr int B = PartialSum<KB>::B;
    uint32_t start = __builtin_amdgcn_readfirstlane((1u << P) - (uint32_t)(t + 1));
    // opaque to the optimiser: keeps the start planes from being hoisted out
    // of the caller's chunk loop and held in registers across it
    asm volatile("" : "+s"(start));
    bool active[WPL];
    uint64_t D[WPL][NP], U[WPL][NP], dov[WPL], uov[WPL];
#pragma unroll
    for (int v = 0; v < WPL; v++) {
        active[v] = w + kWave * v < wlim;
#pragma unroll
        for (int p = 0; p < P; p++) D[v][p] = U[v][p] = ((start >> p) & 1u) ? ~0ull : 0ull;
        dov[v] = uov[v] = 0;
    }
    int j = 1;
    while (j < k) {
        const int n = (k - j) < KB ? (k - j) : KB;
        uint64_t up[WPL][KB], dn[WPL][KB];
#pragma unroll
        for (int q = 0; q < KB; q++) {
            // a step's rows against the decreasing trend (u) and against the
            // increasing one (d)
            uint64_t u[WPL], d[WPL];
#pragma unroll
            for (int v = 0; v < WPL; v++) u[v] = d[v] = 0;
            if (q < n) {
                const int pd = __builtin_amdgcn_readfirstlane(s_pd[j + q]);
                const int64_t at = (int64_t)(pd & 0x7fffffff) * pstride;
                const auto *vec = gmem(pairs) + at;
#pragma unroll
                for (int v = 0; v < WPL; v++) {
                    const uint64_t le = active[v] ? vec[w + kWave * v] : 0ull;
                    if constexpr (TWO) {
                        // le: lo at or below hi, lt: strictly below. Strict
                        // rule, step lo -> hi: ups le, downs ~lt; loose: ups
                        // lt, downs ~le; a step hi -> lo swaps the roles.
                        const uint64_t lt = active[v] ? gmem(strict)[at + w + kWave * v] : 0ull;
                        const uint64_t a = loose ? lt : le, b = loose ? le : lt;
                        u[v] = pd < 0 ? ~b : a;
                        d[v] = pd < 0 ? a : ~b;
                    } else {
                        u[v] = pd < 0 ? ~le : le;  // 1 = up-step in this row
                        d[v] = ~u[v];
                    }
                }
            }
            const uint64_t vm = q < n ? ~0ull : 0ull;  // steps past the end count nothing
#pragma unroll
            for (int v = 0; v < WPL; v++) {
                up[v][q] = u[v] & vm;
                dn[v][q] = d[v] & vm;
            }
        }
        bool live = false;
#pragma unroll
        for (int v = 0; v < WPL; v++) {
            uint64_t S[B];
            PartialSum<KB>::sum(dn[v], S);
            add_sticky<P, B>(D[v], S, dov[v]);
            if (NEG) {
                PartialSum<KB>::sum(up[v], S);
                add_sticky<P, B>(U[v], S, uov[v]);
            }
            const uint64_t dead = dov[v] & (NEG ? uov[v] : ~0ull);
            live |= active[v] && dead != ~0ull;
        }
        j += n;
        if (__ballot(live) == 0) break;
    }
#pragma unroll
    for (int v = 0; v < WPL; v++) fit[v] = ~dov[v] | (NEG ? ~uov[v] : 0ull);
}

// Three-input bitwise operation (v_bitop3_b32). IMM is the truth table:
// bit (a << 2 | b << 1 | c) of IMM is the result for input bits a, b, c,
// i.e. the operation applied to a = 0xF0, b = 0xCC, c = 0xAA.
template <int IMM>
__device__ __forceinline__ uint32_t lop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
}
constexpr int kXor3 = 0x96;    // a ^ b ^ c
constexpr int kMaj = 0xE8;     // at least two of a, b, c
constexpr int kAndXor = 0x60;  // a & (b ^ c)
constexpr int kOr3 = 0xFE;     // a | b | c
constexpr int kNor2 = 0x03;    // ~(a | b)
constexpr int kNor3 = 0x01;    // ~(a | b | c)

// C (P planes of one 32-bit half) += S (B planes); the carry out of the top
// plane, and any bit of S at or above plane P, set the sticky flag ov.
template <int P, int B>
__device__ __forceinline__ void add_half(uint32_t *C, const uint32_t *S, uint32_t &ov) {
    if constexpr (P == 0) {
        // no room: any step against the trend ends the row
        if constexpr (B == 1) ov |= S[0];
        else if constexpr (B == 2) ov = lop3<kOr3>(ov, S[0], S[1]);
        else ov = lop3<kOr3>(ov, S[0], S[1]) | S[2];
    } else {
        uint32_t c;
        {
            const uint32_t a = C[0];
            C[0] = a ^ S[0];
            c = a & S[0];
        }
#pragma unroll
        for (int p = 1; p < P; p++) {
            const uint32_t a = C[p];
            if (p < B) {
                C[p] = lop3<kXor3>(a, S[p], c);
                c = lop3<kMaj>(a, S[p], c);
            } else {
                C[p] = a ^ c;
                c = a & c;
            }
        }
#pragma unroll
        for (int p = P; p < B; p++) c |= S[p];
        ov |= c;
    }
}

// Bit-sliced count of n in {1, 2, 3, 4} steps of one 32-bit half: the rows'
// up-steps (ups) and down-steps (dns, n - ups), B = 1, 2, 2, 3 planes. A
// step's up bits are its table bits b, inverted when the step runs from the
// higher column to the lower one (m = ~0 then, uniform).
template <int N>
struct StepSum {
    static constexpr int B = N == 1 ? 1 : N == 4 ? 3 : 2;
    __device__ __forceinline__ static void sum(const uint32_t *b, const uint32_t *m, uint32_t *ups,
                                               uint32_t *dns) {
        if constexpr (N == 1) {
            ups[0] = b[0] ^ m[0];
            dns[0] = ~ups[0];
        } else if constexpr (N == 2) {
            const uint32_t x0 = b[0] ^ m[0];
            ups[0] = lop3<kXor3>(x0, b[1], m[1]);
            ups[1] = lop3<kAndXor>(x0, b[1], m[1]);
            dns[0] = ups[0];                         // 2 - u has u's parity
            dns[1] = lop3<kNor2>(ups[0], ups[1], 0);  // 2 - u >= 2 only for u = 0
        } else if constexpr (N == 3) {
            const uint32_t x0 = b[0] ^ m[0], x1 = b[1] ^ m[1], x2 = b[2] ^ m[2];
            ups[0] = lop3<kXor3>(x0, x1, x2);
            ups[1] = lop3<kMaj>(x0, x1, x2);
            dns[0] = ~ups[0];  // 3 - u is u's two-bit complement
            dns[1] = ~ups[1];
        } else {
            const uint32_t x0 = b[0] ^ m[0], x1 = b[1] ^ m[1], x2 = b[2] ^ m[2];
            const uint32_t a0 = lop3<kXor3>(x0, x1, x2), a1 = lop3<kMaj>(x0, x1, x2);
            // add the fourth step, x3 = b3 ^ m3
            const uint32_t c = lop3<kAndXor>(a0, b[3], m[3]);
            ups[0] = lop3<kXor3>(a0, b[3], m[3]);
            ups[1] = a1 ^ c;
            ups[2] = a1 & c;
            // 4 - u: same parity; bit 1 set for u = 1, 2; bit 2 only for u = 0
            dns[0] = ups[0];
            dns[1] = ups[1] ^ ups[0];
            dns[2] = lop3<kNor3>(ups[0], ups[1], ups[2]);
        }
    }
};

// The column-index tie rule (one table; every step is either up or down in
// a row): the same counters as pairs_count_two, on 32-bit halves with
// three-input logic, groups of KB steps loaded together through buffer
// loads with a scalar row offset. FLAT (a table below 4 GB): the step
// descriptors hold each pair row's byte offset (bit 0: the step runs from
// the higher column to the lower one) and every load goes through one
// resource for the whole table; else they hold the pair index (sign bit:
// direction) and each step builds its row's resource. The next group's
// descriptors are read from LDS while this group's loads are in flight.
// KB = 8 loads eight steps at once and counts them as two groups of four.
template <int P, bool NEG, int KB, int WPL, bool FLAT>
__device__ __forceinline__ void pairs_count_one(const uint64_t *__restrict__ pairs,
                                                int64_t pstride, uint32_t table_bytes, int wlim,
                                                const int32_t *s_pd, int k, int t, int w,
                                                uint64_t *fit) {
    constexpr int NP = P > 0 ? P : 1;
    uint32_t start = __builtin_amdgcn_readfirstlane((1u << P) - (uint32_t)(t + 1));
    asm volatile("" : "+s"(start));
    const uint32_t row_bytes = (uint32_t)(pstride * 8);
    const __amdgpu_buffer_rsrc_t trs = make_rsrc(pairs, FLAT ? table_bytes : row_bytes);
    bool active[WPL];
    int voff[WPL];
    uint32_t D[WPL][2][NP], U[WPL][2][NP], dov[WPL][2], uov[WPL][2];
#pragma unroll
    for (int v = 0; v < WPL; v++) {
        active[v] = w + kWave * v < wlim;
        // an inactive lane reads the row's first word (FLAT) or past the
        // row's end (the buffer returns 0); its result is never used
        voff[v] = active[v] ? (w + kWave * v) * 8 : (FLAT ? 0 : (int)row_bytes);
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int p = 0; p < P; p++) D[v][h][p] = U[v][h][p] = ((start >> p) & 1u) ? ~0u : 0u;
            dov[v][h] = uov[v][h] = 0;
        }
    }
    // descriptors of KB steps from step j on (indexes past the series read
    // unused LDS words inside the array)
    auto descr = [&](int j, int32_t *pd) {
#pragma unroll
        for (int q = 0; q < KB; q++) {
            const int i = j + q < EBIC_MAX_K ? j + q : EBIC_MAX_K - 1;
            pd[q] = s_pd[i];
        }
    };
    // loads and flips of the first n of those steps
    auto load = [&](const int32_t *pdv, int n, uint32_t (*b)[WPL][2], uint32_t *m) {
#pragma unroll
        for (int q = 0; q < KB; q++) {
            if (q < n) {
                const int pd = __builtin_amdgcn_readfirstlane(pdv[q]);
                __amdgpu_buffer_rsrc_t rs = trs;
                uint32_t soff = 0;
                if constexpr (FLAT) {
                    m[q] = (pd & 1) ? ~0u : 0u;
                    soff = (uint32_t)pd & ~1u;
                } else {
                    const uint64_t *row = pairs + (int64_t)(pd & 0x7fffffff) * pstride;
                    rs = make_rsrc(row, row_bytes);
                    m[q] = pd < 0 ? ~0u : 0u;
                }
#pragma unroll
                for (int v = 0; v < WPL; v++) {
                    const auto x = __builtin_amdgcn_raw_buffer_load_b64(rs, voff[v], soff, 0);
                    b[q][v][0] = x[0];
                    b[q][v][1] = x[1];
                }
            }
        }
    };
    auto count = [&](auto nconst, uint32_t (*b)[WPL][2], const uint32_t *m) {
        constexpr int N = decltype(nconst)::value;
        constexpr int B = StepSum<N>::B;
#pragma unroll
        for (int v = 0; v < WPL; v++) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint32_t bb[N], ups[B], dns[B];
#pragma unroll
                for (int q = 0; q < N; q++) bb[q] = b[q][v][h];
                StepSum<N>::sum(bb, m, ups, dns);
                add_half<P, B>(D[v][h], dns, dov[v][h]);
                if (NEG) add_half<P, B>(U[v][h], ups, uov[v][h]);
            }
        }
    };
    // n in 0 .. 3 steps
    auto count_few = [&](int n, uint32_t (*b)[WPL][2], const uint32_t *m) {
        if (n == 1) count(std::integral_constant<int, 1>{}, b, m);
        if constexpr (KB > 2) {
            if (n == 2) count(std::integral_constant<int, 2>{}, b, m);
            if (n == 3) count(std::integral_constant<int, 3>{}, b, m);
        }
    };
    int32_t pn[KB];
    descr(1, pn);
    int j = 1;
    for (; j + KB <= k; j += KB) {
        uint32_t b[KB][WPL][2], m[KB];
        load(pn, KB, b, m);
        descr(j + KB, pn);
        if constexpr (KB == 8) {
            count(std::integral_constant<int, 4>{}, b, m);
            count(std::integral_constant<int, 4>{}, b + 4, m + 4);
        } else {
            count(std::integral_constant<int, KB>{}, b, m);
        }
        bool live = false;
#pragma unroll
        for (int v = 0; v < WPL; v++) {
            const uint32_t lo = NEG ? dov[v][0] & uov[v][0] : dov[v][0];
            const uint32_t hi = NEG ? dov[v][1] & uov[v][1] : dov[v][1];
            live |= active[v] && (lo & hi) != ~0u;
        }
        if (__ballot(live) == 0) {
            j = k + 1;  // every row is out of both trends: skip the tail
            break;
        }
    }
    const int rest = k - j;  // 0 .. KB - 1 steps left (negative after an early exit)
    if (rest > 0) {
        uint32_t b[KB][WPL][2], m[KB];
        load(pn, rest, b, m);
        if constexpr (KB == 8) {
            if (rest >= 4) {
                count(std::integral_constant<int, 4>{}, b, m);
                count_few(rest - 4, b + 4, m + 4);
            } else {
                count_few(rest, b, m);
            }
        } else {
            count_few(rest, b, m);
        }
    }
#pragma unroll
    for (int v = 0; v < WPL; v++) {
        const uint32_t lo = ~dov[v][0] | (NEG ? ~uov[v][0] : 0u);
        const uint32_t hi = ~dov[v][1] | (NEG ? ~uov[v][1] : 0u);
        fit[v] = ((uint64_t)hi << 32) | lo;
    }
}

// flat: the one-table descriptors hold byte offsets (a table below 4 GB of
// table_bytes); the two-table path always takes pair indexes, at most four
// loads in flight.
template <int P, bool NEG, int KB, int WPL, bool TWO>
__device__ __forceinline__ void pairs_count(const uint64_t *__restrict__ pairs,
                                            const uint64_t *__restrict__ strict, bool loose,
                                            int64_t pstride, bool flat, uint32_t table_bytes,
                                            int wlim, const int32_t *s_pd, int k, int t, int w,
                                            uint64_t *fit) {
    if constexpr (TWO)
        pairs_count_two<P, NEG, (KB > 4 ? 4 : KB), WPL, true>(pairs, strict, loose, pstride, wlim,
                                                              s_pd, k, t, w, fit);
    else if (flat)
        pairs_count_one<P, NEG, KB, WPL, true>(pairs, pstride, table_bytes, wlim, s_pd, k, t, w,
                                               fit);
    else
        pairs_count_one<P, NEG, KB, WPL, false>(pairs, pstride, table_bytes, wlim, s_pd, k, t, w,
                                                fit);
}

// Widest counter the pair path instantiates for KB steps per group and WPL
// words per lane: with one word per lane and two or four loads in flight,
// what keeps the kernel within 64 VGPRs (8 waves per SIMD); eight loads in
// flight hold 72 (7 waves) from P = 4 on; with two words, the widths past
// which registers climb steeply. Items with a larger tolerance (t >= 2^P)
// take the gather form.
template <int KB, int WPL>
struct PairLimit {
    static constexpr int P = WPL == 1 ? (KB == 8 ? 4 : KB == 4 ? 5 : 8) : (KB == 4 ? 3 : 4);
    static constexpr int T = (1 << P) - 1;
};

template <int PP, int MAXP, bool NEG, int KB, int WPL, bool TWO>
__device__ __forceinline__ void pairs_width(int P, const uint64_t *pairs, const uint64_t *strict,
                                            bool loose, int64_t pstride, bool flat,
                                            uint32_t table_bytes, int wlim, const int32_t *s_pd,
                                            int k, int t, int w, uint64_t *fit) {
    if constexpr (PP == MAXP) {
        pairs_count<PP, NEG, KB, WPL, TWO>(pairs, strict, loose, pstride, flat, table_bytes, wlim,
                                           s_pd, k, t, w, fit);
    } else {
        if (P == PP)
            return pairs_count<PP, NEG, KB, WPL, TWO>(pairs, strict, loose, pstride, flat,
                                                      table_bytes, wlim, s_pd, k, t, w, fit);
        pairs_width<PP + 1, MAXP, NEG, KB, WPL, TWO>(P, pairs, strict, loose, pstride, flat,
                                                     table_bytes, wlim, s_pd, k, t, w, fit);
    }
}

// Counter width for tolerance t <= PairLimit<KB, WPL>::T: the least P with
// 2^P >= t+1.
// TWO: both tables (the strict and loose tie rules; loose selects which).
template <bool NEG, int KB, int WPL, bool TWO>
__device__ __forceinline__ void pairs_dispatch(const uint64_t *pairs, const uint64_t *strict,
                                               bool loose, int64_t pstride, bool flat,
                                               uint32_t table_bytes, int wlim,
                                               const int32_t *s_pd, int k, int t, int w,
                                               uint64_t *fit) {
    const int P = t == 0 ? 0 : 32 - __builtin_clz((unsigned)t);
    pairs_width<0, PairLimit<KB, WPL>::P, NEG, KB, WPL, TWO>(P, pairs, strict, loose, pstride,
                                                             flat, table_bytes, wlim, s_pd, k, t,
                                                             w, fit);
}

// One or more individuals per workgroup (ipw, each with its own waves and
// LDS), one wave per item (a few 4096-row chunks of the individual's rows);
// the last of an individual's waves to finish reduces it. Slots follow a
// round-robin schedule over the jobs' individuals (phase p interleaves the
// first njobs - p jobs of the job table, which is sorted by population size,
// descending), so each job's longest-first processing order holds across the
// batch.
//
// 1. All threads stage the series in LDS (one pair descriptor per step, or
//    each column's byte offset for the gather form) and mark its columns in
//    an LDS bitmap; a column out of range or repeated anywhere in the series
//    makes the individual invalid.
// 2. Wave w counts the rows of its chunks (pair counters or gather form),
//    writes the support words, and adds their row count to an LDS sum.
// 3. Every wave then counts itself done in LDS (after a workgroup-scope
//    release); the last one (after the matching acquire) reduces: n from the
//    LDS sum; the columns g shared with each archive member from the
//    member's columns and the bitmap; the rows h shared with the members
//    whose penalty can depend on them (h <= n, so only if 1000 g > theta k,
//    or all of them when the overlap output is requested), a few members per
//    pass with all loads issued together; then count, overlap and fitness.
// When the size score is 0 the fitness is 0 whatever the penalty, so the
// members are only visited for the overlap output.
// LDS bytes of one individual (the workgroup holds ipw of these, each at a
// 16-byte boundary): support, step descriptors, column bitmap, archive
// offsets, archive columns, 8 bytes of alignment slack, their hit masks.
__host__ __device__ constexpr size_t lds_ind_bytes(int32_t sup_words, int32_t bits_words,
                                                   int32_t acol_words) {
    return ((size_t)sup_words * 8 + (size_t)EBIC_MAX_K * 4 + (size_t)bits_words * 4 +
            (size_t)(EBIC_MAX_ARCHIVE + 1) * 4 + (size_t)acol_words * 2 + 8 +
            (size_t)(acol_words + kWave - 1) / kWave * 8 + 15) /
           16 * 16;
}

// Staging copies to LDS, kStageRound values per lane and round (each wave a
// block of kStageRound x 64 consecutive values): a round's loads are all
// issued before the first of them is waited on, one memory round trip per
// round rather than one per value. A lane past the end loads and writes the
// last value again (the same value to the same place), so that no load
// depends on a branch.
constexpr int kStageRound = 8;
template <class T, class F>
__device__ __forceinline__ void stage_round(const T *src, int n, int q0, F &put) {
    T v[kStageRound];
#pragma unroll
    for (int u = 0; u < kStageRound; u++) {
        const int q = q0 + u * kWave;
        v[u] = gmem(src)[q < n ? q : n - 1];
    }
#pragma unroll
    for (int u = 0; u < kStageRound; u++) {
        const int q = q0 + u * kWave;
        put(q < n ? q : n - 1, v[u]);
    }
}

// At most 80 scalar registers: from 81 on, gfx950 holds only 7 waves per
// SIMD (the compiler's occupancy estimate still says 8), and the item shapes
// are sized for 8 (the compiler keeps a value or two in vector-register lanes
// instead).
template <int KB, int WPL, bool TWO>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_num_sgpr(80)))
    batch_kernel(const DevJob *__restrict__ jobs, const int64_t *__restrict__ sched,
                 int32_t njobs, int64_t ph1, int32_t sup_words, int32_t bits_words,
                 int32_t acol_words, int32_t ipw, int32_t wpi, int32_t total) {
    // ipw individuals per workgroup (slots a grid apart), each with its own
    // wpi waves and its own part of the LDS. The wave's index is made
    // uniform (a scalar), and so is everything derived from it; its
    // individual is found by subtraction (ipw <= kMaxIpw), not a division
    const int gw = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    int sub = 0;
    for (int r = gw - wpi; r >= 0 && sub < kMaxIpw - 1; r -= wpi) sub++;
    const int wave = gw - sub * wpi, lane = threadIdx.x % kWave;
    const int nwaves = wpi;
    const int bdim = wpi * kWave;                    // threads per individual
    const int tid = (int)threadIdx.x - sub * bdim;   // thread among them
    // dynamic LDS: the support words (sup_words, 0 when they stay in global
    // memory only), the series' step descriptors, the column bitmap, the
    // archive's offsets and columns (acol_words, 0 when they stay global)
    extern __shared__ uint64_t s_lds[];
    uint64_t *const s_dyn =
        s_lds + (size_t)sub * (lds_ind_bytes(sup_words, bits_words, acol_words) / 8);
    uint64_t *s_sup = s_dyn;
    int32_t *s_pd = reinterpret_cast<int32_t *>(s_dyn + sup_words);
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(s_pd + EBIC_MAX_K);
    int32_t *s_aoff = reinterpret_cast<int32_t *>(s_bits + bits_words);
    uint16_t *s_acols = reinterpret_cast<uint16_t *>(s_aoff + EBIC_MAX_ARCHIVE + 1);
    // hit masks of the archive's columns, 64 per word (after the columns,
    // at the next 8-byte boundary; indexed from the LDS base so that the
    // pointer stays an LDS one)
    uint64_t *s_ahit =
        s_dyn + ((size_t)sup_words * 8 + EBIC_MAX_K * 4 + (size_t)bits_words * 4 +
                 (EBIC_MAX_ARCHIVE + 1) * 4 + (size_t)acol_words * 2 + 7) / 8;
    __shared__ int32_t s_bad_i[kMaxIpw], s_done_i[kMaxIpw], s_n_i[kMaxIpw];
    int32_t &s_bad = s_bad_i[sub], &s_done = s_done_i[sub], &s_n = s_n_i[sub];
    // the workgroup's individuals are slots a grid apart (g, g + G, ...), so
    // that the longest individuals, first in slot order, spread over the
    // grid rather than pairing up. Slots past the last (total) stay idle:
    // they pass the workgroup's barriers, then end; their loads below read
    // the last slot's
    // G = ceil(total / ipw), ipw being 1, 2 or 4
    const int32_t G = ipw == 1 ? total : ipw == 2 ? (total + 1) >> 1 : (total + 3) >> 2;
    const int64_t slot0 = (int64_t)blockIdx.x + (int64_t)sub * G;
    bool idle = slot0 >= total;
    const uint32_t slot = idle ? (uint32_t)(total - 1) : (uint32_t)slot0;
    // phase of this slot: the last phase start at or below it. Phase 0
    // (every job, from round 0) ends at ph1, a kernel argument, so its slots
    // (all of them when the jobs have equal populations) load nothing; past
    // it the starts and first rounds of kSchedBatch phases are loaded
    // together (independent scalar loads), then selected in registers.
    int p = 0;
    int64_t st = 0, rd = 0;
    for (int q0 = (int64_t)slot < ph1 ? njobs : 0; q0 < njobs; q0 += kSchedBatch) {
        int64_t qs[kSchedBatch], qr[kSchedBatch];
#pragma unroll
        for (int u = 0; u < kSchedBatch; u++) {
            const int q = q0 + u < njobs ? q0 + u : njobs - 1;
            qs[u] = sched[q];
            qr[u] = sched[njobs + q];
        }
#pragma unroll
        for (int u = 0; u < kSchedBatch; u++) {
            if (q0 + u < njobs && (q0 + u == 0 || qs[u] <= (int64_t)slot)) {
                p = q0 + u;
                st = qs[u];
                rd = qr[u];
            }
        }
    }
    const uint32_t rel = slot - (uint32_t)st, m = (uint32_t)(njobs - p);
    const DevJob &J = jobs[rel % m];
    const int32_t oi = (int32_t)(rd + rel / m);
    // the job fields the staging reads, all loaded before the first of them
    // is used (one scalar round trip instead of one per branch that first
    // needs a field): a job the host built never fails this check
    const int32_t *const j_order = J.order, *const j_off = J.pop_off;
    const uint16_t *const j_cols = J.pop_cols;
    const int32_t j_psize = J.pop_size, j_plen = J.pop_len, j_ncols = J.cols,
                  j_pstride = J.pstride, j_mode = J.mode, j_tie = J.tie_rule,
                  j_apx = J.approx_permille, j_asize = J.arch_size, j_alen = J.arch_len;
    if ((j_psize | j_plen | j_ncols | j_pstride | j_mode | j_tie | j_apx | j_asize | j_alen) < 0 ||
        !j_off || !j_cols || ((uintptr_t)j_order & 3u))
        idle = true;
    int32_t ind = 0, beg = 0, end = 0;
    if (!idle) {
        ind = j_order ? gmem(j_order)[oi] : oi;
        if (ind < 0 || ind >= j_psize) idle = true;  // not a permutation: no output
    }
    if (!idle) {
        beg = gmem(j_off)[ind];
        end = gmem(j_off)[ind + 1];
    }
    const int k = end - beg;
    const bool bad0 = idle || !(beg >= 0 && end <= j_plen && k >= 2 && k <= EBIC_MAX_K);
    const int t = bad0 ? 0 : tol(k, j_apx);
    // pair table when the batch has one, it serves the tie rule and the
    // counters fit; else gather
    const bool two = TWO && j_tie != EBIC_TIE_INDEX;  // both tables
    const bool use_pairs = j_mode == 1 && t <= PairLimit<KB, WPL>::T &&
                           (j_tie == EBIC_TIE_INDEX || (TWO && J.pairs_strict));
    // one table below 4 GB: descriptors hold byte offsets into it
    const int64_t tbytes = (int64_t)j_ncols * (j_ncols - 1) / 2 * j_pstride * 8;
    const bool flat = use_pairs && !two && tbytes <= (int64_t)0xFFFFFFFF;

    // 1. stage and validate the series. This thread's first column of the
    // series (and the one before it) is loaded first, then the archive's
    // offsets and columns (for the reduction), so that all of these loads
    // are in flight together
    const int K = j_asize;
    const bool arch_lds = K > 0 && j_alen <= acol_words;
    const int j0 = tid;
    int c0 = 0, a0 = 0;
    if (!bad0 && j0 < k) {
        c0 = gmem(j_cols)[beg + j0];
        if (j0 > 0) a0 = gmem(j_cols)[beg + j0 - 1];
    }
    if (arch_lds && !bad0) {
        // the offsets (K + 1 <= 2 x 64 values, two per thread) and the first
        // round of columns, loaded together; then any further rounds
        const int32_t *const aoff = J.arch_off;
        const uint16_t *const acols = J.arch_cols;
        const int bd = bdim;
        const int qa = tid < K ? tid : K;
        const int qb = tid + bd < K ? tid + bd : K;
        const int32_t oa = gmem(aoff)[qa], ob = gmem(aoff)[qb];
        auto put_col = [&](int q, uint16_t c) { s_acols[q] = c; };
        const int q0 = wave * (kStageRound * kWave) + lane;
        if (j_alen > 0) stage_round(acols, j_alen, q0, put_col);
        s_aoff[qa] = oa < 0 ? 0 : (oa > j_alen ? j_alen : oa);
        s_aoff[qb] = ob < 0 ? 0 : (ob > j_alen ? j_alen : ob);
        for (int q = q0 + kStageRound * bd; q < j_alen; q += kStageRound * bd)
            stage_round(acols, j_alen, q, put_col);
    }
    if (tid == 0) {
        s_bad = bad0;
        s_done = 0;
        s_n = 0;
    }
    if (!bad0)
        for (int q = tid; q < (j_ncols + 31) / 32; q += bdim) s_bits[q] = 0;
    __syncthreads();
    if (!bad0) {
        int lbad = 0;
        for (int j = tid; j < k; j += bdim) {
            const int c = j == j0 ? c0 : gmem(j_cols)[beg + j];
            if (c >= j_ncols) {
                lbad = 1;
            } else {
                const uint32_t bit = 1u << (c % 32);
                if (atomicOr(&s_bits[c / 32], bit) & bit) lbad = 1;
            }
            if (use_pairs) {
                if (j > 0) {
                    const int a = j == j0 ? a0 : gmem(j_cols)[beg + j - 1];
                    const int lo = a < c ? a : c, hi = a < c ? c : a;
                    if (hi < j_ncols) {
                        const int64_t pi = pair_index(lo, hi, j_ncols);
                        s_pd[j] = flat ? (int32_t)((uint32_t)(pi * j_pstride * 8) |
                                                   (a > c ? 1u : 0u))
                                       : (int32_t)pi | (a > c ? (int32_t)0x80000000 : 0);
                    }
                }
            } else {
                s_pd[j] = (int32_t)((uint32_t)c * (uint32_t)J.rows_pad * 2u);
            }
        }
        if (lbad) s_bad = 1;
    }
    {
        // the fields the waves read first after the barrier, loaded before it
        // (together, while the other waves finish staging)
        const int32_t w64 = J.w64, ipi = J.ipi, cpi = J.cpi, nch = J.nchunks,
                      neg = J.negative_trends;
        const uint64_t *const pairs = J.pairs;
        uint64_t *const sup = J.support;
        asm volatile("" ::"s"(w64), "s"(ipi), "s"(cpi), "s"(nch), "s"(neg), "s"(pairs), "s"(sup));
    }
    __syncthreads();
    if (idle) return;  // after the workgroup's last barrier
    const bool bad = s_bad != 0;
    const bool sup_lds = J.w64 <= sup_words;

    // 2. this wave's item: chunks [ch0, ch1), WPL at a time
    int nloc = 0;
    if (wave < J.ipi) {
        const int32_t ch0 = wave * J.cpi;
        const int32_t ch1 = ch0 + J.cpi < J.nchunks ? ch0 + J.cpi : J.nchunks;
        auto *S = gmem(J.support) + (int64_t)ind * J.w64;
        if (bad) {
            for (int32_t w = ch0 * 64 + lane; w < ch1 * 64 && w < J.w64; w += kWave) S[w] = 0;
        } else {
            const bool neg = J.negative_trends != 0;
            for (int32_t c0 = ch0; c0 < ch1; c0 += WPL) {
                if (use_pairs) {
                    const int w = c0 * 64 + lane;
                    const int wlim = J.w64 < ch1 * 64 ? J.w64 : ch1 * 64;
                    uint64_t fit[WPL];
                    const bool loose = J.tie_rule == EBIC_TIE_LOOSE;
                    const uint32_t tb = (uint32_t)(flat ? tbytes : 0);
                    if (two) {
                        if (neg)
                            pairs_dispatch<true, KB, WPL, TWO>(J.pairs, J.pairs_strict, loose,
                                                               J.pstride, false, 0, wlim, s_pd, k,
                                                               t, w, fit);
                        else
                            pairs_dispatch<false, KB, WPL, TWO>(J.pairs, J.pairs_strict, loose,
                                                                J.pstride, false, 0, wlim, s_pd, k,
                                                                t, w, fit);
                    } else if (neg) {
                        pairs_dispatch<true, KB, WPL, false>(J.pairs, nullptr, false, J.pstride,
                                                             flat, tb, wlim, s_pd, k, t, w, fit);
                    } else {
                        pairs_dispatch<false, KB, WPL, false>(J.pairs, nullptr, false, J.pstride,
                                                              flat, tb, wlim, s_pd, k, t, w, fit);
                    }
#pragma unroll
                    for (int v = 0; v < WPL; v++) {
                        const int wv = w + kWave * v, r0 = wv * 64;
                        uint64_t f = fit[v];
                        if (r0 + 64 > J.rows)
                            f &= r0 >= J.rows ? 0ull : ((1ull << (J.rows - r0)) - 1ull);
                        if (wv < wlim) {
                            S[wv] = f;
                            if (sup_lds) s_sup[wv] = f;
                            nloc += __popcll(f);
                        }
                    }
                } else {
                    const __amdgpu_buffer_rsrc_t rs =
                        make_rsrc(J.ranks, (uint32_t)((size_t)J.cols * J.rows_pad * 2));
                    for (int32_t chunk = c0; chunk < c0 + WPL && chunk < ch1; chunk++) {
                        const int w = chunk * 64 + lane;  // this lane's 64-row word
                        int lo = 0, hi = 0;
                        const int b0 = chunk * 64;
                        for (int b = 0; b < 64 && b0 + b < J.w64; b++) {
                            const int r = (b0 + b) * kWave + lane;
                            const uint64_t word =
                                block_support(rs, s_pd, k, t, neg, J.tie_rule, r * 2, r < J.rows);
                            lo = writelane((int)(uint32_t)word, b, lo);
                            hi = writelane((int)(uint32_t)(word >> 32), b, hi);
                        }
                        if (w < J.w64) {
                            const uint64_t f = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
                            S[w] = f;
                            if (sup_lds) s_sup[w] = f;
                            nloc += __popcll(f);
                        }
                    }
                }
            }
        }
    }

    // 3. the last wave to finish reduces the individual
    const int nw = wave_sum(nloc);
    int done = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) {
        atomicAdd(&s_n, nw);
        done = atomicAdd(&s_done, 1);
    }
    done = __builtin_amdgcn_readfirstlane(done);
    if (done != nwaves - 1) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (bad) {
        if (J.overlap)
            for (int j = lane; j < K; j += kWave) gmem(J.overlap)[(int64_t)ind * K + j] = 0;
        if (lane == 0) {
            gmem(J.count)[ind] = -1;
            gmem(J.fitness)[ind] = -1.0;
        }
        return;
    }
    const int n = __builtin_amdgcn_readfirstlane(s_n);
    const double score = (n >= J.min_rows && k >= J.k_score_min) ? ldexp((double)n, k) : 0.0;
    int mover = 0;
    int32_t my_h = 0;  // lane j keeps h of member j
    if (K > 0 && (score > 0.0 || J.overlap)) {
        auto hit = [&](int c) {
            return c >= 0 && c < J.cols && ((s_bits[c / 32] >> (c % 32)) & 1u);
        };
        int my_g = 0;  // lane j ends with g_j
        if (arch_lds) {
            // from LDS: one ballot per 64 archive columns marks those in the
            // series; lane j then counts the marks in its member's range
            const int nblk = (J.arch_len + kWave - 1) / kWave;
            for (int bb = 0; bb < nblk; bb++) {
                const int q = bb * kWave + lane;
                const uint64_t hm = __ballot(q < J.arch_len && hit(s_acols[q]));
                if (lane == 0) s_ahit[bb] = hm;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < K) {
                const int mb = s_aoff[lane], me = s_aoff[lane + 1];
                for (int q0 = mb & ~(kWave - 1); q0 < me; q0 += kWave) {
                    const int lo = mb > q0 ? mb - q0 : 0;
                    const int hi = me < q0 + kWave ? me - q0 : kWave;
                    const uint64_t range =
                        (hi == kWave ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
                    my_g += __popcll(s_ahit[q0 / kWave] & range);
                }
            }
        } else {
            // from global memory: lane j holds arch_off[j] (one load for all
            // members); members' first 64 columns loaded kGGroup at a time
            const int32_t aoff = lane <= K ? gmem(J.arch_off)[lane] : 0;
            const int32_t aoff_k = gmem(J.arch_off)[K];
            auto clampo = [&](int32_t o) {
                return o < 0 ? 0 : (o > J.arch_len ? J.arch_len : o);
            };
            for (int j0 = 0; j0 < K; j0 += kGGroup) {
                int col[kGGroup], mb[kGGroup], me[kGGroup];
#pragma unroll
                for (int u = 0; u < kGGroup; u++) {
                    const int j = j0 + u < K ? j0 + u : K - 1;
                    mb[u] = clampo(__builtin_amdgcn_readlane(aoff, j));
                    me[u] = clampo(j + 1 < kWave ? __builtin_amdgcn_readlane(aoff, j + 1) : aoff_k);
                    const int q = mb[u] + lane;
                    col[u] = q < me[u] ? (int)gmem(J.arch_cols)[q] : -1;
                }
#pragma unroll
                for (int u = 0; u < kGGroup; u++) {
                    if (j0 + u < K) {  // uniform; no break, so the loop unrolls fully
                        int g = __popcll(__ballot(hit(col[u])));
                        for (int q0 = mb[u] + kWave; q0 < me[u]; q0 += kWave) {
                            const int q = q0 + lane;
                            g += __popcll(__ballot(hit(q < me[u] ? (int)gmem(J.arch_cols)[q] : -1)));
                        }
                        if (lane == j0 + u) my_g = g;
                    }
                }
            }
        }
        // members whose rows must be counted: kHGroup per pass, kHWords
        // words per lane and pass, all archive loads of a pass issued
        // together; the individual's own words come from LDS when staged
        const bool my_need = lane < K && n > 0 &&
                             (J.overlap || 1000LL * my_g > (long long)J.overlap_permille * k);
        uint64_t need = __ballot(my_need);
        const auto *S = gmem(J.support) + (int64_t)ind * J.w64;
        while (need) {
            int js[kHGroup];
#pragma unroll
            for (int g = 0; g < kHGroup; g++) {
                js[g] = need ? __ffsll((unsigned long long)need) - 1 : js[g > 0 ? g - 1 : 0];
                need &= need - 1;
            }
            int hp[kHGroup];
#pragma unroll
            for (int g = 0; g < kHGroup; g++) hp[g] = 0;
            for (int w0 = lane; w0 < J.w64; w0 += kWave * kHWords) {
                uint64_t aw[kHGroup][kHWords];
#pragma unroll
                for (int u = 0; u < kHWords; u++) {
                    const int w = w0 + kWave * u;
#pragma unroll
                    for (int g = 0; g < kHGroup; g++)
                        aw[g][u] = w < J.w64 ? gmem(J.arch_support)[(int64_t)js[g] * J.w64 + w] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < kHWords; u++) {
                    const int w = w0 + kWave * u;
                    const uint64_t sw = w < J.w64 ? (sup_lds ? s_sup[w] : S[w]) : 0ull;
#pragma unroll
                    for (int g = 0; g < kHGroup; g++) hp[g] += __popcll(sw & aw[g][u]);
                }
            }
#pragma unroll
            for (int g = 0; g < kHGroup; g++) {
                const int h = wave_sum(hp[g]);
                if (lane == js[g]) my_h = h;  // a repeated member writes the same h
            }
        }
        const bool over = lane < K && 1000LL * my_h * my_g > (long long)J.overlap_permille * n * k;
        mover = __popcll(__ballot(over));
    }
    if (J.overlap && lane < K) gmem(J.overlap)[(int64_t)ind * K + lane] = my_h;
    if (lane == 0) {
        gmem(J.count)[ind] = n;
        gmem(J.fitness)[ind] = ldexp(score, -mover);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: the batch object and its autotuner.
// ---------------------------------------------------------------------------

struct Batch {
    int device = 0;
    int32_t flags = 0;
    bool two = false;          // some job reads both pair tables (strict or loose rule)
    std::vector<DevJob> jobs;
    std::vector<int> perm;     // scratch of lay_out
    DevJob *d_jobs = nullptr;  // device: DevJob[njobs] by population size, descending;
    int64_t *d_sched = nullptr;  // then the schedule (phase starts, phase rounds)
    int32_t cap_jobs = 0;      // capacity of d_jobs / h_stage
    const ebic_allocator *al = nullptr;  // device memory of d_jobs (NULL: hipMalloc)
    hipStream_t al_stream = nullptr;
    void *h_stage = nullptr;   // pinned staging of the table
    std::vector<void *> scratch;
    int64_t total_ind = 0;
    int64_t ph1 = 0;           // first slot past phase 0 (kernel argument, kept alive for a graph)
    int32_t njobs = 0;
    int waves = 1;             // waves per individual: the largest items per individual
    int32_t ipw = 1;           // individuals per workgroup
    int32_t total32 = 0;       // total_ind as a kernel argument
    int32_t sup_words = 0;     // LDS support words per individual (0: global only)
    int32_t bits_words = 1;    // LDS column-bitmap words per individual
    int32_t acol_words = 0;    // LDS archive columns per individual (0: global only)
    int kb = 4;                // pair-bitmap loads in flight (template)
    int wpl = 1;               // 64-row words per lane (template)
    int cpi = 1;               // chunk groups (of wpl chunks) per item
    bool tuned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // timing: two events per profiled run (around the kernel)
    std::vector<hipEvent_t> events;
    int32_t prof_cap = 0, prof_used = 0;
};

namespace {

// Chunk groups per item before any tuning (ebic_batch_set_tuning or
// EBIC_BATCH_TUNE change it): 0 = chosen per job, one chunk per item up to
// two chunks, two up to four, else four (with one word per lane), so that a
// 10,000-row individual takes two waves and shares its workgroup with
// another; the shapes the tuner picks for 10,000 and 40,000 rows.
constexpr int kDefaultCpi = 0;

int check_job(const ebic_job *j, int idx) {
    const ebic_matrix *m = &j->matrix;
    if (!m->d_ranks || m->rows < 1 || m->rows > EBIC_MAX_ROWS || m->cols < 2 ||
        m->cols > EBIC_MAX_COLS || m->rows_pad != rows_padded(m->rows) ||
        (int64_t)m->cols * m->rows_pad > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad matrix view", idx);
    int rc = check_eval_params(&j->params);
    if (rc) return rc;
    const ebic_archive *a = &j->archive;
    if (a->size < 0 || a->size > EBIC_MAX_ARCHIVE ||
        (a->size > 0 && (!a->d_support || !a->d_offsets || !a->d_cols || a->length < 0)))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad archive", idx);
    const ebic_population *p = &j->population;
    if (p->size < 0 || (p->size > 0 && (!p->d_offsets || !p->d_cols)))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad population", idx);
    if (p->size > 0 && (!j->out.d_fitness || !j->out.d_count))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: fitness and count outputs are required", idx);
    return EBIC_OK;
}

DevJob make_devjob(const ebic_job &j, int32_t flags) {
    DevJob d{};
    d.ranks = j.matrix.d_ranks;
    d.pairs = j.matrix.d_pairs;
    d.pairs_strict = j.matrix.d_pairs_strict;
    d.rows = j.matrix.rows;
    d.cols = j.matrix.cols;
    d.rows_pad = j.matrix.rows_pad;
    d.w32 = j.matrix.rows_pad / 32;
    d.w64 = j.matrix.rows_pad / 64;
    d.pstride = pair_words(j.matrix.rows_pad);
    d.mode = (j.matrix.d_pairs && !(flags & EBIC_BATCH_GATHER)) ? 1 : 0;
    d.nchunks = (j.matrix.rows_pad + kItemRows - 1) / kItemRows;
    d.pop_size = j.population.size;
    d.pop_len = j.population.length;
    d.pop_off = j.population.d_offsets;
    d.pop_cols = j.population.d_cols;
    d.order = j.population.d_order;
    d.arch_size = j.archive.size;
    d.arch_len = j.archive.length;
    d.arch_support = j.archive.d_support;
    d.arch_off = j.archive.d_offsets;
    d.arch_cols = j.archive.d_cols;
    d.approx_permille = j.params.approx_permille;
    d.negative_trends = j.params.negative_trends;
    d.overlap_permille = j.params.overlap_permille;
    d.min_rows = j.params.min_rows;
    d.k_score_min = j.params.k_score_min;
    d.tie_rule = j.params.tie_rule;
    d.fitness = j.out.d_fitness;
    d.count = j.out.d_count;
    d.support = j.out.d_support;
    d.overlap = j.out.d_overlap;
    return d;
}

// What a launch needs besides the job table: the workgroup shape, the LDS
// partition and the grid.
struct Layout {
    bool two = false;        // some job reads both pair tables
    int waves = 1;           // waves per individual: the largest items per individual
    int32_t ipw = 1;         // individuals per workgroup
    int32_t sup_words = 0;   // LDS support words per individual (0: global only)
    int32_t bits_words = 1;  // LDS column-bitmap words per individual
    int32_t acol_words = 0;  // LDS archive columns per individual (0: global only)
    int64_t total_ind = 0;   // individuals (slots)
    int64_t ph1 = 0;         // first slot past phase 0
};

constexpr size_t table_bytes_max(int32_t n) {
    return sizeof(DevJob) * n + sizeof(int64_t) * 2 * n;
}
size_t table_bytes(int32_t n) { return table_bytes_max(n); }
// Size of the array behind the allocation-free batched evaluation.
constexpr size_t kNoAllocScratchBytes = 16384;

// Lay the items out for `cpi` groups of `wpl` chunks per item (0: chosen per
// job, as for kDefaultCpi; more when an individual would need more than
// kMaxWaves items) and write the job table (jobs by population size,
// descending) and the schedule (phase starts, phase rounds) to h,
// table_bytes(n) bytes. `perm` is scratch for n ints. Allocates nothing.
Layout lay_out(DevJob *jobs, int32_t n, int cpi, int wpl, int *perm, char *h) {
    Layout L;
    for (int32_t i = 0; i < n; i++) {
        const DevJob &d = jobs[i];
        L.two |= d.mode == 1 && d.tie_rule != EBIC_TIE_INDEX && d.pairs_strict != nullptr;
    }
    // Items per individual: `cpi` groups each, at most kMaxWaves items. The
    // workgroup has as many waves as the job with the most items needs, so
    // when jobs of different row counts share a launch, a small job's
    // workgroups would carry idle waves through staging and hold wave
    // slots; there the larger jobs' items are widened to at most
    // kMixedWaves per individual.
    auto items = [&](DevJob &d, int32_t waves_max) {
        // whole groups per item, so that no two items share a group
        int32_t cpc = cpi > 0 ? cpi * wpl : d.nchunks <= 2 ? 1 : d.nchunks <= 4 ? 2 : 4;
        const int32_t need = (d.nchunks + waves_max - 1) / waves_max;
        if (cpc < need) cpc = (need + wpl - 1) / wpl * wpl;
        d.cpi = cpc < d.nchunks ? cpc : d.nchunks;
        if (d.cpi < 1) d.cpi = 1;
        d.ipi = (d.nchunks + d.cpi - 1) / d.cpi;
    };
    int32_t ipi_min = kMaxWaves, ipi_max = 0, busy = 0;
    for (int32_t i = 0; i < n; i++) {
        items(jobs[i], kMaxWaves);
        if (jobs[i].pop_size > 0) {
            busy++;
            ipi_min = jobs[i].ipi < ipi_min ? jobs[i].ipi : ipi_min;
            ipi_max = jobs[i].ipi > ipi_max ? jobs[i].ipi : ipi_max;
        }
    }
    if (busy > 1 && ipi_max > kMixedWaves && ipi_min < ipi_max)
        for (int32_t i = 0; i < n; i++)
            if (jobs[i].ipi > kMixedWaves) items(jobs[i], kMixedWaves);
    int32_t wmax = 0, cmax = 0, amax = 0;
    for (int32_t i = 0; i < n; i++) {
        const DevJob &d = jobs[i];
        L.waves = d.ipi > L.waves ? d.ipi : L.waves;
        wmax = d.w64 > wmax ? d.w64 : wmax;
        cmax = d.cols > cmax ? d.cols : cmax;
        amax = d.arch_len > amax ? d.arch_len : amax;
    }
    L.sup_words = wmax <= kSupLdsWords ? wmax : 0;
    L.bits_words = (cmax + 31) / 32;
    L.acol_words = amax <= kArchLdsCols ? amax : 0;
    const size_t ind_lds = lds_ind_bytes(L.sup_words, L.bits_words, L.acol_words);
    while (L.ipw * 2 <= kMaxIpw && L.ipw * 2 * L.waves <= kGroupWaves &&
           (size_t)L.ipw * 2 * ind_lds <= kGroupLds)
        L.ipw *= 2;
    // Individuals of all jobs are interleaved round-robin, so that each
    // job's longest-first order holds across the batch: with the jobs stored
    // by population size, descending, phase p takes one individual of each
    // of the first n - p jobs per round, over the rounds that those jobs
    // still have. (Stable insertion sort: no temporary buffer.)
    for (int32_t i = 0; i < n; i++) {
        int32_t q = i;
        while (q > 0 && jobs[perm[q - 1]].pop_size < jobs[i].pop_size) {
            perm[q] = perm[q - 1];
            q--;
        }
        perm[q] = i;
    }
    const size_t jbytes = sizeof(DevJob) * n;
    DevJob *hj = reinterpret_cast<DevJob *>(h);
    int64_t *ph_start = reinterpret_cast<int64_t *>(h + jbytes);
    int64_t *ph_round = ph_start + n;
    int64_t start = 0;
    for (int32_t p = 0; p < n; p++) {
        hj[p] = jobs[perm[p]];
        const int64_t first = p == 0 ? 0 : jobs[perm[n - p]].pop_size;
        ph_start[p] = start;
        ph_round[p] = first;
        start += (int64_t)(n - p) * (jobs[perm[n - 1 - p]].pop_size - first);
    }
    L.total_ind = start;
    L.ph1 = n > 1 ? ph_start[1] : start;
    return L;
}

// Lay the batch's items out for `cpi` chunk groups per item and queue the
// table's upload on `stream` from pinned staging, growing the device table
// when needed.
int upload_table(Batch *b, int cpi, hipStream_t stream) {
    b->cpi = cpi;
    const int32_t n = b->njobs;
    const size_t bytes = table_bytes(n);
    const bool moved = n > b->cap_jobs;  // a new device table
    if (n > b->cap_jobs) {
        if (b->d_jobs) device_release(b->al, b->d_jobs, b->al_stream);
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        b->d_jobs = nullptr;
        b->h_stage = nullptr;
        b->cap_jobs = 0;
        void *mem = device_alloc(b->al, bytes, b->al_stream);
        if (!mem) return fail(EBIC_ERR_OOM, "batch job table (%zu bytes)", bytes);
        b->d_jobs = static_cast<DevJob *>(mem);
        EBIC_HIP(hipHostMalloc(&b->h_stage, bytes, hipHostMallocDefault));
        b->cap_jobs = n;
    }
    b->perm.resize(n);
    const Layout L =
        lay_out(b->jobs.data(), n, cpi, b->wpl, b->perm.data(), static_cast<char *>(b->h_stage));
    if (moved || L.two != b->two || L.waves != b->waves || L.ipw != b->ipw ||
        L.total_ind != b->total_ind || L.ph1 != b->ph1 || L.sup_words != b->sup_words ||
        L.bits_words != b->bits_words || L.acol_words != b->acol_words) {
        // another kernel, grid or argument: a graph of the old launch is
        // rebuilt on the next run
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->two = L.two;
    }
    b->waves = L.waves;
    b->ipw = L.ipw;
    b->sup_words = L.sup_words;
    b->bits_words = L.bits_words;
    b->acol_words = L.acol_words;
    b->total_ind = L.total_ind;
    b->total32 = (int32_t)(L.total_ind < INT32_MAX ? L.total_ind : INT32_MAX);
    b->ph1 = L.ph1;
    b->d_sched = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(b->d_jobs) +
                                             sizeof(DevJob) * n);
    EBIC_HIP(hipMemcpyAsync(b->d_jobs, b->h_stage, bytes, hipMemcpyHostToDevice, stream));
    return EBIC_OK;
}

template <bool TWO>
void *kernel_fn(int kb, int wpl) {
    if (wpl == 2)
        return kb == 4 ? reinterpret_cast<void *>(batch_kernel<4, 2, TWO>)
                       : reinterpret_cast<void *>(batch_kernel<2, 2, TWO>);
    if (kb == 8) return reinterpret_cast<void *>(batch_kernel<8, 1, TWO>);
    return kb == 4 ? reinterpret_cast<void *>(batch_kernel<4, 1, TWO>)
                   : reinterpret_cast<void *>(batch_kernel<2, 1, TWO>);
}
// The kernel for the batch: with the strict-table path only when some job
// takes it, so the others keep the leaner kernel.
void *kernel_fn(const Batch *b, int kb, int wpl) {
    return b->two ? kernel_fn<true>(kb, wpl) : kernel_fn<false>(kb, wpl);
}

size_t lds_bytes(int32_t ipw, int32_t sup_words, int32_t bits_words, int32_t acol_words) {
    return (size_t)ipw * lds_ind_bytes(sup_words, bits_words, acol_words);
}
size_t lds_bytes(const Batch *b) {
    return lds_bytes(b->ipw, b->sup_words, b->bits_words, b->acol_words);
}
// workgroups: ipw slots each (g, g + G, ...)
unsigned groups(int64_t total_ind, int32_t ipw) { return (unsigned)((total_ind + ipw - 1) / ipw); }

int launch_batch(Batch *b, hipStream_t stream) {
    void *args[] = {&b->d_jobs,     &b->d_sched, &b->njobs, &b->ph1,    &b->sup_words,
                    &b->bits_words, &b->acol_words, &b->ipw, &b->waves, &b->total32};
    EBIC_HIP(hipLaunchKernel(kernel_fn(b, b->kb, b->wpl), dim3(groups(b->total_ind, b->ipw)),
                             dim3(b->ipw * b->waves * kWave), args, lds_bytes(b), stream));
    return EBIC_OK;
}

int build_graph(Batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    // one kernel node (no stream capture)
    hipGraphNode_t node = nullptr;
    void *args[] = {&b->d_jobs,     &b->d_sched, &b->njobs, &b->ph1,    &b->sup_words,
                    &b->bits_words, &b->acol_words, &b->ipw, &b->waves, &b->total32};
    hipKernelNodeParams pk{};
    pk.func = kernel_fn(b, b->kb, b->wpl);
    pk.gridDim = dim3(groups(b->total_ind, b->ipw));
    pk.blockDim = dim3(b->ipw * b->waves * kWave);
    pk.sharedMemBytes = (unsigned)lds_bytes(b);
    pk.kernelParams = args;
    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &pk);
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return check_hip(e, "batch graph");
    return EBIC_OK;
}

// ---- autotuner: item shapes, cached per batch shape ----

constexpr int kTuneLaunches = 10;     // launches per timed sample
constexpr float kTuneMargin = 0.98f;  // required gain over the current best

std::mutex g_tune_mu;
struct Shape {
    int cpi, kb, wpl;
};
std::map<std::string, Shape> g_tune;

bool valid_shape(int cpi, int kb, int wpl) {
    return (cpi == 1 || cpi == 2 || cpi == 4) && (wpl == 1 || wpl == 2) &&
           (kb == 2 || kb == 4 || (kb == 8 && wpl == 1));
}
bool g_tune_loaded = false;

const char *tune_file() { return getenv("EBIC_TUNE_CACHE"); }

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = tune_file();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    // entries look like  "key": [cpi, kb, wpl]  inside one JSON object
    size_t pos = 0;
    for (;;) {
        const size_t q0 = text.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        int a = 0, c = 0, v = 0;
        if (sscanf(text.c_str() + q1 + 1, " : [ %d , %d , %d ]", &a, &c, &v) == 3 &&
            valid_shape(a, c, v))
            g_tune[text.substr(q0 + 1, q1 - q0 - 1)] = {a, c, v};
        const size_t close = text.find(']', q1);
        if (close == std::string::npos) break;
        pos = close + 1;
    }
}

void tune_save_locked() {
    const char *path = tune_file();
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{");
    bool first = true;
    for (auto &kv : g_tune) {
        fprintf(f, "%s\n \"%s\": [%d, %d, %d]", first ? "" : ",", kv.first.c_str(),
                kv.second.cpi, kv.second.kb, kv.second.wpl);
        first = false;
    }
    fprintf(f, "\n}\n");
    fclose(f);
}

std::string tune_key(const Batch *b) {
    int32_t w = 0, mode = 0;
    for (const DevJob &d : b->jobs) {
        w = d.w64 > w ? d.w64 : w;
        mode |= 1 << d.mode;
    }
    char buf[128];
    snprintf(buf, sizeof buf, "m%d_w%d_i%lld_j%d%s", mode, w, (long long)b->total_ind, b->njobs,
             b->two ? "_s" : "");
    return buf;
}

// Time every item shape (chunk groups per item, loads in flight, words per
// lane) on this batch's inputs with HIP events around blocks of evaluation
// launches (median of 3 blocks) and keep the fastest. Results never depend
// on the choice.
int tune(Batch *b, hipStream_t stream) {
    b->tuned = true;
    const std::string key = tune_key(b);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            b->kb = it->second.kb;
            b->wpl = it->second.wpl;
            return upload_table(b, it->second.cpi, stream);
        }
    }
    int32_t maxch = 1;
    for (const DevJob &d : b->jobs) maxch = d.nchunks > maxch ? d.nchunks : maxch;
    hipEvent_t e0, e1;
    EBIC_HIP(hipEventCreate(&e0));
    EBIC_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    Shape pick{1, 2, 1};
    int rc = EBIC_OK;
    for (int wpl : {1, 2}) {
        if (wpl > maxch) break;
        for (int cpi : {1, 2, 4}) {
            if (cpi > 1 && cpi * wpl > maxch) break;
            for (int kb : {2, 4, 8}) {
                // two words per lane leave room for narrow counters only
                // with four loads in flight: not a candidate
                if (wpl == 2 && kb >= 4) continue;
                b->kb = kb;
                b->wpl = wpl;
                rc = upload_table(b, cpi, stream);
                if (rc == EBIC_OK) rc = launch_batch(b, stream);  // warm-up
                float t[3];
                for (int r = 0; r < 3 && rc == EBIC_OK; r++) {
                    (void)hipEventRecord(e0, stream);
                    for (int l = 0; l < kTuneLaunches && rc == EBIC_OK; l++)
                        rc = launch_batch(b, stream);
                    (void)hipEventRecord(e1, stream);
                    (void)hipEventSynchronize(e1);
                    (void)hipEventElapsedTime(&t[r], e0, e1);
                }
                if (rc) break;
                std::sort(t, t + 3);
                // a later (larger) shape must win clearly, so that timing
                // noise does not flip the choice from run to run
                if (t[1] < best * kTuneMargin) {
                    best = t[1];
                    pick = {cpi, kb, wpl};
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = pick;
        tune_save_locked();
    }
    b->kb = pick.kb;
    b->wpl = pick.wpl;
    return upload_table(b, pick.cpi, stream);
}

}  // namespace

// Re-target a batch at a new set of jobs (every job must bring its support
// output): the job table and the start arrays go to the device with one
// asynchronous copy on `stream` from pinned staging, reusing the device
// table when it is large enough. Creates the batch when *bp is NULL.
int batch_set(Batch **bp, const ebic_job *jobs, int32_t njobs, hipStream_t stream,
              const ebic_allocator *al) {
    if (!bp || njobs < 1 || !jobs) return fail(EBIC_ERR_INVALID_ARG, "no jobs");
    for (int i = 0; i < njobs; i++) {
        int rc = check_job(&jobs[i], i);
        if (rc) return rc;
        if (jobs[i].population.size > 0 && !jobs[i].out.d_support)
            return fail(EBIC_ERR_INVALID_ARG, "job %d: support output required", i);
    }
    Batch *b = *bp;
    if (!b) {
        b = new Batch();
        b->al = al;
        b->al_stream = stream;
        EBIC_HIP(hipGetDevice(&b->device));
        b->cpi = kDefaultCpi;
        *bp = b;
    }
    b->jobs.clear();
    for (int i = 0; i < njobs; i++) b->jobs.push_back(make_devjob(jobs[i], 0));
    // new jobs: a graph of the old launch (its job count among the
    // arguments) is rebuilt on the next run
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->njobs = njobs;
    return upload_table(b, b->cpi, stream);
}

int batch_create(const ebic_job *jobs, int32_t njobs, int32_t flags, Batch **out) {
    if (!out || njobs < 1 || !jobs) return fail(EBIC_ERR_INVALID_ARG, "no jobs");
    for (int i = 0; i < njobs; i++) {
        int rc = check_job(&jobs[i], i);
        if (rc) return rc;
    }
    Batch *b = new Batch();
    b->flags = flags;
    b->cpi = kDefaultCpi;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return check_hip(e, "hipGetDevice");
    }
    b->njobs = njobs;
    for (int i = 0; i < njobs; i++) {
        DevJob d = make_devjob(jobs[i], flags);
        if (!d.support && d.pop_size > 0) {
            void *p = nullptr;
            e = hipMalloc(&p, (size_t)d.pop_size * d.w64 * sizeof(uint64_t));
            if (e != hipSuccess) {
                batch_destroy(b);
                return check_hip(e, "hipMalloc(support scratch)");
            }
            b->scratch.push_back(p);
            d.support = static_cast<uint64_t *>(p);
        }
        b->jobs.push_back(d);
    }
    int rc = upload_table(b, b->cpi, nullptr);
    if (rc == EBIC_OK) {
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) rc = check_hip(e, "batch job table");
    }
    if (rc) {
        batch_destroy(b);
        return rc;
    }
    *out = b;
    return EBIC_OK;
}

int batch_run(Batch *b, hipStream_t stream) {
    if (!b) return fail(EBIC_ERR_INVALID_ARG, "batch is NULL");
    if (b->total_ind == 0) return EBIC_OK;
    if (b->total_ind > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "%lld individuals in one launch",
                    (long long)b->total_ind);
    if ((b->flags & EBIC_BATCH_TUNE) && !b->tuned) {
        int rc = tune(b, stream);
        if (rc) return rc;
    }
    if ((b->flags & EBIC_BATCH_GRAPH) && !b->exec) {
        EBIC_HIP(hipStreamSynchronize(stream));  // the table upload must land first
        int rc = build_graph(b);
        if (rc) return rc;
    }
    hipEvent_t *ev = nullptr;
    if (b->prof_used < b->prof_cap) ev = &b->events[2 * b->prof_used++];
    if (ev) EBIC_HIP(hipEventRecord(ev[0], stream));
    if (b->exec) {
        EBIC_HIP(hipGraphLaunch(b->exec, stream));
    } else {
        int rc = launch_batch(b, stream);
        if (rc) return rc;
    }
    if (ev) EBIC_HIP(hipEventRecord(ev[1], stream));
    return EBIC_OK;
}

int batch_archive_fields(Batch *b, int32_t job, int32_t **size, int32_t **len) {
    if (!b || job < 0 || job >= b->njobs || !b->d_jobs)
        return fail(EBIC_ERR_INVALID_ARG, "bad batch or job");
    // the table holds the jobs by population size, descending (stable)
    int32_t at = 0;
    for (int32_t i = 0; i < b->njobs; i++)
        if (b->jobs[i].pop_size > b->jobs[job].pop_size ||
            (b->jobs[i].pop_size == b->jobs[job].pop_size && i < job))
            at++;
    DevJob *d = b->d_jobs + at;
    *size = &d->arch_size;
    *len = &d->arch_len;
    return EBIC_OK;
}

int batch_tuning(Batch *b, int32_t *cpi, int32_t *kb, int32_t *wpl) {
    if (!b) return fail(EBIC_ERR_INVALID_ARG, "batch is NULL");
    if (cpi) *cpi = b->cpi;
    if (kb) *kb = b->kb;
    if (wpl) *wpl = b->wpl;
    return EBIC_OK;
}

int batch_set_tuning(Batch *b, int32_t cpi, int32_t kb, int32_t wpl) {
    if (!b) return fail(EBIC_ERR_INVALID_ARG, "batch is NULL");
    if (!valid_shape(cpi, kb, wpl))
        return fail(EBIC_ERR_INVALID_ARG, "item shape (%d, %d, %d): chunk groups per item 1, 2 "
                    "or 4, loads in flight 2, 4 or 8 (8 with one word per lane), words per lane 1 or 2",
                    cpi, kb, wpl);
    // a graph holds the old grid and kernel: rebuilt on the next run
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->kb = kb;
    b->wpl = wpl;
    b->tuned = true;
    int rc = upload_table(b, cpi, nullptr);
    if (rc) return rc;
    EBIC_HIP(hipStreamSynchronize(nullptr));
    return EBIC_OK;
}

int batch_profile(Batch *b, int32_t n) {
    if (!b || n < 0) return fail(EBIC_ERR_INVALID_ARG, "bad batch or count");
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.clear();
    b->prof_cap = b->prof_used = 0;
    for (int32_t i = 0; i < 2 * n; i++) {
        hipEvent_t e;
        EBIC_HIP(hipEventCreate(&e));
        b->events.push_back(e);
    }
    b->prof_cap = n;
    return EBIC_OK;
}

int batch_timings(Batch *b, float *ms, int32_t *n) {
    if (!b || !ms || !n || *n < 0) return fail(EBIC_ERR_INVALID_ARG, "bad arguments");
    const int32_t m = b->prof_used < *n ? b->prof_used : *n;
    for (int32_t i = 0; i < m; i++) {
        hipEvent_t *ev = &b->events[2 * i];
        EBIC_HIP(hipEventSynchronize(ev[1]));
        EBIC_HIP(hipEventElapsedTime(&ms[i], ev[0], ev[1]));
    }
    *n = m;
    return EBIC_OK;
}

int batch_destroy(Batch *b) {
    if (!b) return EBIC_OK;
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_jobs) device_release(b->al, b->d_jobs, b->al_stream);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    for (void *p : b->scratch) (void)hipFree(p);
    delete b;
    return EBIC_OK;
}

// ---------------------------------------------------------------------------
// Batched evaluation that allocates nothing: the job table and schedule go
// to a fixed device array of this library instead of a batch's allocation.
// ---------------------------------------------------------------------------

namespace {

constexpr int kNoAllocDevices = 64;  // devices a process can use this entry point on
static_assert(table_bytes_max(EBIC_NOALLOC_MAX_JOBS) <= kNoAllocScratchBytes,
              "the job table of the largest call fits the array");

// The array itself. Its name in host code is a host-side stand-in, not the
// device address: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu[kNoAllocDevices];  // one call at a time per device
void *g_noalloc_ptr[kNoAllocDevices];       // the array's address on each device

// The array's address on `dev` (current), looked up once per device with
// the device's mutex held.
int scratch_address(int dev, void **out) {
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(EBIC_ERR_DEVICE, "scratch array has no address on device %d", dev);
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return EBIC_OK;
}

}  // namespace

int batch_run_noalloc(const ebic_job *jobs, int32_t njobs, hipStream_t stream) {
    if (!jobs || njobs < 1) return fail(EBIC_ERR_INVALID_ARG, "no jobs");
    if (njobs > EBIC_NOALLOC_MAX_JOBS)
        return fail(EBIC_ERR_INVALID_ARG, "%d jobs: the allocation-free batched evaluation "
                    "takes at most %d", njobs, EBIC_NOALLOC_MAX_JOBS);
    for (int i = 0; i < njobs; i++) {
        int rc = check_job(&jobs[i], i);
        if (rc) return rc;
        if (jobs[i].population.size > 0 && !jobs[i].out.d_support)
            return fail(EBIC_ERR_INVALID_ARG, "job %d: support output required", i);
    }
    int dev = 0;
    EBIC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices)
        return fail(EBIC_ERR_INVALID_ARG, "device %d: at most %d devices", dev, kNoAllocDevices);
    DevJob dj[EBIC_NOALLOC_MAX_JOBS];
    int perm[EBIC_NOALLOC_MAX_JOBS];
    alignas(16) char h[table_bytes_max(EBIC_NOALLOC_MAX_JOBS)];
    for (int i = 0; i < njobs; i++) dj[i] = make_devjob(jobs[i], 0);
    constexpr int kb = 4, wpl = 1;  // the shape ebic_evaluate_batched runs untuned
    Layout L = lay_out(dj, njobs, kDefaultCpi, wpl, perm, h);
    if (L.total_ind == 0) return EBIC_OK;
    if (L.total_ind > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "%lld individuals in one launch", (long long)L.total_ind);
    std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
    void *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    // the table from the stack: a copy from pageable memory has read it when
    // the call returns
    EBIC_HIP(hipMemcpyAsync(base, h, table_bytes(njobs), hipMemcpyHostToDevice, stream));
    DevJob *d_jobs = static_cast<DevJob *>(base);
    int64_t *d_sched = reinterpret_cast<int64_t *>(static_cast<char *>(base) +
                                                   sizeof(DevJob) * njobs);
    int32_t n = njobs;
    int32_t total = (int32_t)L.total_ind;
    int32_t ipw = L.ipw, wpi = L.waves;
    void *args[] = {&d_jobs,       &d_sched,      &n,   &L.ph1, &L.sup_words,
                    &L.bits_words, &L.acol_words, &ipw, &wpi,   &total};
    void *fn = L.two ? kernel_fn<true>(kb, wpl) : kernel_fn<false>(kb, wpl);
    EBIC_HIP(hipLaunchKernel(fn, dim3(groups(L.total_ind, L.ipw)),
                             dim3(L.ipw * L.waves * kWave), args,
                             lds_bytes(L.ipw, L.sup_words, L.bits_words, L.acol_words), stream));
    // the next call may rewrite the array only after this launch has read it
    EBIC_HIP(hipStreamSynchronize(stream));
    return EBIC_OK;
}

}  // namespace ebic
