// The generations of the evolutionary loop (Sec. 2.4, steps 3-7) on the
// device: after the first population (drawn on the host, step 1) every
// generation runs as kernels, with no population, score or support crossing
// to the host; the host only reads a status block to learn whether the run
// has stopped and how large the top-rank list is.
//
// The draws stay those of the host loop, one SplitMix64 stream per run.
// SplitMix64 is counter-based (the n-th output is the finaliser applied to
// seed + n * gamma), and a mutation attempt's draws never depend on whether
// an earlier attempt's child was rejected (tabu hits only decide which
// children fill the population and when the loop ends). So a generation's
// attempts are found in parallel: every draw offset of a span is tried as
// the start of an attempt to learn how many draws an attempt starting there
// takes; the chain of attempts from the span's start is then extracted
// (segment walks from every possible entry offset, then the segments linked
// in order); every attempt's child is built and looked up in the tabu set
// at once; and the sequential rules (a slot's attempt limit, the tabu-hit
// limit, the population filling up) are applied afterwards with block-wide
// scans, so the result is the sequential loop's, attempt for attempt.
//
// Readings (top-rank list, crowding, tournament, operators, tabu key) are
// the ones the host loop in job.h / run.cpp follows.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "device.h"
#include "internal.h"
#include "job.h"

namespace ebic {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr int kDlMaxT = 16;        // largest tournament of the device loop
constexpr int kDlMaxP = 8192;      // largest population (sort keys of the list update in LDS)
constexpr int kSeg = 256;          // draw offsets per segment of the chain walk
constexpr int kSpanMax = 65535;    // draw offsets tried per chunk
constexpr int kChunkMax = 6144;    // attempts per chunk
constexpr int kDedupSlots = 8192;  // LDS hash table of a chunk's children (load <= 3/4)
constexpr int kBlock = 1024;       // threads of the single-workgroup kernels
constexpr int kChildWaves = 4;     // waves per workgroup of the child kernel
constexpr int kMaxCols = EBIC_MAX_COLS;

// What the kernels need of the run parameters, and the shapes.
struct DlParams {
    int32_t P, C, W, kmin, kmax, K, T, G;
    int32_t max_att, min_rows, k_score_min, neg, theta;
    int32_t opw[5];          // operator weights (all-zero op_permille: 200 each)
    int64_t max_hits;
    uint64_t tabu_mask;      // table slots - 1 (a power of two)
    int32_t tabu_cap;        // arena entries
    int32_t span_e;          // largest draw count of an attempt on the segment walk
};

// Device state of the run, read by the host between kernels.
struct DlState {
    uint64_t rng;         // SplitMix64 state: the next draw is mix(rng + gamma)
    int64_t hits;         // tabu hits so far (cumulative over the run)
    int64_t evaluations;  // individuals scored
    int32_t g;            // populations scored
    int32_t stop;         // EBIC_STOP_* once the run ends
    int32_t nA;           // top-rank list size
    int32_t Nn;           // next population filled so far
    int32_t att;          // attempts spent on the slot being filled
    int32_t need_more;    // the fill needs another chunk of attempts
    int32_t chunk_n;      // attempts extracted for the current chunk
    int32_t chunk_span;   // draw offsets tried for the current chunk
    int32_t tabu_n;       // tabu entries
    int32_t error;        // the tabu arena is full
    int32_t arch_len;     // columns of the packed top-rank list
    int32_t slow;         // chunks whose chain needed the sequential walk
    int32_t over;         // the run has stopped: every later kernel does nothing
    int32_t pending;      // the chunk's accepted children await insertion
    int32_t stalled;      // a fill needs more chunks than were queued: kernels
                          // wait (do nothing) until the host has finished it
    int32_t packed;       // the chunk's acceptance completed the fill and packed
                          // its offsets: its insert kernel copies the population
    int32_t chunk_first;  // slots filled before the chunk (Nn at its start)
    int32_t slot[EBIC_MAX_ARCHIVE + 2];   // the list in rank order: slot ids
    int32_t a_len[EBIC_MAX_ARCHIVE + 2];  // per slot id: length, rows, score
    int32_t a_n[EBIC_MAX_ARCHIVE + 2];
    double a_score[EBIC_MAX_ARCHIVE + 2];
};

// Device buffers, passed by value to every kernel.
struct DlBufs {
    uint16_t *pop[2];       // populations, [P][kmax] fixed stride
    int32_t *plen[2];       // their lengths
    int32_t *csr_off;       // the scored population packed for the evaluator
    uint16_t *csr_cols;
    double *fit;            // evaluator outputs
    int32_t *cnt;
    uint64_t *sup;          // [P][W]
    double *keys;           // tournament keys
    int32_t *use[2];        // column use counts of a population (by its parity), [C]
    uint16_t *aslot_cols;   // top-rank list members by slot, [K+2][kmax]
    uint64_t *aslot_sup;    // [K+2][W]
    int32_t *arch_off;      // the list packed for the evaluator, in rank order
    uint16_t *arch_cols;
    uint64_t *arch_sup;     // [K][W]
    uint8_t *span;          // [kSpanMax] draws taken by an attempt starting at each offset
    int32_t *att_off;       // [kChunkMax] the chunk's attempts: start offsets
    uint16_t *child;        // [kChunkMax][kmax] children (as drawn, not canonical)
    int32_t *clen;          // [kChunkMax] 0: no weighted operator applied
    uint32_t *cflag;        // [kChunkMax] kValid, kRev, kInSet, kAccept
    uint64_t *chash;        // [kChunkMax] hash of the canonical child
    int32_t *cslot;         // [kChunkMax] an accepted child's slot in the next population
    int32_t *carena;        // [kChunkMax] and its tabu arena entry
    uint64_t *thash;        // tabu table: hash (0 = empty slot)
    int32_t *tref;          // tabu table: arena entry
    uint16_t *tarena;       // [tabu_cap][kmax] canonical series
    int32_t *tlen;          // [tabu_cap]
    double *trace;          // [G][4]
    DlState *st;
};

constexpr uint32_t kValid = 1, kRev = 2, kInSet = 4, kAccept = 8, kDup = 16;

// ---- SplitMix64 at any position, bounded draws ----

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Draws from the stream whose state is s, starting p draws in.
struct Draws {
    uint64_t s, p;
    // Uniform in [0, n): draws below 2^64 mod n are rejected (the accepted
    // range is a whole number of periods of n).
    __device__ uint32_t below(uint32_t n) {
        const uint64_t low = (0 - (uint64_t)n) % n;
        for (;;) {
            const uint64_t x = sm_mix(s + (p + 1) * kGamma);
            p++;
            if (x >= low) return (uint32_t)(x % n);
        }
    }
};

// One mutation attempt's draws (step 5): tournament, operator among those
// that apply to the parent, weighted; then the operator's own draws.
struct Attempt {
    int32_t parent, k, op;  // op -1: no weighted operator applies
    int32_t pos, pick;      // position; index of the unused column
    int32_t a, b;           // swap positions, or crossover cuts
    int32_t parent2, k2;
};

enum { OP_INSERT, OP_DELETE, OP_SUBST, OP_SWAP, OP_CROSS };

__device__ int tournament_at(Draws &d, const double *keys, int Pn, int T) {
    int best = -1;
    double bk = 0.0;
    for (int t = 0; t < T; t++) {
        const int i = (int)d.below((uint32_t)Pn);
        const double ki = keys[i];
        if (best < 0 || ki > bk || (ki == bk && i < best)) {
            best = i;
            bk = ki;
        }
    }
    return best;
}

__device__ void draw_attempt(Draws &d, const DlParams &q, const double *keys, const int32_t *plen,
                             int Pn, Attempt &at) {
    at.parent = tournament_at(d, keys, Pn, q.T);
    const int k = plen[at.parent];
    at.k = k;
    const bool ap[5] = {k < q.kmax && k < q.C, k > q.kmin, k < q.C, true, true};
    int total = 0;
    for (int o = 0; o < 5; o++) total += ap[o] ? q.opw[o] : 0;
    if (total == 0) {
        at.op = -1;
        return;
    }
    int x = (int)d.below((uint32_t)total);
    int op = 0;
    for (;; op++) {
        const int w = ap[op] ? q.opw[op] : 0;
        if (x < w) break;
        x -= w;
    }
    at.op = op;
    switch (op) {
        case OP_INSERT:
            at.pos = (int)d.below((uint32_t)(k + 1));
            at.pick = (int)d.below((uint32_t)(q.C - k));
            break;
        case OP_DELETE:
            at.pos = (int)d.below((uint32_t)k);
            break;
        case OP_SUBST:
            at.pos = (int)d.below((uint32_t)k);
            at.pick = (int)d.below((uint32_t)(q.C - k));
            break;
        case OP_SWAP:
            at.a = (int)d.below((uint32_t)k);
            at.b = (int)d.below((uint32_t)(k - 1));
            if (at.b >= at.a) at.b++;
            break;
        default:
            at.parent2 = tournament_at(d, keys, Pn, q.T);
            at.k2 = plen[at.parent2];
            at.a = 1 + (int)d.below((uint32_t)(k - 1));
            at.b = 1 + (int)d.below((uint32_t)(at.k2 - 1));
    }
}

// ---- series helpers ----

// Element j of a series in its canonical orientation.
__device__ __forceinline__ int canon_at(const uint16_t *s, int len, bool rev, int j) {
    return rev ? s[len - 1 - j] : s[j];
}

// Hash of a canonical series (placement only: membership compares columns).
// XOR over positions, so a wave can take it in parallel.
__device__ __forceinline__ uint64_t col_hash(int c, int j, int len) {
    return sm_mix(((uint64_t)(uint32_t)c << 32 | (uint32_t)j) * kGamma + (uint64_t)len);
}
__device__ uint64_t series_hash_seq(const uint16_t *s, int len, bool rev) {
    uint64_t h = sm_mix((uint64_t)len + 0x632BE59BD9B4E019ULL);
    for (int j = 0; j < len; j++) h ^= col_hash(canon_at(s, len, rev, j), j, len);
    return h | 1;
}

// Whether the series' reverse is smaller (the canonical form with negative
// trends on), sequentially.
__device__ bool reverse_smaller_seq(const uint16_t *s, int len) {
    for (int i = 0; i < len; i++)
        if (s[len - 1 - i] != s[i]) return s[len - 1 - i] < s[i];
    return false;
}

// Lexicographic order of two series as drawn (a proper prefix first).
__device__ int series_cmp_seq(const uint16_t *a, int la, const uint16_t *b, int lb) {
    const int m = la < lb ? la : lb;
    for (int i = 0; i < m; i++)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return (la > lb) - (la < lb);
}

// Top-rank order: larger score first, then the smaller series.
__device__ bool ranks_above_dev(double sa, const uint16_t *a, int la, double sb, const uint16_t *b,
                                int lb) {
    if (sa != sb) return sa > sb;
    return series_cmp_seq(a, la, b, lb) < 0;
}

// ---- block-wide helpers (blockDim.x a multiple of 64, at most 1024) ----

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum over the block; *total gets the sum. s_tmp holds 33 ints.
__device__ int block_excl_scan(int v, int *s_tmp, int *total) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int inc = wave_incl_scan(v);
    if (lane == kWave - 1) s_tmp[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const int x = lane < nw ? s_tmp[lane] : 0;
        const int y = wave_incl_scan(x);
        if (lane < nw) s_tmp[lane] = y - x;
        if (lane == kWave - 1) s_tmp[32] = y;
    }
    __syncthreads();
    const int r = s_tmp[wave] + inc - v;
    *total = s_tmp[32];
    __syncthreads();
    return r;
}

// Largest value of v over the block's threads before this one (-1 if none).
__device__ int block_excl_max(int v, int *s_tmp) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc = inc > t ? inc : t;
    }
    const int prev_in_wave = __shfl_up(inc, 1, kWave);
    if (lane == kWave - 1) s_tmp[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int x = lane < nw ? s_tmp[lane] : -1;
        int y = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(y, o, kWave);
            if (lane >= o) y = y > t ? y : t;
        }
        const int before = __shfl_up(y, 1, kWave);
        if (lane < nw) s_tmp[lane] = lane == 0 ? -1 : before;
    }
    __syncthreads();
    int r = s_tmp[wave];
    if (lane > 0) r = r > prev_in_wave ? r : prev_in_wave;
    __syncthreads();
    return r;
}

__device__ int block_min(int v, int *s_tmp) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int t = __shfl_xor(v, o, kWave);
        v = v < t ? v : t;
    }
    if (lane == 0) s_tmp[wave] = v;
    __syncthreads();
    int r = s_tmp[0];
    for (int w = 1; w < nw; w++) r = r < s_tmp[w] ? r : s_tmp[w];
    __syncthreads();
    return r;
}

// Ascending bitonic sort of n (a power of two) 128-bit keys (hi, lo) in LDS.
__device__ void bitonic_sort(uint64_t *hi, uint64_t *lo, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t ah = hi[i], al = lo[i], bh = hi[j], bl = lo[j];
                const bool gt = ah > bh || (ah == bh && al > bl);
                if (gt == up) {
                    hi[i] = bh;
                    lo[i] = bl;
                    hi[j] = ah;
                    lo[j] = al;
                }
            }
            __syncthreads();
        }
    }
}


// ---- kernels ----

// Whether the fill has a chunk of attempts to run now.
__device__ __forceinline__ bool fill_active(const DlState *st) {
    return !st->over && !st->stalled && st->need_more;
}

// Steps 3 and 7 (top-rank list) for the population just scored, the trace
// entry, the stop checks and step 4 (elitism); finally the list packed for
// the next evaluation. One workgroup.
//
// Candidates (a positive size score, not on the list already in canonical
// form) are sorted by (score descending, series ascending): a bitonic sort
// on (score bits, first three columns, index), runs that tie on both then
// ordered by their whole series. They are then taken in that order as on
// the host, a batch at a time: each wave compares one candidate of the
// batch with every member of the list as it stands (shared columns from the
// candidate's column bitmap, shared rows when the columns allow a clash),
// and one thread applies the admission rule to the batch's candidates in
// order. A rejected candidate leaves the list as it was, so the next
// candidate's comparisons still hold; after an admission the next batch
// starts from the following candidate against the new list.
constexpr int kListWaves = kBlock / kWave;
constexpr int kListSlots = EBIC_MAX_ARCHIVE + 2;

// Dynamic LDS of the list kernel: the sort keys, later the candidate order
// and one column bitmap per wave; then a byte per individual (its tier).
__host__ __device__ inline size_t list_lds_shared(int Ppad, int C) {
    const size_t sort = (size_t)Ppad * 16;
    const size_t loop = (size_t)Ppad * 4 + (size_t)kListWaves * ((C + 31) / 32) * 4;
    return ((sort > loop ? sort : loop) + 7) & ~(size_t)7;
}
size_t list_lds_bytes(int Ppad, int C) { return list_lds_shared(Ppad, C) + (size_t)Ppad; }

__device__ inline uint32_t pow2_dev(uint32_t x) {
    uint32_t v = 1;
    while (v < x) v <<= 1;
    return v;
}

__global__ void __launch_bounds__(kBlock) dl_list_kernel(DlParams q, DlBufs B, int cur, int Pn,
                                                         int Ppad) {
    extern __shared__ uint64_t s_dyn[];
    uint64_t *s_k1 = s_dyn, *s_k2 = s_dyn + Ppad;
    int32_t *s_order = reinterpret_cast<int32_t *>(s_dyn);
    const int BW = (q.C + 31) / 32;
    uint32_t *s_wbits = reinterpret_cast<uint32_t *>(s_dyn) + Ppad;
    uint8_t *s_tier = reinterpret_cast<uint8_t *>(s_dyn) + list_lds_shared(Ppad, q.C);
    __shared__ int32_t s_list[kListSlots], s_arev[kListSlots];
    __shared__ int32_t s_alen[kListSlots], s_an[kListSlots];
    __shared__ double s_asc[kListSlots];
    __shared__ int8_t s_ov[kListWaves][kListSlots], s_abv[kListWaves][kListSlots];
    __shared__ int32_t s_nA, s_nc, s_fix, s_next, s_done, s_new, s_newi, s_stop;
    (void)s_next;
    DlState *st = B.st;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % kWave, wave = tid / kWave;
    const int kmax = q.kmax, W = q.W;
    const uint16_t *pop = B.pop[cur];
    const int32_t *plen = B.plen[cur];
    auto score_of = [&](int i) {
        const int n = B.cnt[i], k = plen[i];
        return (n >= q.min_rows && k >= q.k_score_min) ? ldexp((double)n, k) : 0.0;
    };
    auto mcols = [&](int sl) { return B.aslot_cols + (size_t)sl * kmax; };
    if (st->over || st->stalled) return;
    if (tid == 0) {
        s_nA = st->nA;
        s_nc = 0;
        s_fix = 0;
    }
    for (int j = tid; j < kListSlots; j += nt) {
        s_list[j] = st->slot[j];
        s_alen[j] = st->a_len[j];
        s_an[j] = st->a_n[j];
        s_asc[j] = st->a_score[j];
    }
    __syncthreads();
    int nA = s_nA;
    for (int j = tid; j < nA; j += nt) {
        const int sl = s_list[j];
        s_arev[j] = q.neg && reverse_smaller_seq(mcols(sl), s_alen[sl]);
    }
    __syncthreads();
    // Candidates in two tiers: while the list is full only those ranking
    // above its last member can enter (tier 1); the rest (tier 2) are needed
    // only if the list falls short of full after tier 1 (an admission can
    // remove several members). Each tier is sorted when it is reached.
    const int nA0 = nA;
    // every length and count of this thread's candidates loaded first, all
    // in flight together
    constexpr int kPer = kDlMaxP / kBlock;
    int klen[kPer], kcnt[kPer];
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        const int i = tid + r * nt;
        klen[r] = i < Pn ? plen[i] : 0;
        kcnt[r] = i < Pn ? B.cnt[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        const int i = tid + r * nt;
        if (i >= Ppad) break;
        int t = 0;
        if (i < Pn) {
            const int k = klen[r];
            const uint16_t *si = pop + (size_t)i * kmax;
            const double sc = (kcnt[r] >= q.min_rows && k >= q.k_score_min)
                                  ? ldexp((double)kcnt[r], k) : 0.0;
            bool cand = sc > 0.0;
            if (cand) {
                // a series already listed (or its reverse) has the member's
                // length and, being the same rows, its score: only such
                // members are compared column by column
                int rv = -1;  // the series' canonical direction, found when first needed
                for (int j = 0; j < nA && cand; j++) {
                    const int sl = s_list[j];
                    if (s_alen[sl] != k || s_asc[sl] != sc) continue;
                    if (rv < 0) rv = q.neg && reverse_smaller_seq(si, k);
                    const uint16_t *ms = mcols(sl);
                    // sixteen columns at a time, their loads in flight together
                    // (the population's copies of the members match to the
                    // end); positions past the series repeat its last one
                    bool same = true;
                    const bool mrev = s_arev[j] != 0;
                    for (int e0 = 0; e0 < k && same; e0 += 16) {
                        int ca[16], cb[16];
#pragma unroll
                        for (int u = 0; u < 16; u++) {
                            const int e = e0 + u < k ? e0 + u : k - 1;
                            ca[u] = canon_at(si, k, rv != 0, e);
                            cb[u] = canon_at(ms, k, mrev, e);
                        }
#pragma unroll
                        for (int u = 0; u < 16; u++) same &= ca[u] == cb[u];
                    }
                    if (same) cand = false;
                }
            }
            if (cand) {
                t = 1;
                if (nA0 == q.K) {
                    const int sl = s_list[nA0 - 1];
                    if (!ranks_above_dev(sc, si, k, s_asc[sl], mcols(sl), s_alen[sl])) t = 2;
                }
            }
        }
        s_tier[i] = (uint8_t)t;
    }
    __syncthreads();
    uint32_t *bits = s_wbits + (size_t)wave * BW;
    // one wave: its candidate against the member in slot sl
    auto compare = [&](int i, int sl) {
        const int k = plen[i], n = B.cnt[i], lj = s_alen[sl];
        const double sc = score_of(i);
        const uint16_t *si = pop + (size_t)i * kmax, *ms = mcols(sl);
        const long long bound = (long long)q.theta * n * k;
        int g = 0;
        for (int e = lane; e < lj; e += kWave) {
            const int c = ms[e];
            g += (bits[c >> 5] >> (c & 31)) & 1;
        }
        g = wave_sum(g);
        const int nj = s_an[sl];
        int ov = 0;
        // h <= min(n, n_j): when even that cannot reach the bound the rows
        // need no counting
        if (1000LL * (n < nj ? n : nj) * g > bound) {
            const uint64_t *supi = B.sup + (size_t)i * W, *supj = B.aslot_sup + (size_t)sl * W;
            int h = 0;
            for (int w = lane; w < W; w += kWave) h += __popcll(supi[w] & supj[w]);
            h = wave_sum(h);
            ov = 1000LL * h * g > bound;
        }
        if (lane == 0) {
            s_ov[wave][sl] = (int8_t)ov;
            s_abv[wave][sl] = (int8_t)(ov ? ranks_above_dev(sc, si, k, s_asc[sl], ms, lj) : 1);
        }
    };
    if (tid == 0) s_done = 0;
    for (int tier = 1; tier <= 2; tier++) {
        if (tid == 0) {
            s_nc = 0;
            // every tier-2 candidate ranks below the list's last member while
            // it is full: nothing more can enter
            if (tier == 2 && s_nA == q.K) s_done = 1;
        }
        __syncthreads();
        if (s_done) break;
        for (int i = tid; i < Pn; i += nt) {
            if (s_tier[i] != tier) continue;
            const int k = plen[i];
            const uint16_t *si = pop + (size_t)i * kmax;
            uint64_t pre = 0;
            for (int e = 0; e < 3; e++) pre = pre << 17 | (e < k ? (uint64_t)si[e] + 1 : 0);
            const int x = atomicAdd(&s_nc, 1);
            s_k1[x] = ~(uint64_t)__double_as_longlong(score_of(i));
            s_k2[x] = pre << 13 | (uint64_t)i;
        }
        __syncthreads();
        const int nc = s_nc;
        if (nc == 0) continue;
        const int Pt = (int)pow2_dev((uint32_t)(nc < 2 ? 2 : nc));
        for (int x = nc + tid; x < Pt; x += nt) s_k1[x] = s_k2[x] = ~0ull;
        if (tid == 0) s_fix = 0;
        __syncthreads();
        bitonic_sort(s_k1, s_k2, Pt);
        for (int x = tid; x + 1 < nc; x += nt)
            if (s_k1[x] == s_k1[x + 1] && (s_k2[x] >> 13) == (s_k2[x + 1] >> 13)) s_fix = 1;
        __syncthreads();
        if (s_fix) {
            // runs equal in score and first three columns: by the whole series,
            // each run by the thread that finds its start
            auto same_key = [&](int x, int y) {
                return s_k1[x] == s_k1[y] && (s_k2[x] >> 13) == (s_k2[y] >> 13);
            };
            for (int a = tid; a + 1 < nc; a += nt) {
                if ((a > 0 && same_key(a - 1, a)) || !same_key(a, a + 1)) continue;
                int b = a + 1;
                while (b < nc && same_key(a, b)) b++;
                for (int x = a + 1; x < b; x++) {
                    const uint64_t kx = s_k2[x];
                    const int ix = (int)(kx & 0x1FFF);
                    int y = x - 1;
                    while (y >= a) {
                        const int iy = (int)(s_k2[y] & 0x1FFF);
                        if (series_cmp_seq(pop + (size_t)ix * kmax, plen[ix],
                                           pop + (size_t)iy * kmax, plen[iy]) >= 0)
                            break;
                        s_k2[y + 1] = s_k2[y];
                        y--;
                    }
                    s_k2[y + 1] = kx;
                }
            }
        }
        __syncthreads();
        // the order, then the waves' column bitmaps, in the sort's LDS
        {
            constexpr int kMaxPer = kDlMaxP / kBlock;
            int32_t mine[kMaxPer];
#pragma unroll
            for (int r = 0; r < kMaxPer; r++) {
                const int x = tid + r * nt;
                mine[r] = x < nc ? (int32_t)(s_k2[x] & 0x1FFF) : 0;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kMaxPer; r++) {
                const int x = tid + r * nt;
                if (x < nc) s_order[x] = mine[r];
            }
            for (int w = tid; w < kListWaves * BW; w += nt) s_wbits[w] = 0;
            __syncthreads();
        }
        for (int ci = 0; ci < nc; ci += kListWaves) {
            // each wave: one candidate of the batch against the list
            nA = s_nA;
            const int cw = ci + wave, ic = cw < nc ? s_order[cw] : -1;
            if (ic >= 0) {
                const uint16_t *si = pop + (size_t)ic * kmax;
                for (int e = lane; e < plen[ic]; e += kWave) {
                    const int c = si[e];
                    atomicOr(&bits[c >> 5], 1u << (c & 31));
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (int j = 0; j < nA; j++) compare(ic, s_list[j]);
            }
            __syncthreads();
            int from = 0;
            for (;;) {
                if (tid == 0) {
                    int ns = -1, ni = -1, w = from;
                    for (; w < kListWaves; w++) {
                        const int c = ci + w;
                        if (c >= nc) break;
                        const int i = s_order[c], k = plen[i];
                        const double sc = score_of(i);
                        const uint16_t *si = pop + (size_t)i * kmax;
                        if (nA == q.K) {
                            const int sl = s_list[nA - 1];
                            if (!ranks_above_dev(sc, si, k, s_asc[sl], mcols(sl), s_alen[sl])) {
                                s_done = 1;
                                break;
                            }
                        }
                        bool any = false, beats = true;
                        for (int j = 0; j < nA; j++) {
                            const int sl = s_list[j];
                            if (s_ov[w][sl]) {
                                any = true;
                                if (!s_abv[w][sl]) beats = false;
                            }
                        }
                        if (any && !beats) continue;  // rejected: the list stays as it is
                        // admitted: the members it overlaps leave (it outranks them)
                        int m = 0;
                        for (int j = 0; j < nA; j++)
                            if (!s_ov[w][s_list[j]]) s_list[m++] = s_list[j];
                        nA = m;
                        for (ns = 0;; ns++) {  // a free slot (at most K are in use)
                            bool taken = false;
                            for (int j = 0; j < nA; j++) taken |= s_list[j] == ns;
                            if (!taken) break;
                        }
                        int pos = 0;
                        while (pos < nA) {
                            const int sl = s_list[pos];
                            if (!ranks_above_dev(s_asc[sl], mcols(sl), s_alen[sl], sc, si, k)) break;
                            pos++;
                        }
                        for (int j = nA; j > pos; j--) s_list[j] = s_list[j - 1];
                        s_list[pos] = ns;
                        nA++;
                        s_alen[ns] = k;
                        s_an[ns] = B.cnt[i];
                        s_asc[ns] = sc;
                        if (nA > q.K) nA--;  // the last one leaves
                        ni = i;
                        w++;
                        break;
                    }
                    s_nA = nA;
                    s_new = ns;
                    s_newi = ni;
                    s_next = w;
                }
                __syncthreads();
                const int ns = s_new;
                if (ns < 0) break;
                {
                    const int i = s_newi, k = plen[i];
                    for (int e = tid; e < k; e += nt)
                        B.aslot_cols[(size_t)ns * kmax + e] = pop[(size_t)i * kmax + e];
                    for (int w = tid; w < W; w += nt)
                        B.aslot_sup[(size_t)ns * W + w] = B.sup[(size_t)i * W + w];
                }
                __syncthreads();
                from = s_next;
                if (s_done) break;
                // the rest of the batch against the new member only
                if (ic >= 0 && wave >= from) compare(ic, ns);
                __syncthreads();
                nA = s_nA;
            }
            if (ic >= 0) {
                const uint16_t *si = pop + (size_t)ic * kmax;
                for (int e = lane; e < plen[ic]; e += kWave) {
                    const int c = si[e];
                    atomicAnd(&bits[c >> 5], ~(1u << (c & 31)));
                }
            }
            __syncthreads();
            if (s_done) break;
        }
        __syncthreads();
    }
    nA = s_nA;
    if (tid == 0) {
        st->nA = nA;
        for (int j = 0; j < kListSlots; j++) {
            st->slot[j] = j < nA ? s_list[j] : -1;
            st->a_len[j] = s_alen[j];
            st->a_n[j] = s_an[j];
            st->a_score[j] = s_asc[j];
        }
        const int g = st->g;
        double *tr = B.trace + (size_t)g * 4;
        tr[0] = (double)Pn;
        tr[1] = (double)nA;
        tr[2] = nA ? s_asc[s_list[0]] : 0.0;
        tr[3] = (double)st->hits;
        st->evaluations += Pn;
        st->g = g + 1;
        if (!st->stop && g + 1 == q.G) st->stop = EBIC_STOP_GENERATIONS;
        if (st->stop) st->over = 1;
        int at = 0;
        for (int j = 0; j < nA; j++) {
            B.arch_off[j] = at;
            at += s_alen[s_list[j]];
        }
        B.arch_off[nA] = at;
        st->arch_len = at;
        s_stop = st->stop;
    }
    __syncthreads();
    // the list packed for the evaluator, in rank order: a wave per member
    for (int j = wave; j < nA; j += kListWaves) {
        const int sl = s_list[j], lj = s_alen[sl], at = B.arch_off[j];
        for (int e = lane; e < lj; e += kWave)
            B.arch_cols[at + e] = B.aslot_cols[(size_t)sl * kmax + e];
        for (int w = lane; w < W; w += kWave)
            B.arch_sup[(size_t)j * W + w] = B.aslot_sup[(size_t)sl * W + w];
    }
    if (s_stop) return;
    // step 4: the list's first members (at most half the population) start
    // the next one
    const int nxt = cur ^ 1, ne = nA < q.P / 2 ? nA : q.P / 2;
    for (int j = wave; j < ne; j += kListWaves) {
        const int sl = s_list[j], lj = s_alen[sl];
        for (int e = lane; e < lj; e += kWave)
            B.pop[nxt][(size_t)j * kmax + e] = B.aslot_cols[(size_t)sl * kmax + e];
        if (lane == 0) B.plen[nxt][j] = lj;
    }
    if (tid == 0) {
        st->Nn = ne;
        st->att = 0;
        st->need_more = ne < q.P;
    }
}

// Step 5, tournament keys: each fitness halved once per column of the
// individual that more individuals hold than ceil(sum k / C). The column use
// counts (into the count array of the population's parity) are taken when
// the population is copied for the evaluator (dl_copy_kernel); this kernel,
// a wave per individual, makes the keys and clears the counts of the other
// parity for the next population.
__global__ void __launch_bounds__(256) dl_keys_kernel(DlParams q, DlBufs B, int cur, int Pn) {
    if (B.st->over || B.st->stalled) return;
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = gt; c < q.C; c += gridDim.x * blockDim.x) B.use[cur ^ 1][c] = 0;
    const int i = gt / kWave, lane = threadIdx.x % kWave;
    if (i >= Pn) return;
    const long long ksum = B.csr_off[Pn];  // columns of the population
    const long long share = (ksum + q.C - 1) / q.C;
    const int k = B.plen[cur][i];
    const uint16_t *s = B.pop[cur] + (size_t)i * q.kmax;
    int over = 0;
    for (int e = lane; e < k; e += kWave) over += B.use[cur][s[e]] > share;
    over = wave_sum(over);
    if (lane == 0) B.keys[i] = ldexp(B.fit[i], -over);
}

// The number of draws an attempt starting at each offset of the span would
// take (capped at 255).
__global__ void __launch_bounds__(256) dl_span_kernel(DlParams q, DlBufs B, int cur, int Pn,
                                                      int S) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= S || !fill_active(B.st)) return;
    Draws d{B.st->rng, (uint64_t)o};
    Attempt at;
    draw_attempt(d, q, B.keys, B.plen[cur], Pn, at);
    const uint64_t c = d.p - (uint64_t)o;
    B.span[o] = (uint8_t)(c > 255 ? 255 : c);
}

// The chain of attempts from the span's start: each segment of kSeg offsets
// is walked from every offset the chain can enter it at (an attempt takes
// at most span_e - 1 draws on this path), the segments are linked in order,
// and each segment then writes its attempts' offsets. Any attempt longer
// than that (draws rejected by a bounded draw) sends the chunk down the
// sequential walk, which draws every attempt. One workgroup; att_end[i] is
// where attempt i ends (att_off + its draws).
__global__ void __launch_bounds__(kBlock) dl_chain_kernel(DlParams q, DlBufs B, int32_t *att_end,
                                                          int cur, int Pn, int S, int A_target) {
    extern __shared__ uint64_t s_dyn[];
    uint8_t *s_c = reinterpret_cast<uint8_t *>(s_dyn);
    const int E = q.span_e, nseg = (S + kSeg - 1) / kSeg;
    // (each array starts on an 8-byte boundary)
    uint16_t *s_cnt = reinterpret_cast<uint16_t *>(s_c + ((S + 7) & ~7));
    uint8_t *s_exit = reinterpret_cast<uint8_t *>(s_cnt) + (((size_t)nseg * E * 2 + 7) & ~(size_t)7);
    int32_t *s_entry = reinterpret_cast<int32_t *>(s_exit + (((size_t)nseg * E + 7) & ~(size_t)7));
    int32_t *s_base = s_entry + nseg;
    __shared__ int s_bad, s_total;
    constexpr int kGroup = 16, kMaxGroups = (kSpanMax / kSeg + 1 + kGroup - 1) / kGroup;
    __shared__ uint16_t s_gcnt[kMaxGroups * (2 * kDlMaxT + 12)];
    __shared__ uint8_t s_gexit[kMaxGroups * (2 * kDlMaxT + 12)];
    __shared__ int32_t s_gentry[kMaxGroups], s_gbase[kMaxGroups];
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) B.st->pending = 0;  // nothing of an earlier chunk is inserted again
    if (!fill_active(B.st)) return;
    if (tid == 0) {
        s_bad = 0;
        s_total = 0;
    }
    __syncthreads();
    // the draw counts into LDS, 16 bytes per load (a byte per load would
    // take one round trip per 1,024 offsets)
    {
        const uint4 *sp4 = reinterpret_cast<const uint4 *>(B.span);
        int bad = 0;
        for (int v = tid; v * 16 < S; v += nt) {
            const uint4 x = sp4[v];
            const uint32_t wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int b = 0; b < 16; b++) {
                const int o = v * 16 + b;
                const int c = (int)((wd[b >> 2] >> ((b & 3) * 8)) & 0xFFu);
                if (o < S) {
                    s_c[o] = (uint8_t)c;
                    bad |= c >= E;
                }
            }
        }
        if (bad) s_bad = 1;
    }
    __syncthreads();
    if (!s_bad) {
        for (int pr = tid; pr < nseg * E; pr += nt) {
            const int sg = pr / E, e = pr % E;
            const int end = (sg + 1) * kSeg < S ? (sg + 1) * kSeg : S;
            int pos = sg * kSeg + e, cnt = 0;
            while (pos < end) {
                cnt++;
                pos += s_c[pos];
            }
            s_cnt[pr] = (uint16_t)cnt;
            const int ex = pos - (sg + 1) * kSeg;
            s_exit[pr] = (uint8_t)(ex > 0 ? ex : 0);
        }
        __syncthreads();
        // link the segments: groups of kGroup segments composed from every
        // entry offset in parallel, the groups linked in order, then each
        // group's segments given their entries and first attempt indices
        const int ngroup = (nseg + kGroup - 1) / kGroup;
        for (int pr = tid; pr < ngroup * E; pr += nt) {
            const int gr = pr / E, s0 = gr * kGroup;
            const int s1 = s0 + kGroup < nseg ? s0 + kGroup : nseg;
            int e = pr % E, cnt = 0;
            for (int sg = s0; sg < s1; sg++) {
                cnt += s_cnt[sg * E + e];
                e = s_exit[sg * E + e];  // the next segment's entry offset (below E)
            }
            s_gcnt[pr] = (uint16_t)cnt;
            s_gexit[pr] = (uint8_t)e;
        }
        __syncthreads();
        if (tid == 0) {
            int e = 0, idx = 0;
            for (int gr = 0; gr < ngroup; gr++) {
                s_gentry[gr] = e;
                s_gbase[gr] = idx;
                idx += s_gcnt[gr * E + e];
                e = s_gexit[gr * E + e];
            }
            s_total = idx;
        }
        __syncthreads();
        for (int gr = tid; gr < ngroup; gr += nt) {
            const int s0 = gr * kGroup, s1 = s0 + kGroup < nseg ? s0 + kGroup : nseg;
            int e = s_gentry[gr], idx = s_gbase[gr];
            for (int sg = s0; sg < s1; sg++) {
                s_entry[sg] = sg * kSeg + e;
                s_base[sg] = idx;
                idx += s_cnt[sg * E + e];
                e = s_exit[sg * E + e];
            }
        }
        __syncthreads();
    }
    if (!s_bad) {
        for (int sg = tid; sg < nseg; sg += nt) {
            const int end = (sg + 1) * kSeg < S ? (sg + 1) * kSeg : S;
            int pos = s_entry[sg], i = s_base[sg];
            while (pos < end && i < A_target) {
                B.att_off[i] = pos;
                att_end[i] = pos + s_c[pos];
                i++;
                pos += s_c[pos];
            }
        }
        if (tid == 0) B.st->chunk_n = s_total < A_target ? s_total : A_target;
    } else if (tid == 0) {
        // sequential: draw each attempt to learn where the next one starts
        uint64_t pos = 0;
        int i = 0;
        while (i < A_target) {
            Draws d{B.st->rng, pos};
            Attempt at;
            draw_attempt(d, q, B.keys, B.plen[cur], Pn, at);
            B.att_off[i] = (int32_t)pos;
            att_end[i] = (int32_t)d.p;
            pos = d.p;
            i++;
        }
        B.st->chunk_n = i;
        B.st->slow += 1;
    }
}

// The unused-column draw: the pick-th column (from 0) not in the parent, in
// ascending order. `bits` is the wave's all-zero column bitmap in LDS (left
// all-zero again). Wave-uniform result.
__device__ int unused_col_wave(uint32_t *bits, const uint16_t *par, int k, int C, int pick) {
    const int lane = threadIdx.x % kWave;
    for (int e = lane; e < k; e += kWave) {
        const int c = par[e];
        atomicOr(&bits[c >> 5], 1u << (c & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int nw = (C + 31) / 32, per = (nw + kWave - 1) / kWave;
    const int w0 = lane * per, w1 = w0 + per < nw ? w0 + per : nw;
    auto free_mask = [&](int w) {
        const uint32_t valid = (w == nw - 1 && (C & 31)) ? ((1u << (C & 31)) - 1u) : ~0u;
        return ~bits[w] & valid;
    };
    int zeros = 0;
    for (int w = w0; w < w1; w++) zeros += __popc(free_mask(w));
    const int before = wave_incl_scan(zeros) - zeros;
    int col = -1;
    if (pick >= before && pick < before + zeros) {
        int r = pick - before;
        for (int w = w0; w < w1; w++) {
            uint32_t z = free_mask(w);
            const int cz = __popc(z);
            if (r < cz) {
                while (r-- > 0) z &= z - 1;
                col = w * 32 + __ffs(z) - 1;
                break;
            }
            r -= cz;
        }
    }
    const uint64_t who = __ballot(col >= 0);
    const int src = __ffsll((unsigned long long)who) - 1;
    col = __shfl(col, src < 0 ? 0 : src, kWave);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < k; e += kWave) {
        const int c = par[e];
        atomicAnd(&bits[c >> 5], ~(1u << (c & 31)));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return col;
}

// Every attempt of the chunk at once, a wave each: its draws, its child
// (built in LDS, then stored as drawn), the child's canonical orientation
// and hash, and whether the tabu set already holds it.
__global__ void __launch_bounds__(kChildWaves *kWave) dl_child_kernel(DlParams q, DlBufs B,
                                                                     int cur, int Pn) {
    __shared__ uint32_t s_bits[kChildWaves][kMaxCols / 32];
    __shared__ uint16_t s_child[kChildWaves][EBIC_MAX_K];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int i = blockIdx.x * kChildWaves + wave;
    const int A = B.st->chunk_n;
    if (i >= A || !fill_active(B.st)) return;  // whole wave
    uint32_t *bits = s_bits[wave];
    uint16_t *ch = s_child[wave];
    const int kmax = q.kmax;
    for (int w = lane; w < (q.C + 31) / 32; w += kWave) bits[w] = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    Draws d{B.st->rng, (uint64_t)B.att_off[i]};
    Attempt at;
    draw_attempt(d, q, B.keys, B.plen[cur], Pn, at);
    const uint16_t *par = B.pop[cur] + (size_t)at.parent * kmax;
    const int k = at.k;
    int len = 0;
    switch (at.op) {
        case OP_INSERT: {
            const int u = unused_col_wave(bits, par, k, q.C, at.pick);
            for (int j = lane; j <= k; j += kWave)
                ch[j] = (uint16_t)(j < at.pos ? par[j] : (j == at.pos ? u : par[j - 1]));
            len = k + 1;
            break;
        }
        case OP_DELETE:
            for (int j = lane; j < k - 1; j += kWave) ch[j] = j < at.pos ? par[j] : par[j + 1];
            len = k - 1;
            break;
        case OP_SUBST: {
            const int u = unused_col_wave(bits, par, k, q.C, at.pick);
            for (int j = lane; j < k; j += kWave) ch[j] = (uint16_t)(j == at.pos ? u : par[j]);
            len = k;
            break;
        }
        case OP_SWAP:
            for (int j = lane; j < k; j += kWave)
                ch[j] = j == at.a ? par[at.b] : (j == at.b ? par[at.a] : par[j]);
            len = k;
            break;
        case OP_CROSS: {
            // the first parent's first a columns, then the columns of the
            // second parent from b on that they lack
            const uint16_t *par2 = B.pop[cur] + (size_t)at.parent2 * kmax;
            for (int e = lane; e < at.a; e += kWave) {
                const int c = par[e];
                ch[e] = (uint16_t)c;
                atomicOr(&bits[c >> 5], 1u << (c & 31));
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            len = at.a;
            for (int t0 = at.b; t0 < at.k2; t0 += kWave) {
                const int t = t0 + lane;
                const int c = t < at.k2 ? par2[t] : 0;
                const bool keep = t < at.k2 && !((bits[c >> 5] >> (c & 31)) & 1u);
                const uint64_t m = __ballot(keep);
                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                if (keep && len + rank < kmax) ch[len + rank] = (uint16_t)c;
                len += __popcll(m);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < at.a; e += kWave) {
                const int c = par[e];
                atomicAnd(&bits[c >> 5], ~(1u << (c & 31)));
            }
            break;
        }
        default:
            len = 0;  // no weighted operator applies: a failed attempt
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const bool valid = at.op >= 0 && len >= q.kmin && len <= kmax;
    uint32_t flag = 0;
    uint64_t h = 0;
    if (valid) {
        flag |= kValid;
        // canonical orientation: the reverse when it is smaller (negative trends)
        bool rev = false;
        if (q.neg) {
            for (int i0 = 0; i0 < len / 2; i0 += kWave) {
                const int x = i0 + lane;
                const uint64_t m = __ballot(x < len / 2 && ch[x] != ch[len - 1 - x]);
                if (m) {
                    const int f = i0 + __ffsll((unsigned long long)m) - 1;
                    rev = ch[len - 1 - f] < ch[f];
                    break;
                }
            }
        }
        if (rev) flag |= kRev;
        uint64_t hl = 0;
        for (int j = lane; j < len; j += kWave) hl ^= col_hash(canon_at(ch, len, rev, j), j, len);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) hl ^= __shfl_xor(hl, o, kWave);
        h = (sm_mix((uint64_t)len + 0x632BE59BD9B4E019ULL) ^ hl) | 1;
        // the tabu set as it stood before this chunk
        uint64_t slot = h & q.tabu_mask;
        for (;;) {
            const uint64_t th = B.thash[slot];
            if (th == 0) break;
            if (th == h) {
                const int e = B.tref[slot];
                if (B.tlen[e] == len) {
                    const uint16_t *ts = B.tarena + (size_t)e * kmax;
                    bool mis = false;
                    for (int j = lane; j < len; j += kWave) mis |= ts[j] != canon_at(ch, len, rev, j);
                    if (__ballot(mis) == 0) {
                        flag |= kInSet;
                        break;
                    }
                }
            }
            slot = (slot + 1) & q.tabu_mask;
        }
    }
    const int stored = len < kmax ? len : kmax;
    for (int j = lane; j < stored; j += kWave) B.child[(size_t)i * kmax + j] = ch[j];
    if (lane == 0) {
        B.clen[i] = len;
        B.cflag[i] = flag;
        B.chash[i] = h;
    }
}

// (defined with dl_pack_kernel below)
__device__ void pack_offsets(DlBufs B, int which, int n, int *s_tmp);

// Steps 5-6 in attempt order, for the chunk: a child repeating an earlier
// child of the chunk (same canonical series) or one in the tabu set is a tabu
// hit; a child of the wrong length (or none) fails; the rest fill the
// population's slots. The run stops when a slot has used max_attempts
// attempts (the next attempt is not drawn), or when the hits reach
// max_tabu_hits. Repeats are found by sorting (hash, index); the rules are
// then applied with block scans. Accepted children go to their slots of the
// next population. One workgroup.
__global__ void __launch_bounds__(kBlock) dl_accept_kernel(DlParams q, DlBufs B,
                                                           const int32_t *att_end, int cur,
                                                           int last_chunk) {
    extern __shared__ uint64_t s_dyn[];
    // the table: a 32-bit tag of each hash (its high half, odd; 0 = empty)
    // in the slot its low bits pick, and the smallest attempt with that tag
    uint32_t *s_th = reinterpret_cast<uint32_t *>(s_dyn);
    uint32_t *s_ti = s_th + kDedupSlots;
    __shared__ int s_tmp[33];
    DlState *st = B.st;
    const int tid = threadIdx.x, nt = blockDim.x, kmax = q.kmax;
    if (!fill_active(st)) return;
    const int A = st->chunk_n;
    constexpr uint32_t kMask = kDedupSlots - 1;
    // each thread takes a contiguous range of attempts; their flags, hashes
    // and lengths are loaded once, all in flight together, and kept in
    // registers
    constexpr int kPer = (kChunkMax + kBlock - 1) / kBlock;
    const int per = (A + nt - 1) / nt, lo = tid * per, hi = lo + per < A ? lo + per : A;
    uint32_t fl[kPer];
    uint64_t hh[kPer];
    int cl[kPer];
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        const bool in = lo + r < hi;
        fl[r] = in ? B.cflag[lo + r] : 0u;
        hh[r] = in ? B.chash[lo + r] : 0ull;
        cl[r] = in ? B.clen[lo + r] : 0;
    }
    for (int x = tid; x < kDedupSlots; x += nt) {
        s_th[x] = 0;
        s_ti[x] = 0xFFFFFFFFu;
    }
    __syncthreads();
    // a chunk's children that repeat an earlier child of the chunk: every
    // valid child enters a table keyed by its hash's tag, keeping the
    // smallest attempt index; a child whose entry holds a smaller index with
    // the same canonical series repeats it (a different series under the
    // same tag, vanishingly rare, falls back to comparing every earlier
    // child with the same hash)
    auto tag_of = [](uint64_t h) { return (uint32_t)(h >> 32) | 1u; };
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        if (!(fl[r] & kValid)) continue;
        const uint32_t tg = tag_of(hh[r]);
        uint32_t slot = (uint32_t)hh[r] & kMask;
        for (;;) {
            const uint32_t prev = atomicCAS(&s_th[slot], 0u, tg);
            if (prev == 0u || prev == tg) {
                atomicMin(&s_ti[slot], (uint32_t)(lo + r));
                break;
            }
            slot = (slot + 1) & kMask;
        }
    }
    __syncthreads();
    auto same_series = [&](int i, int li, int j) {
        if (B.clen[j] != li) return false;
        if (li <= 0) return true;
        const bool ri = (B.cflag[i] & kRev) != 0, rj = (B.cflag[j] & kRev) != 0;
        const uint16_t *ci = B.child + (size_t)i * kmax, *cj = B.child + (size_t)j * kmax;
        // sixteen columns per round of loads (a repeated child matches to
        // the end); positions past the series repeat its last one
        bool same = true;
        for (int e0 = 0; e0 < li && same; e0 += 16) {
            int ca[16], cb[16];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int e = e0 + u < li ? e0 + u : li - 1;
                ca[u] = canon_at(ci, li, ri, e);
                cb[u] = canon_at(cj, li, rj, e);
            }
#pragma unroll
            for (int u = 0; u < 16; u++) same &= ca[u] == cb[u];
        }
        return same;
    };
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        const int i = lo + r;
        if (!(fl[r] & kValid)) continue;
        const uint64_t h = hh[r];
        const uint32_t tg = tag_of(h);
        uint32_t slot = (uint32_t)h & kMask;
        while (s_th[slot] != tg) slot = (slot + 1) & kMask;
        const int m = (int)s_ti[slot];
        if (m >= i) continue;
        bool dup = same_series(i, cl[r], m);
        for (int j = 0; j < i && !dup; j++)
            if (j != m && (B.cflag[j] & kValid) && B.chash[j] == h && same_series(i, cl[r], j))
                dup = true;
        if (dup) fl[r] |= kDup;  // only this kernel reads it
    }
    __syncthreads();
    const int Nn0 = st->Nn, att0 = st->att, tabu0 = st->tabu_n;
    const int64_t hits0 = st->hits;
    auto is_hit = [&](uint32_t f) { return (f & kValid) && (f & (kInSet | kDup)); };
    auto is_acc = [&](uint32_t f) { return (f & kValid) && !(f & (kInSet | kDup)); };
    int nacc = 0, nhit = 0, last = -1;
#pragma unroll
    for (int r = 0; r < kPer; r++) {
        nhit += is_hit(fl[r]);
        if (is_acc(fl[r])) {
            nacc++;
            last = lo + r;
        }
    }
    int tot_acc = 0, tot_hit = 0;
    const int e_acc = block_excl_scan(nacc, s_tmp, &tot_acc);
    const int e_hit = block_excl_scan(nhit, s_tmp, &tot_hit);
    const int prev_last = block_excl_max(last, s_tmp);
    // the first event (index * 4 + kind: 0 exhausted, 1 tabu limit, 2 full)
    int event = 0x7fffffff;
    {
        int acc = e_acc, hit = e_hit, la = prev_last;
        for (int r = 0; r < kPer && lo + r < hi; r++) {
            const int i = lo + r;
            const int att_before = la < 0 ? att0 + i : i - la - 1;
            if (att_before >= q.max_att) {
                event = i * 4;
                break;
            }
            if (is_hit(fl[r])) {
                hit++;
                if (hits0 + hit >= q.max_hits) {
                    event = i * 4 + 1;
                    break;
                }
            }
            if (is_acc(fl[r])) {
                acc++;
                la = i;
                if (Nn0 + acc == q.P) {
                    event = i * 4 + 2;
                    break;
                }
            }
        }
    }
    const int ev = block_min(event, s_tmp);
    const int kind = ev == 0x7fffffff ? -1 : ev & 3, iev = ev == 0x7fffffff ? A : ev >> 2;
    const int lim = kind < 0 ? A : (kind == 0 ? iev : iev + 1);  // attempts made
    // accepted children of the attempts made: their slots in the next
    // population and their tabu arena entries (the insert kernel copies them)
    int uacc = 0, uhit = 0, ulast = -1;
    {
        const int nxt = cur ^ 1;
        int acc = e_acc;
        for (int r = 0; r < kPer && lo + r < hi && lo + r < lim; r++) {
            const int i = lo + r;
            uhit += is_hit(fl[r]);
            if (!is_acc(fl[r])) continue;
            B.cslot[i] = Nn0 + acc;
            B.carena[i] = tabu0 + acc;
            B.plen[nxt][Nn0 + acc] = cl[r];
            B.cflag[i] = fl[r] | kAccept;
            acc++;
            uacc++;
            ulast = i;
        }
    }
    int used_acc = 0, used_hit = 0;
    (void)block_excl_scan(uacc, s_tmp, &used_acc);
    (void)block_excl_scan(uhit, s_tmp, &used_hit);
    const int last_acc = block_min(ulast < 0 ? 0x7fffffff : -ulast, s_tmp);  // -(largest)
    if (tid == 0) {
        st->hits = hits0 + used_hit;
        st->Nn = Nn0 + used_acc;
        int64_t consumed = 0;
        if (kind < 0) {
            st->att = last_acc == 0x7fffffff ? att0 + A : A - 1 - (-last_acc);
            st->need_more = 1;
            consumed = A > 0 ? att_end[A - 1] : 0;
        } else {
            st->need_more = 0;
            if (kind == 0) st->stop = EBIC_STOP_EXHAUSTED;
            if (kind == 1) st->stop = EBIC_STOP_TABU;
            if (kind == 2) st->att = 0;
            consumed = kind == 0 ? B.att_off[iev] : att_end[iev];
        }
        st->rng += (uint64_t)consumed * kGamma;
        st->tabu_n = tabu0 + used_acc;
        if (tabu0 + used_acc > q.tabu_cap) st->error = 1;
        st->pending = 1;
        st->packed = kind == 2;
        st->chunk_first = Nn0;
        if (st->stop) st->over = 1;
        // the queued chunks are used up and the fill goes on: the host runs
        // the rest of it
        if (last_chunk && st->need_more && !st->stop) st->stalled = 1;
    }
    // the fill is complete: the next population's offsets for the evaluator
    // (every length is written: the elites' by the list update, the
    // children's above, before the scans' barriers)
    if (kind == 2) pack_offsets(B, cur ^ 1, q.P, s_tmp);
}

// Inserts canonical series into the tabu set, a wave each: the chunk's
// accepted children (cols = the children, flags with kAccept), each also
// copied to its slot of the next population (buffer nxt); or (flags NULL)
// the n series given, already canonical.
constexpr int kInsertWaves = 4;

__global__ void __launch_bounds__(kInsertWaves *kWave)
    dl_insert_kernel(DlParams q, DlBufs B, const uint16_t *cols, const int32_t *lens,
                     const uint32_t *flags, const uint64_t *hashes, int n, int nxt,
                     int32_t *size_field, int32_t *len_field) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int i = blockIdx.x * kInsertWaves + wave;
    // the list's size and length into the evaluator's table (final for the
    // generation by now), whether or not the run goes on
    if (size_field && blockIdx.x == 0 && threadIdx.x == 0) {
        *size_field = B.st->nA;
        *len_field = B.st->arch_len;
    }
    // a fill completed by this chunk: the population packed for the
    // evaluator with its columns' use counts (dl_copy_kernel's work), the
    // slots filled before the chunk from the population, the chunk's
    // children below from their source
    const bool pack = flags && B.st->pending && B.st->packed;
    if (pack && i < B.st->chunk_first) {
        const int k = B.plen[nxt][i], o = B.csr_off[i];
        const uint16_t *src = B.pop[nxt] + (size_t)i * q.kmax;
        for (int e = lane; e < k; e += kWave) {
            const uint16_t c = src[e];
            B.csr_cols[o + e] = c;
            atomicAdd(&B.use[nxt][c], 1);
        }
    }
    if (i >= n) return;
    const int kmax = q.kmax;
    const int len = lens[i];
    const uint16_t *s = cols + (size_t)i * kmax;
    bool rev = false;
    uint64_t h;
    if (flags) {
        // the accepted children of a chunk whose acceptance ran
        if (!B.st->pending) return;
        if (i >= B.st->chunk_n || !(flags[i] & kAccept)) return;
        rev = (flags[i] & kRev) != 0;
        h = hashes[i];
        const int slot = B.cslot[i];
        for (int j = lane; j < len; j += kWave) B.pop[nxt][(size_t)slot * kmax + j] = s[j];
        if (pack) {
            const int o = B.csr_off[slot];
            for (int j = lane; j < len; j += kWave) {
                B.csr_cols[o + j] = s[j];
                atomicAdd(&B.use[nxt][s[j]], 1);
            }
        }
    } else {
        uint64_t hl = 0;
        for (int j = lane; j < len; j += kWave) hl ^= col_hash(s[j], j, len);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) hl ^= __shfl_xor(hl, o, kWave);
        h = (sm_mix((uint64_t)len + 0x632BE59BD9B4E019ULL) ^ hl) | 1;
    }
    // the arena entry: given by the acceptance (children), or the entry's
    // own index (the first population's series)
    const int e = flags ? B.carena[i] : i;
    if (e >= q.tabu_cap) return;
    for (int j = lane; j < len; j += kWave)
        B.tarena[(size_t)e * kmax + j] = (uint16_t)canon_at(s, len, rev, j);
    if (lane == 0) {
        B.tlen[e] = len;
        uint64_t slot = h & q.tabu_mask;
        while (atomicCAS(reinterpret_cast<unsigned long long *>(&B.thash[slot]), 0ull,
                         (unsigned long long)h) != 0ull)
            slot = (slot + 1) & q.tabu_mask;
        B.tref[slot] = e;
    }
}

// The evaluator's job table takes the list's size and length from the state
// (the table was laid out for the largest list).
__global__ void dl_patch_kernel(DlBufs B, int32_t *size_field, int32_t *len_field) {
    if (threadIdx.x == 0) {
        *size_field = B.st->nA;
        *len_field = B.st->arch_len;
    }
}

__global__ void dl_resume_kernel(DlBufs B) {
    if (threadIdx.x == 0) B.st->stalled = 0;
}

// The population in buffer `which` packed as CSR for the evaluator: its
// offsets, by one workgroup (s_tmp holds 33 ints).
__device__ void pack_offsets(DlBufs B, int which, int n, int *s_tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (n + nt - 1) / nt, lo = tid * per, hi = lo + per < n ? lo + per : n;
    int sum = 0;
    for (int i = lo; i < hi; i++) sum += B.plen[which][i];
    int total = 0;
    int at = block_excl_scan(sum, s_tmp, &total);
    for (int i = lo; i < hi; i++) {
        B.csr_off[i] = at;
        at += B.plen[which][i];
    }
    if (tid == 0) B.csr_off[n] = total;
}

// pack_offsets as a kernel of its own (with `check`, only while the run goes
// on), for the first population; the acceptance kernel packs each later
// population, the one whose fill it completes.
__global__ void __launch_bounds__(kBlock) dl_pack_kernel(DlParams q, DlBufs B, int which, int n,
                                                         int check) {
    __shared__ int s_tmp[33];
    if (check && (B.st->over || B.st->stalled)) return;
    pack_offsets(B, which, n, s_tmp);
}

// The columns of the first population packed for the evaluator, a wave per
// individual (after its offsets), and their use counts for the crowding keys
// (later populations: the insert kernel of the chunk that completes a fill).
__global__ void __launch_bounds__(256) dl_copy_kernel(DlParams q, DlBufs B, int which, int n,
                                                      int check) {
    if (check && (B.st->over || B.st->stalled)) return;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    if (i >= n) return;
    const int k = B.plen[which][i], o = B.csr_off[i];
    const uint16_t *s = B.pop[which] + (size_t)i * q.kmax;
    for (int e = lane; e < k; e += kWave) {
        const uint16_t c = s[e];
        B.csr_cols[o + e] = c;
        atomicAdd(&B.use[which][c], 1);
    }
}

// ---- host driver ----

size_t pow2_at_least(size_t x) {
    size_t v = 1;
    while (v < x) v <<= 1;
    return v;
}

size_t chain_lds(int S, int E) {
    const size_t nseg = (size_t)(S + kSeg - 1) / kSeg;
    size_t b = ((size_t)S + 7) & ~(size_t)7;
    b += (nseg * E * 2 + 7) & ~(size_t)7;
    b += (nseg * E + 7) & ~(size_t)7;
    b += nseg * 8;
    return b;
}

}  // namespace

namespace {
// Device memory of a run's loop: the tabu set (cap series in an arena, a
// table of `slots`), two populations with their packed copies, supports,
// keys and use counts, the list's slots, one chunk's attempts, the span
// and the trace.
size_t loop_bytes(int64_t cap, size_t slots, int P, int K, int kmax, int W, int G) {
    return (size_t)cap * (2 * kmax + 4) + slots * 12 +
           (size_t)P * (2 * 2 * kmax + 8 + 2 * kmax + 4 + 8 + 4 + 8 * W + 8) +
           (size_t)(K + 2) * (2 * kmax + 8 * W) * 2 +
           (size_t)kChunkMax * (2 * kmax + 4 + 4 + 4 + 8 + 4) + kSpanMax + (size_t)G * 32;
}
}  // namespace

size_t devloop_bytes(int32_t rows, int32_t cols, const ebic_params &p) {
    (void)cols;
    const int P = p.population, G = p.generations > 1 ? p.generations : 1;
    // the first population's series and one per slot of every later generation
    const int64_t cap = (int64_t)P * G + 1;
    return loop_bytes(cap, pow2_at_least((size_t)(2 * cap)), P, p.archive_size, p.k_max,
                      rows_padded(rows) / 64, G);
}

int devloop_check(int32_t cols, const ebic_params &p) {
    (void)cols;
    if (p.tournament > kDlMaxT)
        return fail(EBIC_ERR_INVALID_ARG, "tournament %d: the device loop takes at most %d "
                    "(ebic_run takes any)", p.tournament, kDlMaxT);
    if (p.population > kDlMaxP)
        return fail(EBIC_ERR_INVALID_ARG, "population %d: the device loop takes at most %d "
                    "(ebic_run takes any)", p.population, kDlMaxP);
    return EBIC_OK;
}

struct DevLoopAccess {
    static int run(Job &job, Batch **batch, hipStream_t stream);
};

int devloop_run(Job &job, Batch **batch, hipStream_t stream) {
    return DevLoopAccess::run(job, batch, stream);
}

#define DL_HIP(call) EBIC_HIP(call)

int DevLoopAccess::run(Job &job, Batch **batch, hipStream_t stream) {
    const ebic_params &p = job.p_;
    int rc = devloop_check(job.C_, p);
    if (rc) return rc;
    DlParams q{};
    q.P = p.population;
    q.C = job.C_;
    q.W = job.W_;
    q.kmin = p.k_min;
    q.kmax = p.k_max;
    q.K = p.archive_size;
    q.T = p.tournament;
    q.G = p.generations;
    q.max_att = p.max_attempts;
    q.min_rows = p.min_rows;
    q.k_score_min = p.k_score_min;
    q.neg = p.negative_trends;
    q.theta = p.overlap_permille;
    for (int o = 0; o < 5; o++) q.opw[o] = job.op_w_[o];
    q.max_hits = p.max_tabu_hits;
    q.span_e = 2 * q.T + 12;  // at most 2T + 3 draws, and up to 8 rejected ones
    const int P = q.P, K = q.K, kmax = q.kmax, W = q.W, C = q.C;
    const int Pn0 = (int)job.pop_.size();
    // every series that can enter the tabu set: the first population's and
    // one per slot of every later generation
    const int64_t cap = (int64_t)job.tabu_.size() + (int64_t)P * (q.G > 1 ? q.G - 1 : 0) + 1;
    const size_t slots = pow2_at_least((size_t)(2 * cap));
    q.tabu_mask = slots - 1;
    if (cap > INT32_MAX / 4) return fail(EBIC_ERR_CAPACITY, "tabu set of %lld series", (long long)cap);
    q.tabu_cap = (int32_t)cap;
    const size_t bytes = loop_bytes(cap, slots, P, K, kmax, W, q.G);
    size_t free_b = 0, total_b = 0;
    DL_HIP(hipMemGetInfo(&free_b, &total_b));
    if (bytes > free_b / 2)
        return fail(EBIC_ERR_CAPACITY, "the device loop needs %zu bytes (tabu set of %lld series)",
                    bytes, (long long)cap);
    const ebic_allocator *al = job.al_;
    DeviceArray<uint16_t> pop0, pop1, csr_cols, aslot_cols, arch_cols, child, tarena;
    DeviceArray<int32_t> plen0, plen1, csr_off, cnt, arch_off, att_off, att_end, clen, tref, tlen,
        cslot, carena, use0, use1;
    DeviceArray<double> fit, keys, trace;
    DeviceArray<uint64_t> sup, aslot_sup, arch_sup, chash, thash;
    DeviceArray<uint8_t> span;
    DeviceArray<uint32_t> cflag;
    DeviceArray<DlState> st;
    DL_HIP(pop0.alloc((size_t)P * kmax, al, stream));
    DL_HIP(pop1.alloc((size_t)P * kmax, al, stream));
    DL_HIP(plen0.alloc(P, al, stream));
    DL_HIP(plen1.alloc(P, al, stream));
    DL_HIP(csr_off.alloc(P + 1, al, stream));
    DL_HIP(csr_cols.alloc((size_t)P * kmax, al, stream));
    DL_HIP(fit.alloc(P, al, stream));
    DL_HIP(cnt.alloc(P, al, stream));
    DL_HIP(sup.alloc((size_t)P * W, al, stream));
    DL_HIP(keys.alloc(P, al, stream));
    DL_HIP(aslot_cols.alloc((size_t)(K + 2) * kmax, al, stream));
    DL_HIP(aslot_sup.alloc((size_t)(K + 2) * W, al, stream));
    DL_HIP(arch_off.alloc(K + 3, al, stream));
    DL_HIP(arch_cols.alloc((size_t)(K + 2) * kmax, al, stream));
    DL_HIP(arch_sup.alloc((size_t)(K + 2) * W, al, stream));
    DL_HIP(span.alloc(kSpanMax + 16, al, stream));  // whole 16-byte loads past the last offset
    DL_HIP(att_off.alloc(kChunkMax, al, stream));
    DL_HIP(att_end.alloc(kChunkMax, al, stream));
    DL_HIP(child.alloc((size_t)kChunkMax * kmax, al, stream));
    DL_HIP(clen.alloc(kChunkMax, al, stream));
    DL_HIP(cslot.alloc(kChunkMax, al, stream));
    DL_HIP(carena.alloc(kChunkMax, al, stream));
    DL_HIP(use0.alloc(C, al, stream));
    DL_HIP(use1.alloc(C, al, stream));
    DL_HIP(hipMemsetAsync(use0.p, 0, sizeof(int32_t) * C, stream));
    DL_HIP(hipMemsetAsync(use1.p, 0, sizeof(int32_t) * C, stream));
    DL_HIP(cflag.alloc(kChunkMax, al, stream));
    DL_HIP(chash.alloc(kChunkMax, al, stream));
    DL_HIP(thash.alloc(slots, al, stream));
    DL_HIP(tref.alloc(slots, al, stream));
    DL_HIP(tarena.alloc((size_t)cap * kmax, al, stream));
    DL_HIP(tlen.alloc(cap, al, stream));
    DL_HIP(trace.alloc((size_t)q.G * 4, al, stream));
    DL_HIP(st.alloc(1, al, stream));
    DL_HIP(hipMemsetAsync(thash.p, 0, slots * sizeof(uint64_t), stream));

    DlBufs B{};
    B.pop[0] = pop0.p;
    B.pop[1] = pop1.p;
    B.plen[0] = plen0.p;
    B.plen[1] = plen1.p;
    B.csr_off = csr_off.p;
    B.csr_cols = csr_cols.p;
    B.fit = fit.p;
    B.cnt = cnt.p;
    B.sup = sup.p;
    B.keys = keys.p;
    B.use[0] = use0.p;
    B.use[1] = use1.p;
    B.aslot_cols = aslot_cols.p;
    B.aslot_sup = aslot_sup.p;
    B.arch_off = arch_off.p;
    B.arch_cols = arch_cols.p;
    B.arch_sup = arch_sup.p;
    B.span = span.p;
    B.att_off = att_off.p;
    B.child = child.p;
    B.clen = clen.p;
    B.cflag = cflag.p;
    B.chash = chash.p;
    B.cslot = cslot.p;
    B.carena = carena.p;
    B.thash = thash.p;
    B.tref = tref.p;
    B.tarena = tarena.p;
    B.tlen = tlen.p;
    B.trace = trace.p;
    B.st = st.p;

    // the first population (drawn on the host, step 1) and its tabu entries
    PinnedArray<DlState> hs;
    DL_HIP(hs.alloc(1));
    std::memset(hs.p, 0, sizeof(DlState));
    hs.p->rng = job.rng_.state();
    hs.p->hits = job.tabu_hits_;
    hs.p->stop = job.stop_;
    for (int j = 0; j < EBIC_MAX_ARCHIVE + 2; j++) hs.p->slot[j] = -1;
    DL_HIP(hipMemcpyAsync(st.p, hs.p, sizeof(DlState), hipMemcpyHostToDevice, stream));
    {
        std::vector<uint16_t> hp((size_t)std::max(Pn0, 1) * kmax, 0);
        std::vector<int32_t> hl(std::max(Pn0, 1), 0);
        for (int i = 0; i < Pn0; i++) {
            std::copy(job.pop_[i].begin(), job.pop_[i].end(), hp.begin() + (size_t)i * kmax);
            hl[i] = (int32_t)job.pop_[i].size();
        }
        DL_HIP(hipMemcpyAsync(pop0.p, hp.data(), sizeof(uint16_t) * hp.size(),
                              hipMemcpyHostToDevice, stream));
        DL_HIP(hipMemcpyAsync(plen0.p, hl.data(), sizeof(int32_t) * hl.size(),
                              hipMemcpyHostToDevice, stream));
        std::vector<uint16_t> tc;
        std::vector<int32_t> tl;
        job.tabu_.for_each([&](const uint16_t *c, size_t k) {
            const size_t at = tc.size();
            tc.resize(at + kmax, 0);
            std::copy(c, c + k, tc.begin() + at);
            tl.push_back((int32_t)k);
        });
        const int nt = (int)tl.size();
        {
            // the first population's series take arena entries 0 .. nt - 1
            const int32_t ntv = nt;
            DL_HIP(hipMemcpyAsync(&st.p->tabu_n, &ntv, sizeof(int32_t), hipMemcpyHostToDevice,
                                  stream));
            DL_HIP(hipStreamSynchronize(stream));
        }
        if (nt > 0) {
            DeviceArray<uint16_t> dtc;
            DeviceArray<int32_t> dtl;
            DL_HIP(dtc.alloc(tc.size(), al, stream));
            DL_HIP(dtl.alloc(nt, al, stream));
            DL_HIP(hipMemcpyAsync(dtc.p, tc.data(), sizeof(uint16_t) * tc.size(),
                                  hipMemcpyHostToDevice, stream));
            DL_HIP(hipMemcpyAsync(dtl.p, tl.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice,
                                  stream));
            hipLaunchKernelGGL(dl_insert_kernel, dim3((nt + kInsertWaves - 1) / kInsertWaves),
                               dim3(kInsertWaves * kWave), 0, stream, q, B, dtc.p, dtl.p, nullptr,
                               nullptr, nt, 0, (int32_t *)nullptr, (int32_t *)nullptr);
            DL_HIP(hipGetLastError());
            DL_HIP(hipStreamSynchronize(stream));  // before the host copies go out of scope
        }
        if (Pn0 > 0) {
            hipLaunchKernelGGL(dl_pack_kernel, dim3(1), dim3(kBlock), 0, stream, q, B, 0, Pn0, 0);
            hipLaunchKernelGGL(dl_copy_kernel, dim3((Pn0 + 3) / 4), dim3(256), 0, stream, q, B, 0,
                               Pn0, 0);
            DL_HIP(hipGetLastError());
        }
        DL_HIP(hipStreamSynchronize(stream));
    }

    const int Ppad = (int)pow2_at_least((size_t)std::max(P, 2));
    const size_t lds_list = list_lds_bytes(Ppad, C);
    DL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(dl_list_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_list));
    DL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(dl_chain_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)chain_lds(kSpanMax, q.span_e)));
    DL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(dl_accept_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kDedupSlots * 8));
    auto read_state = [&]() -> int {
        DL_HIP(hipMemcpyAsync(hs.p, st.p, sizeof(DlState), hipMemcpyDeviceToHost, stream));
        DL_HIP(hipStreamSynchronize(stream));
        return EBIC_OK;
    };

    // The evaluator's batch, laid out once for the largest list; the list's
    // size and length go into its table before each evaluation: before the
    // first from a kernel of their own, later from the previous generation's
    // insert kernels.
    {
        ebic_job v{};
        v.matrix = job.m_;
        v.population = ebic_population{Pn0, Pn0 * kmax, csr_off.p, csr_cols.p, nullptr};
        v.archive = ebic_archive{K, K * kmax, arch_sup.p, arch_off.p, arch_cols.p};
        v.params = p;
        v.out = ebic_eval_out{fit.p, cnt.p, sup.p, nullptr};
        rc = batch_set(batch, &v, 1, stream, al);
        if (rc) return rc;
    }
    int32_t *f_size = nullptr, *f_len = nullptr;
    rc = batch_archive_fields(*batch, 0, &f_size, &f_len);
    if (rc) return rc;
    // The generations run on a stream of their own (non-blocking) when the
    // caller's is the null stream, which would wait on other streams' work
    // between launches; everything before is finished first, and the loop
    // ends with its stream synchronized.
    struct OwnStream {
        hipStream_t s = nullptr;
        ~OwnStream() {
            if (s) (void)hipStreamDestroy(s);
        }
    } own;
    DL_HIP(hipStreamSynchronize(stream));
    if (!stream && hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking) == hipSuccess)
        stream = own.s;
    auto chunk = [&](int cur, int Pn, int R, int last) -> int {
        const int A_target = std::min(kChunkMax, R + R / 2 + 64);
        const int S = std::min(kSpanMax, A_target * (2 * q.T + 3));
        hipLaunchKernelGGL(dl_span_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, q, B, cur,
                           Pn, S);
        hipLaunchKernelGGL(dl_chain_kernel, dim3(1), dim3(kBlock), chain_lds(S, q.span_e), stream,
                           q, B, att_end.p, cur, Pn, S, A_target);
        hipLaunchKernelGGL(dl_child_kernel, dim3((A_target + kChildWaves - 1) / kChildWaves),
                           dim3(kChildWaves * kWave), 0, stream, q, B, cur, Pn);
        hipLaunchKernelGGL(dl_accept_kernel, dim3(1), dim3(kBlock), (size_t)kDedupSlots * 8,
                           stream, q, B, (const int32_t *)att_end.p, cur, last);
        // a wave per attempt, and per individual for the population's copy
        const int waves = std::max(A_target, P);
        hipLaunchKernelGGL(dl_insert_kernel, dim3((waves + kInsertWaves - 1) / kInsertWaves),
                           dim3(kInsertWaves * kWave), 0, stream, q, B, (const uint16_t *)child.p,
                           (const int32_t *)clen.p, (const uint32_t *)cflag.p,
                           (const uint64_t *)chash.p, A_target, cur ^ 1, f_size, f_len);
        DL_HIP(hipGetLastError());
        return EBIC_OK;
    };
    // One generation queued: score population gi (buffer gi % 2), update the
    // list, keys, the fill's first nq chunks, pack the next population. Every
    // kernel does nothing once the run is over or a fill has stalled.
    // Chunks queued per generation: first enough for a quarter more attempts
    // than the population; after a fill has needed more (many tabu hits or
    // children of the wrong length), enough for half as many again. A chunk
    // queued beyond the fill's need still costs its five launches.
    const int per_chunk = std::min(kChunkMax, P + P / 2 + 64);
    const int nq_lo = std::max(1, (P + P / 4 + 64 + per_chunk - 1) / per_chunk);
    const int nq_hi = std::max(nq_lo, (P + P / 2 + 64 + kChunkMax - 1) / kChunkMax);
    auto queue_generation = [&](int gi, int nq) -> int {
        const int cur = gi & 1, Pn = gi == 0 ? Pn0 : P;
        // later generations take the list's size from the previous one's insert
        if (gi == 0) {
            hipLaunchKernelGGL(dl_patch_kernel, dim3(1), dim3(64), 0, stream, B, f_size, f_len);
            DL_HIP(hipGetLastError());
        }
        if (Pn > 0) {
            int r = batch_run(*batch, stream);
            if (r) return r;
        }
        hipLaunchKernelGGL(dl_list_kernel, dim3(1), dim3(kBlock), lds_list, stream, q, B, cur, Pn,
                           Ppad);
        hipLaunchKernelGGL(dl_keys_kernel, dim3((std::max(Pn, C / 64 + 1) + 3) / 4), dim3(256), 0,
                           stream, q, B, cur, Pn);
        DL_HIP(hipGetLastError());
        for (int c = 0; c < nq; c++) {
            int r = chunk(cur, Pn, P, c == nq - 1);
            if (r) return r;
        }
        // (the acceptance kernel that completes the fill packs the offsets,
        // the chunk's insert kernel the columns)
        return EBIC_OK;
    };
    // Each generation's kernels are launched one by one, a few generations
    // ahead of the GPU: on batched-10000x500, replaying each generation from
    // a captured graph (one per population parity and chunk count) took
    // 262-265 us a generation against 252-256 us launched directly.
    int variant = 0;  // 1 once a fill has stalled: nq_hi chunks from then on
    auto queue = [&](int gi) -> int { return queue_generation(gi, variant ? nq_hi : nq_lo); };
    // generations are queued a few at a time; the host reads the state
    // between groups
    constexpr int kAhead = 8;
    int gi = 0;
    for (;;) {
        const int upto = std::min(q.G, gi + kAhead);
        for (int x = gi; x < upto; x++)
            if ((rc = queue(x))) return rc;
        if ((rc = read_state())) return rc;
        if (hs.p->error) return fail(EBIC_ERR_CAPACITY, "device loop: the tabu set is full");
        if (hs.p->over) break;
        if (hs.p->stalled) {
            // finish the stalled fill chunk by chunk, then go on, queueing
            // more chunks per generation
            variant = 1;
            const int cur = (hs.p->g - 1) & 1;
            dl_resume_kernel<<<1, 64, 0, stream>>>(B);
            for (;;) {
                if ((rc = chunk(cur, P, P - hs.p->Nn, 0))) return rc;
                if ((rc = read_state())) return rc;
                if (hs.p->error) return fail(EBIC_ERR_CAPACITY, "device loop: the tabu set is full");
                if (!hs.p->need_more || hs.p->stop) break;
            }
            if (hs.p->over) break;
            // the chunk that completed the fill has packed the population
        }
        if (hs.p->g >= q.G) return fail(EBIC_ERR_DEVICE, "device loop: no stop after %d generations",
                                         hs.p->g);
        gi = hs.p->g;
    }

    // the run's state back into the job, which then takes the final step
    // (step 9) as the host loop does
    const DlState &S = *hs.p;
    std::vector<double> tr((size_t)S.g * 4);
    if (S.g > 0)
        DL_HIP(hipMemcpyAsync(tr.data(), trace.p, sizeof(double) * tr.size(),
                              hipMemcpyDeviceToHost, stream));
    std::vector<uint16_t> acols((size_t)(K + 2) * kmax);
    std::vector<uint64_t> asup((size_t)(K + 2) * W);
    DL_HIP(hipMemcpyAsync(acols.data(), aslot_cols.p, sizeof(uint16_t) * acols.size(),
                          hipMemcpyDeviceToHost, stream));
    DL_HIP(hipMemcpyAsync(asup.data(), aslot_sup.p, sizeof(uint64_t) * asup.size(),
                          hipMemcpyDeviceToHost, stream));
    DL_HIP(hipStreamSynchronize(stream));
    job.archive_.clear();
    for (int j = 0; j < S.nA; j++) {
        const int sl = S.slot[j];
        Member m;
        m.s.assign(acols.begin() + (size_t)sl * kmax, acols.begin() + (size_t)sl * kmax + S.a_len[sl]);
        m.support.assign(asup.begin() + (size_t)sl * W, asup.begin() + (size_t)(sl + 1) * W);
        m.n = S.a_n[sl];
        m.score = S.a_score[sl];
        job.archive_.push_back(std::move(m));
    }
    job.g_ = S.g;
    job.evaluations_ = S.evaluations;
    job.tabu_hits_ = S.hits;
    job.stop_ = S.stop;
    job.res_->trace = std::move(tr);
    const int32_t nb = std::min((int32_t)job.archive_.size(), std::max(p.n_out, 0));
    job.pop_.clear();
    for (int32_t j = 0; j < nb; j++) job.pop_.push_back(job.archive_[j].s);
    job.phase_ = Job::Phase::FinalEval;
    return EBIC_OK;
}

}  // namespace ebic
