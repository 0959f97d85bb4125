// Sort strategy: conflicts between returns that share a voxel resolved by
// sorting instead of atomics on the voxel planes.
//
// Eq. 4 ANDs masks into a word and eqs. 5-6 add hits to a saturating counter;
// both are commutative, so the changes of all returns of a call to one voxel
// word can be combined first and applied once: the AND of the masks, and the
// count n of hits taken as h -> min(h + n, H_max) with the sign cleared when
// h < T <= min(h + n, H_max) (the composition of n single steps of eqs. 5-6).
// The passes, after the per-point front end and survivor selection that the
// atomic strategy also runs:
//   1. k_mark_pairs: one wavefront per survivor reads its window and shadow
//      words once and keeps, per pass of 64 cells, the ballot of the cells
//      that need a pair: a window word whose mask would lose bits (read
//      first, as eq. 4's skipped writes) or a shadow cell whose counter is
//      below H_max; and its pair count;
//   2. an exclusive sum of the counts (rocPRIM): each survivor's first slot;
//   3. k_emit_pairs: each survivor writes its (key, contribution) pairs from
//      the ballots, with no atomics and no gaps;
//   4. a radix sort of the pairs by key (rocPRIM) over the key bits in use,
//      on 32-bit keys when they fit 31 bits;
//   5. k_reduce_pairs: a wavefront segmented reduction (a 64-lane scan of AND
//      and count that restarts at each new key) over a chunk of sorted pairs,
//      the last lane of each run writing the voxel's words with plain stores:
//      each voxel is one run, so no word is written twice.
// A read-first filter stays exact across rounds: planes only lose mask bits
// and gain hits, so a contribution that changes nothing now changes nothing
// later. Larger calls run in rounds of survivors whose pairs fit the buffers.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "runtime.h"

namespace dbtsdf {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t wave_uniform64(uint64_t v) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ unsigned long long shfl_up64(unsigned long long v, uint32_t d) {
    const uint32_t lo = __shfl_up((uint32_t)v, d, 64), hi = __shfl_up((uint32_t)(v >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long shfl_down64(unsigned long long v, uint32_t d) {
    const uint32_t lo = __shfl_down((uint32_t)v, d, 64), hi = __shfl_down((uint32_t)(v >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}

constexpr int kLoadBatch = 8;        // window loads in flight per lane
constexpr uint32_t kSegChunk = 512;  // sorted pairs per wavefront of the reduction

// The per-survivor geometry both passes walk: lanes cover floor(64 / K) rows
// of K cells per window pass; shadow passes take 64 cells each.
struct Walk {
    int K, R;
    bool l1;
    uint32_t l, wx, rpi, xi, ri, rows, n_pass, mag;
    int ox;
    __device__ Walk(const DevTables &t) {
        K = t.K;
        R = t.R;
        l1 = t.metric == DBTSDF_DIST_L1;
        l = lane_id();
        wx = (uint32_t)K;
        rpi = 64u / wx;
        xi = l % wx;
        ri = l / wx;
        rows = (uint32_t)(K * K);
        n_pass = (rows + rpi - 1u) / rpi;
        mag = ((1u << 20) + wx - 1u) / wx;
        ox = (int)xi - R;
    }
    // window pass p of this lane: row, cell offset from the corner and eq. 3 distance index
    __device__ bool cell(uint32_t p, uint32_t nx, uint32_t ny, uint64_t &off, uint32_t &q) const {
        const uint32_t rr = p * rpi + ri;
        const uint32_t rz = (rr * mag) >> 20, ry = rr - rz * wx;
        const int oy = (int)ry - R, oz = (int)rz - R;
        q = l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
        off = xi + (uint64_t)nx * (ry + (uint64_t)ny * rz);
        return ri < rpi && rr < rows;
    }
};

__device__ __forceinline__ uint64_t shadow_off(uint32_t pk, uint32_t nx, uint32_t ny) {
    return (uint64_t)(pk & 255u) + (uint64_t)nx * ((uint64_t)((pk >> 8) & 255u) + (uint64_t)ny * ((pk >> 16) & 255u));
}

struct Surv {
    uint4 r;
    uint32_t gi, nx, ny, hmax;
    const uint32_t *mask, *packed;
    uint64_t corner;
};
__device__ __forceinline__ Surv load_surv(const PipeArgs &a, uint32_t e, int R) {
    Surv v;
    v.r = a.surv_rec[e];
    v.gi = v.r.w >> 16;
    const DevGrid &g = a.grids[v.gi];
    v.nx = __builtin_amdgcn_readfirstlane(g.nx);
    v.ny = __builtin_amdgcn_readfirstlane(g.ny);
    v.hmax = __builtin_amdgcn_readfirstlane(g.hmax);
    v.mask = reinterpret_cast<const uint32_t *>(wave_uniform64(reinterpret_cast<uint64_t>(g.mask)));
    v.packed = reinterpret_cast<const uint32_t *>(wave_uniform64(reinterpret_cast<uint64_t>(g.packed)));
    v.corner = (uint64_t)(v.r.x - (uint32_t)R) +
               (uint64_t)v.nx * ((uint64_t)(v.r.y - (uint32_t)R) + (uint64_t)v.ny * (uint64_t)(v.r.z - (uint32_t)R));
    return v;
}

// Pass 1: per survivor of the round, the need ballot of every window pass
// (the word would lose mask bits) and shadow pass (the counter is below
// H_max), stored as 64-bit words, and the number of pairs it will emit. A
// return whose voxel an earlier call integrated skips its window (the words
// already hold these masks): its window words are not written nor read.
__global__ __launch_bounds__(kSortThreads) void k_mark_pairs(PipeArgs a, SortArgs s) {
    const DevTables &t = a.tab;
    const Walk w(t);
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t e = s.surv_lo + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < s.surv_hi; e += waves) {
        const Surv v = load_surv(a, e, w.R);
        unsigned long long *bits = s.bits + (uint64_t)(e - s.surv_lo) * s.words;
        uint32_t total = 0;
        if (!(a.revisit_ok && (v.r.w & kRecRevisit))) {
            unsigned long long mine = 0;   // lane u keeps the ballot of pass p0 + u of each 64
            for (uint32_t u0 = 0; u0 < w.n_pass; u0 += kLoadBatch) {
                uint32_t old[kLoadBatch], m[kLoadBatch];
                bool on[kLoadBatch];
#pragma unroll
                for (int u = 0; u < kLoadBatch; ++u) {
                    uint64_t off;
                    uint32_t q;
                    on[u] = w.cell(u0 + (uint32_t)u, v.nx, v.ny, off, q) && u0 + (uint32_t)u < w.n_pass;
                    m[u] = on[u] ? t.mask_by_q[q] : 0xFFFFFFFFu;
                    old[u] = on[u] ? v.mask[v.corner + off] : 0u;
                }
#pragma unroll
                for (int u = 0; u < kLoadBatch; ++u) {
                    const uint32_t p = u0 + (uint32_t)u;
                    const unsigned long long bal = __ballot(on[u] && (old[u] & m[u]) != old[u]);
                    total += (uint32_t)__popcll(bal);
                    if (w.l == (p & 63u)) mine = bal;
                    if ((p & 63u) == 63u || p + 1u == w.n_pass) {
                        if (w.l <= (p & 63u) && p < w.n_pass) bits[(p & ~63u) + w.l] = mine;
                    }
                }
            }
        }
        const uint32_t bin = v.r.w & (a.revisit_ok ? kRowBinMask : 0xFFFFu);
        const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
        const uint32_t n_sp = (s1 - s0 + 63u) / 64u;
        for (uint32_t p = 0; p < n_sp; ++p) {
            const uint32_t j = s0 + p * 64u + w.l;
            bool need = false;
            if (j < s1) need = (v.packed[v.corner + shadow_off(t.sh_off[j], v.nx, v.ny)] & 0xFFFFu) < v.hmax;
            const unsigned long long bal = __ballot(need);
            total += (uint32_t)__popcll(bal);
            if (w.l == 0) bits[w.n_pass + p] = bal;
        }
        if (w.l == 0) s.cnt[e - s.surv_lo] = total;
    }
}

// Pass 3 (after an exclusive sum of the counts): each survivor writes its
// pairs from its offset on, lanes ranked within each pass by its ballot.
template <typename KeyT>
__global__ __launch_bounds__(kSortThreads) void k_emit_pairs(PipeArgs a, SortArgs s) {
    const DevTables &t = a.tab;
    const Walk w(t);
    const unsigned long long below = w.l ? ((1ull << w.l) - 1ull) : 0ull;
    KeyT *keys = reinterpret_cast<KeyT *>(s.keys);
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t e = s.surv_lo + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < s.surv_hi; e += waves) {
        const Surv v = load_surv(a, e, w.R);
        const unsigned long long *bits = s.bits + (uint64_t)(e - s.surv_lo) * s.words;
        uint32_t slot = __builtin_amdgcn_readfirstlane(s.off[e - s.surv_lo]);
        const unsigned long long kbase = ((unsigned long long)v.gi << s.shift) + v.corner;
        if (!(a.revisit_ok && (v.r.w & kRecRevisit))) {
            for (uint32_t p = 0; p < w.n_pass; ++p) {
                const unsigned long long bal = wave_uniform64(bits[p]);
                if ((bal >> w.l) & 1ull) {
                    uint64_t off;
                    uint32_t q;
                    (void)w.cell(p, v.nx, v.ny, off, q);
                    const uint32_t at = slot + (uint32_t)__popcll(bal & below);
                    keys[at] = (KeyT)(kbase + off);
                    s.vals[at] = t.mask_by_q[q];
                }
                slot += (uint32_t)__popcll(bal);
            }
        }
        const uint32_t bin = v.r.w & (a.revisit_ok ? kRowBinMask : 0xFFFFu);
        const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
        const uint32_t n_sp = (s1 - s0 + 63u) / 64u;
        for (uint32_t p = 0; p < n_sp; ++p) {
            const unsigned long long bal = wave_uniform64(bits[w.n_pass + p]);
            if ((bal >> w.l) & 1ull) {
                const uint32_t at = slot + (uint32_t)__popcll(bal & below);
                keys[at] = (KeyT)(kbase + shadow_off(t.sh_off[s0 + p * 64u + w.l], v.nx, v.ny));
                s.vals[at] = kHitPair;
            }
            slot += (uint32_t)__popcll(bal);
        }
    }
}

// Apply one voxel's combined changes: AND of its masks (all ones when it had
// only hits) and its hit count.
__device__ __forceinline__ void apply_voxel(const DevGrid *grids, unsigned long long key, uint32_t shift, uint32_t am,
                                            uint32_t cn) {
    const DevGrid &g = grids[key >> shift];
    const uint64_t v = key & ((1ull << shift) - 1ull);
    if (am != 0xFFFFFFFFu) {
        const uint32_t old = g.mask[v], nw = old & am;
        if (nw != old) g.mask[v] = nw;
    }
    if (cn) {
        const uint32_t p = g.packed[v], h = p & 0xFFFFu, hmax = g.hmax, T = g.T;
        const uint32_t h2 = min(h + cn, hmax);
        uint32_t sign = p >> 31;
        if (sign && T >= 1u && h < T && T <= h2) sign = 0u;
        const uint32_t np = (sign << 31) | h2;
        if (np != p) g.packed[v] = np;
    }
}

__device__ __forceinline__ uint32_t shfl_up_k(uint32_t v, uint32_t d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ unsigned long long shfl_up_k(unsigned long long v, uint32_t d) { return shfl_up64(v, d); }
__device__ __forceinline__ uint32_t shfl_down_k(uint32_t v, uint32_t d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ unsigned long long shfl_down_k(unsigned long long v, uint32_t d) {
    return shfl_down64(v, d);
}
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return __builtin_amdgcn_readfirstlane(__shfl(v, 63, 64)); }
__device__ __forceinline__ unsigned long long lane63(unsigned long long v) {
    return wave_uniform64(__shfl(v, 63, 64));
}

// Wavefront segmented reduction of sorted pairs. Wavefront w owns the runs of
// equal keys that start in [w C, (w + 1) C) (C = kSegChunk), the last of them
// followed past the chunk's end; runs that started before are another's.
// Keys are below 2^31 (KeyT = uint32_t) or 2^63, so all ones marks no pair.
template <typename KeyT>
__global__ __launch_bounds__(kSortThreads) void k_reduce_pairs(const DevGrid *grids, const KeyT *keys,
                                                               const uint32_t *vals, uint32_t n, uint32_t shift) {
    const KeyT none = (KeyT)~(KeyT)0;
    const uint32_t l = lane_id();
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t c0 = (uint64_t)w * kSegChunk;
    if (c0 >= n) return;
    const uint32_t c1 = (uint32_t)min(c0 + kSegChunk, (uint64_t)n);
    // first run head at or after c0
    uint32_t s = c1;
    for (uint32_t p0 = (uint32_t)c0; p0 < c1; p0 += 64) {
        const uint32_t p = p0 + l;
        const bool hd = p < c1 && (p == 0 || keys[p] != keys[p - 1]);
        const unsigned long long bal = __ballot(hd);
        if (bal) {
            s = p0 + (uint32_t)__builtin_ctzll(bal);
            break;
        }
    }
    if (s >= c1) return;
    // end of the run open at c1: the first head at or after c1 (or n)
    uint32_t e = n;
    for (uint32_t p0 = c1; p0 < n; p0 += 64) {
        const uint32_t p = p0 + l;
        const bool hd = p >= n || keys[p] != keys[p - 1];
        const unsigned long long bal = __ballot(hd);
        if (bal) {
            e = p0 + (uint32_t)__builtin_ctzll(bal);
            break;
        }
    }
    // the run open at the start of a window: its key, AND and count so far
    KeyT ck = none;
    uint32_t cand = 0xFFFFFFFFu, ccnt = 0;
    for (uint32_t w0 = s; w0 < e; w0 += 64) {
        const uint32_t p = w0 + l;
        const bool in = p < e;
        const KeyT k = in ? keys[p] : none;
        const uint32_t v = in ? vals[p] : 0xFFFFFFFFu;
        KeyT kp = shfl_up_k(k, 1);
        if (l == 0) kp = ck;
        uint32_t am = v, cn = (in && v == kHitPair) ? 1u : 0u;
        uint32_t f = (in && k != kp) ? 1u : 0u;   // a run starts here
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t am_u = __shfl_up(am, d, 64), cn_u = __shfl_up(cn, d, 64), f_u = __shfl_up(f, d, 64);
            if (l >= d && !f) {
                am &= am_u;
                cn += cn_u;
                f = f_u;
            }
        }
        if (!f) {   // no head up to this lane: the run continues from the previous window
            am &= cand;
            cn += ccnt;
        }
        KeyT kn = shfl_down_k(k, 1);
        if (l == 63) kn = p + 1 < e ? keys[p + 1] : none;
        if (in && kn != k) apply_voxel(grids, (unsigned long long)k, shift, am, cn);
        ck = lane63(k);
        cand = lane63(am);
        ccnt = lane63(cn);
    }
}

template <typename T>
hipError_t grow(T *&p, size_t &cap, size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
}

hipError_t ensure_sort_buffers(SortBuffers &b, size_t pairs, size_t survivors, size_t words) {
    hipError_t e = hipSuccess;
    size_t kc = b.cap, vc = b.cap;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        kc = b.cap;
        vc = b.cap;
        e = grow(b.keys[i], kc, pairs);
        if (e == hipSuccess) e = grow(b.vals[i], vc, pairs);
    }
    if (e == hipSuccess) b.cap = std::max<size_t>(b.cap, pairs);
    size_t cc = b.surv_cap, oc = b.surv_cap;
    if (e == hipSuccess) e = grow(b.cnt, cc, survivors + 1);
    if (e == hipSuccess) e = grow(b.off, oc, survivors + 1);
    if (e == hipSuccess) b.surv_cap = std::max<size_t>(b.surv_cap, survivors + 1);
    if (e == hipSuccess) e = grow(b.bits, b.bits_cap, survivors * words);
    if (e != hipSuccess) free_sort_buffers(b);
    return e;
}

hipError_t ensure_tmp(SortBuffers &b, size_t bytes) {
    if (bytes <= b.tmp_bytes && b.tmp) return hipSuccess;
    if (b.tmp) (void)hipFree(b.tmp);
    b.tmp = nullptr;
    b.tmp_bytes = 0;
    hipError_t e = hipMalloc(&b.tmp, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) b.tmp_bytes = std::max<size_t>(bytes, 256);
    return e;
}

template <typename KeyT>
hipError_t sort_and_reduce(SortBuffers &b, const PipeArgs &a, const SortArgs &s, uint32_t n, uint32_t end_bit,
                           uint32_t emit_blocks, hipStream_t st) {
    k_emit_pairs<KeyT><<<emit_blocks, kSortThreads, 0, st>>>(a, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rocprim::double_buffer<KeyT> kb(reinterpret_cast<KeyT *>(b.keys[0]), reinterpret_cast<KeyT *>(b.keys[1]));
    rocprim::double_buffer<uint32_t> vb(b.vals[0], b.vals[1]);
    size_t bytes = 0;
    e = rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)n, 0u, end_bit, st);
    if (e == hipSuccess) e = ensure_tmp(b, bytes);
    if (e == hipSuccess) e = rocprim::radix_sort_pairs(b.tmp, bytes, kb, vb, (size_t)n, 0u, end_bit, st);
    if (e != hipSuccess) return e;
    const uint32_t waves = (n + kSegChunk - 1) / kSegChunk;
    const uint32_t blocks = (waves + (kSortThreads / 64) - 1) / (kSortThreads / 64);
    k_reduce_pairs<KeyT><<<blocks, kSortThreads, 0, st>>>(a.grids, kb.current(), vb.current(), n, s.shift);
    return hipGetLastError();
}

}  // namespace

const void *sort_emit_kernel() { return reinterpret_cast<const void *>(k_mark_pairs); }

void free_sort_buffers(SortBuffers &b) {
    void *p[] = {b.keys[0], b.keys[1], b.vals[0], b.vals[1], b.cnt, b.off, b.bits, b.tmp};
    for (void *x : p)
        if (x) (void)hipFree(x);
    b = SortBuffers{};
}

hipError_t sort_apply(Workspace &ws, const PipeArgs &a, const SortPlan &plan, hipStream_t st) {
    SortBuffers &b = ws.sorter;
    uint32_t n_surv = 0;
    // the select pass has counted everything: the statistics go out first
    hipError_t e = launch_stats_out(a, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&n_surv, &a.ctrl->n_survivors, sizeof(n_surv), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess || n_surv == 0) return e;
    unsigned long long per_round = std::max(1ull, kSortMaxPairs / plan.pairs_per_point);
    if (plan.round_survivors) per_round = std::min(per_round, (unsigned long long)plan.round_survivors);
    const size_t round = (size_t)std::min((unsigned long long)n_surv, per_round);
    e = ensure_sort_buffers(b, round * plan.pairs_per_point, round, plan.words);
    for (unsigned long long lo = 0; e == hipSuccess && lo < n_surv; lo += per_round) {
        SortArgs s{};
        s.keys = b.keys[0];
        s.vals = b.vals[0];
        s.bits = b.bits;
        s.cnt = b.cnt;
        s.off = b.off;
        s.shift = plan.shift;
        s.words = plan.words;
        s.surv_lo = (uint32_t)lo;
        s.surv_hi = (uint32_t)std::min((unsigned long long)n_surv, lo + per_round);
        const size_t nr = s.surv_hi - s.surv_lo;
        // counts, then their exclusive sum (one extra zero count gives the total)
        k_mark_pairs<<<plan.emit_blocks, kSortThreads, 0, st>>>(a, s);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_fill_u32(b.cnt + nr, 0u, 1, st);
        size_t bytes = 0;
        if (e == hipSuccess)
            e = rocprim::exclusive_scan(nullptr, bytes, b.cnt, b.off, 0u, nr + 1, rocprim::plus<uint32_t>(), st);
        if (e == hipSuccess) e = ensure_tmp(b, bytes);
        if (e == hipSuccess)
            e = rocprim::exclusive_scan(b.tmp, bytes, b.cnt, b.off, 0u, nr + 1, rocprim::plus<uint32_t>(), st);
        uint32_t n = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&n, b.off + nr, sizeof(n), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || n == 0) continue;
        if (n > b.cap) return hipErrorInvalidValue;   // cannot happen: a round's pairs are bounded
        if (plan.end_bit <= 31)
            e = sort_and_reduce<uint32_t>(b, a, s, n, plan.end_bit, plan.emit_blocks, st);
        else
            e = sort_and_reduce<unsigned long long>(b, a, s, n, plan.end_bit, plan.emit_blocks, st);
    }
    return e;
}

}  // namespace dbtsdf
