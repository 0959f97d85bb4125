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
//   1. k_emit_pairs: one wavefront per survivor writes a (key, contribution)
//      pair for every window word whose mask would lose bits (read first, as
//      eq. 4's skipped writes) and every shadow cell whose counter is below
//      H_max; a wavefront reserves the room of up to 32 passes of pairs with
//      one atomic;
//   2. a radix sort of the pairs by key (rocPRIM, over the key bits in use);
//   3. k_reduce_pairs: a wavefront segmented reduction (a 64-lane scan of AND
//      and count that restarts at each new key) over a chunk of sorted pairs,
//      the last lane of each run writing the voxel's words with plain stores:
//      each voxel is one run, so no word is written twice.
// A read-first filter stays exact across rounds: planes only lose mask bits
// and gain hits, so a contribution that changes nothing now changes nothing
// later. Larger calls run in rounds of survivors whose pairs fit the buffers.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

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

constexpr int kGroup = 32;       // passes whose need bits a lane keeps before reserving room
constexpr int kLoadBatch = 8;    // window loads in flight per lane
constexpr uint32_t kSegChunk = 512;  // sorted pairs per wavefront of the reduction

// Reserve room for the pairs flagged in `bits` (bit u: pass u of the group)
// and return the first slot; every lane gets the same value.
__device__ __forceinline__ unsigned long long reserve(unsigned long long *count, uint32_t bits, uint32_t n_pass) {
    uint32_t tot = 0;
    for (uint32_t u = 0; u < n_pass; ++u) tot += (uint32_t)__popcll(__ballot((bits >> u) & 1u));
    unsigned long long base = 0;
    if (tot) {
        if (lane_id() == 0) base = atomicAdd(count, (unsigned long long)tot);
        base = wave_uniform64(__shfl(base, 0, 64));
    }
    return base;
}

__global__ __launch_bounds__(kSortThreads) void k_emit_pairs(PipeArgs a, SortArgs s) {
    const DevTables &t = a.tab;
    const int K = t.K, R = t.R;
    const bool l1 = t.metric == DBTSDF_DIST_L1;
    const uint32_t l = lane_id();
    const unsigned long long below = l ? ((1ull << l) - 1ull) : 0ull;
    const uint32_t wx = (uint32_t)K, rpi = 64u / wx, xi = l % wx, ri = l / wx;
    const bool lane_on = ri < rpi;
    const uint32_t rows = (uint32_t)(K * K);
    const uint32_t n_pass = (rows + rpi - 1u) / rpi;
    const uint32_t mag = ((1u << 20) + wx - 1u) / wx;
    const int ox = (int)xi - R;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t e = s.surv_lo + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < s.surv_hi; e += waves) {
        const uint4 r = a.surv_rec[e];
        const uint32_t gi = r.w >> 16;
        const DevGrid &g = a.grids[gi];
        const uint32_t nx = __builtin_amdgcn_readfirstlane(g.nx), ny = __builtin_amdgcn_readfirstlane(g.ny);
        const uint32_t hmax = __builtin_amdgcn_readfirstlane(g.hmax);
        const uint32_t *mask = reinterpret_cast<const uint32_t *>(wave_uniform64(reinterpret_cast<uint64_t>(g.mask)));
        const uint32_t *packed =
            reinterpret_cast<const uint32_t *>(wave_uniform64(reinterpret_cast<uint64_t>(g.packed)));
        const uint64_t corner = (uint64_t)(r.x - (uint32_t)R) +
                                (uint64_t)nx * ((uint64_t)(r.y - (uint32_t)R) + (uint64_t)ny * (uint64_t)(r.z - (uint32_t)R));
        const unsigned long long kbase = ((unsigned long long)gi << s.shift) + corner;
        // eq. 4 window, skipped for a return whose voxel an earlier call integrated
        // (the window's words already hold these masks)
        if (!(r.w & kRecRevisit)) {
            for (uint32_t p0 = 0; p0 < n_pass; p0 += kGroup) {
                const uint32_t np = min((uint32_t)kGroup, n_pass - p0);
                uint32_t bits = 0;
                for (uint32_t u0 = 0; u0 < np; u0 += kLoadBatch) {
                    uint32_t old[kLoadBatch], m[kLoadBatch];
                    bool on[kLoadBatch];
#pragma unroll
                    for (int u = 0; u < kLoadBatch; ++u) {
                        const uint32_t rr = (p0 + u0 + (uint32_t)u) * rpi + ri;
                        on[u] = lane_on && u0 + (uint32_t)u < np && rr < rows;
                        const uint32_t rz = (rr * mag) >> 20, ry = rr - rz * wx;
                        const int oy = (int)ry - R, oz = (int)rz - R;
                        const uint32_t q =
                            l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
                        m[u] = on[u] ? t.mask_by_q[q] : 0xFFFFFFFFu;
                        old[u] = on[u] ? mask[corner + xi + (uint64_t)nx * (ry + (uint64_t)ny * rz)] : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < kLoadBatch; ++u)
                        if (on[u] && (old[u] & m[u]) != old[u]) bits |= 1u << (u0 + (uint32_t)u);
                }
                unsigned long long slot = reserve(s.count, bits, np);
                for (uint32_t u = 0; u < np; ++u) {
                    const bool need = (bits >> u) & 1u;
                    const unsigned long long bal = __ballot(need);
                    if (need) {
                        const uint32_t rr = (p0 + u) * rpi + ri;
                        const uint32_t rz = (rr * mag) >> 20, ry = rr - rz * wx;
                        const int oy = (int)ry - R, oz = (int)rz - R;
                        const uint32_t q =
                            l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
                        const unsigned long long at = slot + (unsigned long long)__popcll(bal & below);
                        s.keys[at] = kbase + xi + (uint64_t)nx * (ry + (uint64_t)ny * rz);
                        s.vals[at] = t.mask_by_q[q];
                    }
                    slot += (unsigned long long)__popcll(bal);
                }
            }
        }
        // eqs. 5-6: one hit per shadow cell whose counter can still grow
        const uint32_t bin = r.w & kRowBinMask;
        const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
        const uint32_t n_sp = (s1 - s0 + 63u) / 64u;
        for (uint32_t p0 = 0; p0 < n_sp; p0 += kGroup) {
            const uint32_t np = min((uint32_t)kGroup, n_sp - p0);
            uint32_t bits = 0;
            for (uint32_t u = 0; u < np; ++u) {
                const uint32_t j = s0 + (p0 + u) * 64u + l;
                if (j < s1) {
                    const uint32_t pk = t.sh_off[j];
                    const uint64_t so = (uint64_t)(pk & 255u) +
                                        (uint64_t)nx * ((uint64_t)((pk >> 8) & 255u) + (uint64_t)ny * ((pk >> 16) & 255u));
                    if ((packed[corner + so] & 0xFFFFu) < hmax) bits |= 1u << u;
                }
            }
            unsigned long long slot = reserve(s.count, bits, np);
            for (uint32_t u = 0; u < np; ++u) {
                const bool need = (bits >> u) & 1u;
                const unsigned long long bal = __ballot(need);
                if (need) {
                    const uint32_t pk = t.sh_off[s0 + (p0 + u) * 64u + l];
                    const uint64_t so = (uint64_t)(pk & 255u) +
                                        (uint64_t)nx * ((uint64_t)((pk >> 8) & 255u) + (uint64_t)ny * ((pk >> 16) & 255u));
                    const unsigned long long at = slot + (unsigned long long)__popcll(bal & below);
                    s.keys[at] = kbase + so;
                    s.vals[at] = kHitPair;
                }
                slot += (unsigned long long)__popcll(bal);
            }
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

// Wavefront segmented reduction of sorted pairs. Wavefront w owns the runs of
// equal keys that start in [w C, (w + 1) C) (C = kSegChunk), the last of them
// followed past the chunk's end; runs that started before are another's.
__global__ __launch_bounds__(kSortThreads) void k_reduce_pairs(const DevGrid *grids, const unsigned long long *keys,
                                                               const uint32_t *vals, unsigned long long n,
                                                               uint32_t shift) {
    const uint32_t l = lane_id();
    const unsigned long long w = (unsigned long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const unsigned long long c0 = w * kSegChunk;
    if (c0 >= n) return;
    const unsigned long long c1 = min(c0 + kSegChunk, n);
    // first run head at or after c0
    unsigned long long s = c1;
    for (unsigned long long p0 = c0; p0 < c1; p0 += 64) {
        const unsigned long long p = p0 + l;
        const bool hd = p < c1 && (p == 0 || keys[p] != keys[p - 1]);
        const unsigned long long bal = __ballot(hd);
        if (bal) {
            s = p0 + (unsigned long long)__builtin_ctzll(bal);
            break;
        }
    }
    if (s >= c1) return;
    // end of the run open at c1: the first head at or after c1 (or n)
    unsigned long long e = n;
    for (unsigned long long p0 = c1; p0 < n; p0 += 64) {
        const unsigned long long p = p0 + l;
        const bool hd = p >= n || keys[p] != keys[p - 1];
        const unsigned long long bal = __ballot(hd);
        if (bal) {
            e = p0 + (unsigned long long)__builtin_ctzll(bal);
            break;
        }
    }
    // the run open at the start of a window: its key, AND and count so far
    unsigned long long ck = ~0ull;
    uint32_t cand = 0xFFFFFFFFu, ccnt = 0;
    for (unsigned long long w0 = s; w0 < e; w0 += 64) {
        const unsigned long long p = w0 + l;
        const bool in = p < e;
        const unsigned long long k = in ? keys[p] : ~0ull;   // keys use fewer than 64 bits
        const uint32_t v = in ? vals[p] : 0xFFFFFFFFu;
        unsigned long long kp = shfl_up64(k, 1);
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
        unsigned long long kn = shfl_down64(k, 1);
        if (l == 63) kn = p + 1 < e ? keys[p + 1] : ~0ull;
        if (in && kn != k) apply_voxel(grids, k, shift, am, cn);
        ck = wave_uniform64(__shfl(k, 63, 64));
        cand = __builtin_amdgcn_readfirstlane(__shfl(am, 63, 64));
        ccnt = __builtin_amdgcn_readfirstlane(__shfl(cn, 63, 64));
    }
}

hipError_t ensure_sort_buffers(SortBuffers &b, unsigned long long pairs) {
    if (pairs <= b.cap && b.count) return hipSuccess;
    const unsigned long long cap = std::max(pairs, std::min(b.cap * 2ull, kSortMaxPairs));
    free_sort_buffers(b);
    hipError_t e = hipMalloc((void **)&b.count, sizeof(unsigned long long));
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc((void **)&b.keys[i], cap * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMalloc((void **)&b.vals[i], cap * sizeof(uint32_t));
    }
    if (e != hipSuccess) {
        free_sort_buffers(b);
        return e;
    }
    b.cap = cap;
    return hipSuccess;
}

}  // namespace

const void *sort_emit_kernel() { return reinterpret_cast<const void *>(k_emit_pairs); }

void free_sort_buffers(SortBuffers &b) {
    void *p[] = {b.keys[0], b.keys[1], b.vals[0], b.vals[1], b.count, b.tmp};
    for (void *x : p)
        if (x) (void)hipFree(x);
    b = SortBuffers{};
}

hipError_t sort_apply(Workspace &ws, const PipeArgs &a, const SortPlan &plan, hipStream_t st) {
    SortBuffers &b = ws.sorter;
    uint32_t n_surv = 0;
    hipError_t e = hipMemcpyAsync(&n_surv, &a.ctrl->n_survivors, sizeof(n_surv), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess || n_surv == 0) return e;
    unsigned long long per_round = std::max(1ull, kSortMaxPairs / plan.pairs_per_point);
    if (plan.round_survivors) per_round = std::min(per_round, (unsigned long long)plan.round_survivors);
    const unsigned long long need = std::min((unsigned long long)n_surv, per_round) * plan.pairs_per_point;
    e = ensure_sort_buffers(b, need);
    for (unsigned long long lo = 0; e == hipSuccess && lo < n_surv; lo += per_round) {
        SortArgs s{};
        s.keys = b.keys[0];
        s.vals = b.vals[0];
        s.count = b.count;
        s.shift = plan.shift;
        s.surv_lo = (uint32_t)lo;
        s.surv_hi = (uint32_t)std::min((unsigned long long)n_surv, lo + per_round);
        e = launch_fill_u64(b.count, 0ull, 1, st);
        if (e != hipSuccess) break;
        k_emit_pairs<<<plan.emit_blocks, kSortThreads, 0, st>>>(a, s);
        unsigned long long n = 0;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&n, b.count, sizeof(n), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || n == 0) continue;
        if (n > b.cap) return hipErrorInvalidValue;   // cannot happen: a round's pairs are bounded
        rocprim::double_buffer<unsigned long long> kb(b.keys[0], b.keys[1]);
        rocprim::double_buffer<uint32_t> vb(b.vals[0], b.vals[1]);
        size_t bytes = 0;
        e = rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)n, 0u, plan.end_bit, st);
        if (e == hipSuccess && bytes > b.tmp_bytes) {
            if (b.tmp) (void)hipFree(b.tmp);
            b.tmp = nullptr;
            b.tmp_bytes = 0;
            e = hipMalloc(&b.tmp, bytes);
            if (e == hipSuccess) b.tmp_bytes = bytes;
        }
        if (e == hipSuccess) e = rocprim::radix_sort_pairs(b.tmp, bytes, kb, vb, (size_t)n, 0u, plan.end_bit, st);
        if (e != hipSuccess) break;
        const unsigned long long waves = (n + kSegChunk - 1) / kSegChunk;
        const unsigned long long blocks = (waves + (kSortThreads / 64) - 1) / (kSortThreads / 64);
        k_reduce_pairs<<<(uint32_t)blocks, kSortThreads, 0, st>>>(a.grids, kb.current(), vb.current(), n, plan.shift);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace dbtsdf
