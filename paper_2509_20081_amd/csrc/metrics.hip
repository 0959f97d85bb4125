// Reconstruction-accuracy metrics (Sec. IV-A): nearest-neighbour squared
// distances between two point sets and, from them, accuracy, completeness,
// Chamfer-L1, precision, recall and F-score at a tolerance.
//
// Nearest squared distance. The reference points are bucketed by a uniform
// grid of cubic cells of side h over the bounding box of both sets (count,
// prefix, fill). A query walks the cells around its own in shells of growing
// Chebyshev radius r; once shell r is done, every point not yet visited lies
// beyond the block of visited cells on some axis, so the search ends when the
// best squared distance is at most the squared gap between the query and the
// nearest side of the block (less a rounding margin; at least r h), or when
// the shells cover the whole grid. A query still open after kFineShells
// shells continues on a second grid of cells kCoarse times wider (its nearest
// point is far, and fine shells would be many). Either way the result is the
// minimum over all reference points of
// ((qx - rx)^2 + (qy - ry)^2) + (qz - rz)^2 in fp64 (one operation at a time,
// no contraction), the same value whatever the visiting order.
//
// The queries are bucketed by the same cells and taken in cell order, so
// that the lanes of a wavefront walk the same cells. Sums are taken per
// workgroup and then in workgroup order, so repeated calls give the same bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace dbtsdf {
namespace {

constexpr int kMetThreads = 256;
constexpr int kFineShells = 3;   // fine shells (7^3 cells) before the coarse grid takes over
constexpr double kCoarse = 8.0;  // coarse cell side, in fine cells
constexpr uint32_t kScanItems = 1024;          // prefix: elements per workgroup (4 per thread)
constexpr double kMaxCells = 128.0 * 1024 * 1024;   // cell grid: at most ~2x this many cells
constexpr double kCellsPerRef = 64.0;               // and about this many per reference point (min 2^20)

typedef __attribute__((address_space(1))) const float mgf32;

__device__ __forceinline__ uint32_t ord_of(float f) {   // order-preserving float key
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float float_of(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// box[0..2]: min keys, box[3..5]: max keys, box[6]: count of non-finite coordinates
__global__ __launch_bounds__(kMetThreads) void k_bbox(const float *p, uint64_t n, uint32_t *box) {
    uint32_t lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0u, 0u, 0u}, bad = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const mgf32 *q = (mgf32 *)p + 3 * i;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = q[a];
            if (!isfinite(v)) {
                ++bad;
                continue;
            }
            const uint32_t k = ord_of(v);
            lo[a] = min(lo[a], k);
            hi[a] = max(hi[a], k);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], o, 64));
            hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], o, 64));
        }
        bad += (uint32_t)__shfl_xor((int)bad, o, 64);
    }
    if ((threadIdx.x & 63u) == 0u) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(&box[a], lo[a]);
            atomicMax(&box[3 + a], hi[a]);
        }
        if (bad) atomicAdd(&box[6], bad);
    }
}

struct CellGrid {
    double lo[3];
    double inv_h, h;
    int dims[3];
};

__device__ __forceinline__ void cell_of(const CellGrid &cg, float x, float y, float z, int c[3]) {
    const float p[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = ((double)p[a] - cg.lo[a]) * cg.inv_h;
        int v = (int)floor(u);
        c[a] = min(max(v, 0), cg.dims[a] - 1);
    }
}

__device__ __forceinline__ uint32_t cell_lin(const CellGrid &cg, const int c[3]) {
    return (uint32_t)c[0] + (uint32_t)cg.dims[0] * ((uint32_t)c[1] + (uint32_t)cg.dims[1] * (uint32_t)c[2]);
}

__global__ __launch_bounds__(kMetThreads) void k_cell_count(CellGrid cg, const float *p, uint64_t n, uint32_t *cnt,
                                                             uint32_t *cell) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const mgf32 *q = (mgf32 *)p + 3 * i;
    int c[3];
    cell_of(cg, q[0], q[1], q[2], c);
    const uint32_t l = cell_lin(cg, c);
    cell[i] = l;
    atomicAdd(&cnt[l], 1u);
}

// exclusive prefix of v[0..n) in place, in three passes (per-workgroup sums,
// their prefix by one workgroup, the add-back)
__device__ uint32_t block_scan_excl(uint32_t x, uint32_t *s, uint32_t &total) {
    const uint32_t l = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
        if ((int)l >= o) inc += y;
    }
    if (l == 63u) s[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t k = 0; k < blockDim.x / 64u; ++k) {
        if (k < w) before += s[k];
        tot += s[k];
    }
    __syncthreads();
    total = tot;
    return before + inc - x;
}

__global__ __launch_bounds__(kMetThreads) void k_scan_local(uint32_t *v, uint64_t n, uint32_t *sums) {
    __shared__ uint32_t s[kMetThreads / 64];
    const uint64_t base = blockIdx.x * (uint64_t)kScanItems + 4u * threadIdx.x;
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = base + j < n ? v[base + j] : 0u;
    const uint32_t t = x[0] + x[1] + x[2] + x[3];
    uint32_t total;
    uint32_t run = block_scan_excl(t, s, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) v[base + j] = run;
        run += x[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kMetThreads) void k_scan_sums(uint32_t *sums, uint32_t n) {
    __shared__ uint32_t s[kMetThreads / 64];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < n; b += kMetThreads) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t x = i < n ? sums[i] : 0u;
        uint32_t total;
        const uint32_t e = block_scan_excl(x, s, total);
        if (i < n) sums[i] = carry + e;
        carry += total;
    }
}

__global__ __launch_bounds__(kMetThreads) void k_scan_add(uint32_t *v, uint64_t n, const uint32_t *sums) {
    const uint64_t base = blockIdx.x * (uint64_t)kScanItems + 4u * threadIdx.x;
    const uint32_t add = sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j < n) v[base + j] += add;
}

__global__ __launch_bounds__(kMetThreads) void k_cell_fill(const float *p, uint64_t n, const uint32_t *cell,
                                                            const uint32_t *start, uint32_t *cursor, float4 *sorted) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const mgf32 *q = (mgf32 *)p + 3 * i;
    const uint32_t c = cell[i];
    const uint32_t pos = start[c] + atomicAdd(&cursor[c], 1u);
    sorted[pos] = make_float4(q[0], q[1], q[2], 0.0f);
}

// the queries' indices in cell order (lanes of a wavefront then walk the same
// cells and read the same reference points)
__global__ __launch_bounds__(kMetThreads) void k_query_fill(uint64_t n, const uint32_t *cell, const uint32_t *start,
                                                             uint32_t *cursor, uint32_t *perm) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cell[i];
    perm[start[c] + atomicAdd(&cursor[c], 1u)] = (uint32_t)i;
}

__device__ __forceinline__ double sq_dist(double qx, double qy, double qz, float4 r) {
    const double dx = qx - (double)r.x, dy = qy - (double)r.y, dz = qz - (double)r.z;
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// Shells 0 .. r_max of cells around the query's cell c (u: the query in cell
// units) into best; true once nothing unvisited can be closer.
__device__ bool shell_search(const CellGrid &cg, const int c[3], const double u[3], const uint32_t *start,
                             const float4 *sorted, double qx, double qy, double qz, int r_max, double &best) {
    int r_all = 0;   // shells that cover the whole grid from this cell
#pragma unroll
    for (int a = 0; a < 3; ++a) r_all = max(r_all, max(c[a], cg.dims[a] - 1 - c[a]));
    for (int r = 0; r <= min(r_all, r_max); ++r) {
        const int z0 = max(c[2] - r, 0), z1 = min(c[2] + r, cg.dims[2] - 1);
        const int y0 = max(c[1] - r, 0), y1 = min(c[1] + r, cg.dims[1] - 1);
        for (int z = z0; z <= z1; ++z) {
            for (int y = y0; y <= y1; ++y) {
                const bool face = abs(z - c[2]) == r || abs(y - c[1]) == r;
                // on the shell's z or y faces the whole x run; inside them only x = c -+ r
                const int step = face ? 1 : 2 * r;
                for (int x = c[0] - r; x <= c[0] + r; x += max(step, 1)) {
                    if (x < 0 || x >= cg.dims[0]) continue;
                    const uint32_t l = (uint32_t)x + (uint32_t)cg.dims[0] * ((uint32_t)y + (uint32_t)cg.dims[1] * (uint32_t)z);
                    const uint32_t e = start[l + 1];
                    for (uint32_t k = start[l]; k < e; ++k) best = fmin(best, sq_dist(qx, qy, qz, sorted[k]));
                }
            }
        }
        if (r == r_all) return true;
        // after shell r every unvisited point lies in a cell outside the block
        // [c - r, c + r] on some axis, so at least the query's gap to that
        // side of the block away (less a margin for the rounding of the cell
        // indices); sides at the grid's edge have nothing beyond them
        double gap = INFINITY;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c[a] - r > 0) gap = fmin(gap, u[a] - (double)(c[a] - r));
            if (c[a] + r + 1 < cg.dims[a]) gap = fmin(gap, (double)(c[a] + r + 1) - u[a]);
        }
        const double bound = (gap - 1e-9) * cg.h;
        if (bound > 0.0 && best <= bound * bound) return true;
    }
    return false;
}

// One query per lane, in cell order: a few shells of the fine grid, then, for
// a query still open (its nearest point is far), shells of the coarse grid
// (cells kCoarse times wider) until nothing unvisited can be closer or the
// whole grid is covered.
__global__ __launch_bounds__(kMetThreads) void k_nearest(CellGrid cg, CellGrid cg2, const float *qp, uint64_t nq,
                                                          const uint32_t *perm, const uint32_t *start,
                                                          const float4 *sorted, const uint32_t *start2,
                                                          const float4 *sorted2, double *d2_out) {
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= nq) return;
    const uint64_t i = perm[t];
    const mgf32 *q = (mgf32 *)qp + 3 * i;
    const float fx = q[0], fy = q[1], fz = q[2];
    const double qx = fx, qy = fy, qz = fz;
    const float fq[3] = {fx, fy, fz};
    double best = INFINITY;
    int c[3];
    double u[3];   // the query in cell units (as cell_of computes it)
    cell_of(cg, fx, fy, fz, c);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = ((double)fq[a] - cg.lo[a]) * cg.inv_h;
    if (!shell_search(cg, c, u, start, sorted, qx, qy, qz, kFineShells, best)) {
        cell_of(cg2, fx, fy, fz, c);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = ((double)fq[a] - cg2.lo[a]) * cg2.inv_h;
        (void)shell_search(cg2, c, u, start2, sorted2, qx, qy, qz, 1 << 20, best);   // ends by covering the grid
    }
    d2_out[i] = best;
}

// per workgroup: sum of sqrt(d2) and count of d2 < t2
__global__ __launch_bounds__(kMetThreads) void k_reduce(const double *d2, uint64_t n, double t2, double *psum,
                                                         unsigned long long *pcnt) {
    __shared__ double ss[kMetThreads];
    __shared__ unsigned long long sc[kMetThreads];
    double s = 0.0;
    unsigned long long cnt = 0;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = blockIdx.x * per, e = min(n, b + per);
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const double v = d2[i];
        s += sqrt(v);
        cnt += v < t2 ? 1ull : 0ull;
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = cnt;
    __syncthreads();
    for (int o = kMetThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            ss[threadIdx.x] += ss[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = ss[0];
        pcnt[blockIdx.x] = sc[0];
    }
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
    template <class T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t enter(int device) {
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) {
            e = hipSetDevice(device);
            changed = e == hipSuccess;
        }
        return e;
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

// Nearest squared distances of every query to the reference set, into d2
// (device, n_query doubles). cell_hint: the smallest cell side to use.
dbtsdf_status nearest_sq(const float *qp, uint64_t nq, const float *rp, uint64_t nr, double *d2, double cell_hint,
                         hipStream_t st) {
    if (nq == 0) return DBTSDF_OK;
    DevBuf box;
    hipError_t e = box.alloc(8 * sizeof(uint32_t));
    if (e != hipSuccess) return check_hip(e, "allocating the bounding box");
    uint32_t init[8] = {~0u, ~0u, ~0u, 0u, 0u, 0u, 0u, 0u};
    e = hipMemcpyAsync(box.p, init, sizeof(init), hipMemcpyHostToDevice, st);
    auto blocks = [](uint64_t n) { return (unsigned)std::min<uint64_t>(std::max<uint64_t>((n + kMetThreads - 1) / kMetThreads, 1), 4096); };
    if (e == hipSuccess) {
        k_bbox<<<blocks(nq), kMetThreads, 0, st>>>(qp, nq, box.as<uint32_t>());
        k_bbox<<<blocks(nr), kMetThreads, 0, st>>>(rp, nr, box.as<uint32_t>());
        e = hipGetLastError();
    }
    uint32_t hb[8] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(hb, box.p, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(e, "bounding the point sets");
    if (hb[6]) {
        set_error("point coordinates must be finite");
        return DBTSDF_ERR_INVALID_ARG;
    }
    CellGrid cg{};
    double ext[3], vol = 1.0, emax = 0.0;
    for (int a = 0; a < 3; ++a) {
        cg.lo[a] = (double)float_of(hb[a]);
        ext[a] = (double)float_of(hb[3 + a]) - cg.lo[a];
        emax = std::max(emax, ext[a]);
        vol *= std::max(ext[a], 1e-30);
    }
    const double target = std::min(kMaxCells, std::max(1048576.0, kCellsPerRef * (double)nr));
    double h = std::max({cell_hint, std::cbrt(vol / target), emax / 4096.0, 1e-6});
    for (;;) {
        double cells = 1.0;
        for (int a = 0; a < 3; ++a) cells *= std::floor(ext[a] / h) + 1.0;
        if (cells <= 2.0 * target) break;
        h *= 1.25;
    }
    cg.h = h;
    cg.inv_h = 1.0 / h;
    uint64_t n_cells = 1;
    for (int a = 0; a < 3; ++a) {
        cg.dims[a] = (int)(std::floor(ext[a] / h) + 1.0);
        n_cells *= (uint64_t)cg.dims[a];
    }
    if (nr > 0xFFFFFFF0ull || nq > 0xFFFFFFF0ull) {
        set_error("at most 2^32 - 16 points per set");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    CellGrid cg2 = cg;
    cg2.h = kCoarse * h;
    cg2.inv_h = 1.0 / cg2.h;
    uint64_t n_cells2 = 1;
    for (int a = 0; a < 3; ++a) {
        cg2.dims[a] = (int)(std::floor(ext[a] / cg2.h) + 1.0);
        n_cells2 *= (uint64_t)cg2.dims[a];
    }
    DevBuf start, qstart, cursor, cell, qcell, perm, sorted, sums, start2, sorted2;
    const uint64_t n_start = n_cells + 1;
    const uint64_t n_sums = (n_start + kScanItems - 1) / kScanItems;
    e = start.alloc(n_start * 4);
    if (e == hipSuccess) e = qstart.alloc(n_start * 4);
    if (e == hipSuccess) e = cursor.alloc(n_cells * 4);
    if (e == hipSuccess) e = cell.alloc(nr * 4);
    if (e == hipSuccess) e = qcell.alloc(nq * 4);
    if (e == hipSuccess) e = perm.alloc(nq * 4);
    if (e == hipSuccess) e = sorted.alloc(nr * sizeof(float4));
    if (e == hipSuccess) e = sums.alloc(n_sums * 4);
    if (e == hipSuccess) e = start2.alloc((n_cells2 + 1) * 4);
    if (e == hipSuccess) e = sorted2.alloc(nr * sizeof(float4));
    if (e != hipSuccess) return check_hip(e, "allocating the cell grid");
    // counts of the points of p per cell of g into cnt (n_c + 1 words), then their exclusive prefix
    auto bucket = [&](const CellGrid &g, uint64_t n_c, const float *p, uint64_t n, uint32_t *cnt, uint32_t *cl) {
        const uint64_t ns = (n_c + 1 + kScanItems - 1) / kScanItems;
        hipError_t r = launch_fill_u32(cnt, 0u, n_c + 1, st);
        if (r == hipSuccess) r = launch_fill_u32(cursor.as<uint32_t>(), 0u, n_c, st);
        if (r != hipSuccess) return r;
        k_cell_count<<<(unsigned)((n + kMetThreads - 1) / kMetThreads), kMetThreads, 0, st>>>(g, p, n, cnt, cl);
        k_scan_local<<<(unsigned)ns, kMetThreads, 0, st>>>(cnt, n_c + 1, sums.as<uint32_t>());
        k_scan_sums<<<1, kMetThreads, 0, st>>>(sums.as<uint32_t>(), (uint32_t)ns);
        k_scan_add<<<(unsigned)ns, kMetThreads, 0, st>>>(cnt, n_c + 1, sums.as<uint32_t>());
        return hipGetLastError();
    };
    const unsigned gr = (unsigned)((nr + kMetThreads - 1) / kMetThreads);
    const unsigned gq = (unsigned)((nq + kMetThreads - 1) / kMetThreads);
    e = bucket(cg, n_cells, rp, nr, start.as<uint32_t>(), cell.as<uint32_t>());
    if (e == hipSuccess) {
        k_cell_fill<<<gr, kMetThreads, 0, st>>>(rp, nr, cell.as<uint32_t>(), start.as<uint32_t>(),
                                                cursor.as<uint32_t>(), sorted.as<float4>());
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = bucket(cg2, n_cells2, rp, nr, start2.as<uint32_t>(), cell.as<uint32_t>());
    if (e == hipSuccess) {
        k_cell_fill<<<gr, kMetThreads, 0, st>>>(rp, nr, cell.as<uint32_t>(), start2.as<uint32_t>(),
                                                cursor.as<uint32_t>(), sorted2.as<float4>());
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = bucket(cg, n_cells, qp, nq, qstart.as<uint32_t>(), qcell.as<uint32_t>());
    if (e == hipSuccess) {
        k_query_fill<<<gq, kMetThreads, 0, st>>>(nq, qcell.as<uint32_t>(), qstart.as<uint32_t>(),
                                                 cursor.as<uint32_t>(), perm.as<uint32_t>());
        k_nearest<<<gq, kMetThreads, 0, st>>>(cg, cg2, qp, nq, perm.as<uint32_t>(), start.as<uint32_t>(),
                                              sorted.as<float4>(), start2.as<uint32_t>(), sorted2.as<float4>(), d2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return check_hip(e, "nearest-neighbour search");
}

dbtsdf_status reduce(const double *d2, uint64_t n, double t2, double &sum, uint64_t &within, hipStream_t st) {
    const unsigned nb = (unsigned)std::min<uint64_t>(std::max<uint64_t>((n + 4095) / 4096, 1), 1024);
    DevBuf ps, pc;
    hipError_t e = ps.alloc(nb * sizeof(double));
    if (e == hipSuccess) e = pc.alloc(nb * sizeof(unsigned long long));
    if (e != hipSuccess) return check_hip(e, "allocating the reduction");
    k_reduce<<<nb, kMetThreads, 0, st>>>(d2, n, t2, ps.as<double>(), pc.as<unsigned long long>());
    std::vector<double> hs(nb);
    std::vector<unsigned long long> hc(nb);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), ps.p, nb * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), pc.p, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(e, "reducing the distances");
    sum = 0.0;
    within = 0;
    for (unsigned b = 0; b < nb; ++b) {
        sum += hs[b];
        within += hc[b];
    }
    return DBTSDF_OK;
}

}  // namespace
}  // namespace dbtsdf

using namespace dbtsdf;

extern "C" dbtsdf_status dbtsdf_nearest_sq(int device, const float *query_dev, uint64_t n_query, const float *ref_dev,
                                           uint64_t n_ref, double *d2_dev) {
    if ((n_query && (!query_dev || !d2_dev)) || (n_ref && !ref_dev)) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (n_ref == 0 && n_query) {
        set_error("empty reference set");
        return DBTSDF_ERR_INVALID_ARG;
    }
    DeviceGuard dg;
    hipError_t e = dg.enter(device);
    if (e != hipSuccess) return check_hip(e, "selecting the device");
    return nearest_sq(query_dev, n_query, ref_dev, n_ref, d2_dev, 0.0, nullptr);
}

extern "C" dbtsdf_status dbtsdf_surface_metrics(int device, const float *pred_dev, uint64_t n_pred, const float *gt_dev,
                                                uint64_t n_gt, double tolerance, dbtsdf_metrics *out) {
    if (!pred_dev || !gt_dev || !out) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (n_pred == 0 || n_gt == 0) {
        set_error("both point sets must be non-empty");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (!std::isfinite(tolerance) || tolerance < 0.0) {
        set_error("tolerance must be finite and >= 0");
        return DBTSDF_ERR_INVALID_ARG;
    }
    DeviceGuard dg;
    hipError_t e = dg.enter(device);
    if (e != hipSuccess) return check_hip(e, "selecting the device");
    DevBuf dp, dgt;
    e = dp.alloc(n_pred * sizeof(double));
    if (e == hipSuccess) e = dgt.alloc(n_gt * sizeof(double));
    if (e != hipSuccess) return check_hip(e, "allocating the distances");
    dbtsdf_status s = nearest_sq(pred_dev, n_pred, gt_dev, n_gt, dp.as<double>(), 0.0, nullptr);
    if (s == DBTSDF_OK) s = nearest_sq(gt_dev, n_gt, pred_dev, n_pred, dgt.as<double>(), 0.0, nullptr);
    if (s != DBTSDF_OK) return s;
    const double t2 = tolerance * tolerance;
    double sp = 0.0, sg = 0.0;
    uint64_t wp = 0, wg = 0;
    s = reduce(dp.as<double>(), n_pred, t2, sp, wp, nullptr);
    if (s == DBTSDF_OK) s = reduce(dgt.as<double>(), n_gt, t2, sg, wg, nullptr);
    if (s != DBTSDF_OK) return s;
    dbtsdf_metrics m{};
    m.accuracy = sp / (double)n_pred;
    m.completeness = sg / (double)n_gt;
    m.chamfer_l1 = 0.5 * (m.accuracy + m.completeness);
    m.precision = (double)wp / (double)n_pred;
    m.recall = (double)wg / (double)n_gt;
    m.fscore = m.precision + m.recall == 0.0 ? 0.0 : 2.0 * m.precision * m.recall / (m.precision + m.recall);
    m.n_pred = n_pred;
    m.n_gt = n_gt;
    m.n_pred_within = wp;
    m.n_gt_within = wg;
    *out = m;
    return DBTSDF_OK;
}
