/*
 * dbtsdf.h - C ABI of an MI355X (gfx950) implementation of DB-TSDF scan
 * integration: "DB-TSDF: Directional Bitmask-based Truncated Signed Distance
 * Fields for Efficient Volumetric Mapping" (Maese, Merino, Caballero,
 * arXiv 2509.20081).
 *
 * The library keeps dense voxel grids in GPU memory and fuses LiDAR scans
 * into them (Sec. III-C): every return is transformed into the map frame with
 * the scan pose, discarded if its K^3 neighbourhood would leave the map,
 * assigned a direction bin (Sec. III-B, eq. 2), and its kernel is applied:
 * a bitwise AND of the eq. 3 distance masks over the K^3 neighbourhood
 * (eq. 4) and, inside the bin's hemispherical shadow, a saturating hit
 * counter (eq. 5) whose threshold crossing clears the sign bit (eq. 6).
 * Within one scan only the first return per voxel is integrated (Sec. IV-B).
 *
 * Data layout (Sec. III-A, eq. 1: 8 bytes per voxel). A grid is two planes of
 * Nx*Ny*Nz uint32 words, x fastest (linear index x + Nx*(y + Ny*z)):
 *   mask   - the 32-bit distance mask; its popcount is the truncated distance
 *            in voxels; always of the form 2^n - 1 (all ones = never touched);
 *   packed - hit counter h in bits 0-15, bits 16-30 zero, sign in bit 31
 *            (1 = free, 0 = occupied).
 * Initial state: mask 0xFFFFFFFF, packed 0x80000000 (Sec. III-A).
 *
 * Conventions shared by every entry point:
 *   - No call throws; every failure is a dbtsdf_status.
 *   - Arguments are validated before anything is enqueued; on error the grid
 *     is unchanged.
 *   - Device work is enqueued on the grid's HIP stream and is asynchronous
 *     unless an entry point says otherwise (the exports, and integration
 *     with DBTSDF_STRATEGY_SORT, wait for the stream); results (grid
 *     contents, statistics) are valid after dbtsdf_sync().
 *   - A grid must not be used from two threads at once; different grids may.
 *   - Host pointers are only read during the call unless stated otherwise.
 */
#ifndef DBTSDF_H
#define DBTSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DBTSDF_OK = 0,
    DBTSDF_ERR_INVALID_ARG = 1,   /* a parameter or pointer failed validation */
    DBTSDF_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed, or a memory budget refused it */
    DBTSDF_ERR_DEVICE = 3,        /* a HIP call failed; the grid is poisoned */
    DBTSDF_ERR_OUT_OF_RANGE = 4,  /* a read box or size exceeds the grid / a fixed limit */
    DBTSDF_ERR_POISONED = 5,      /* the grid saw a device error earlier and refuses work */
    DBTSDF_ERR_BUSY = 6           /* a server queue is full (try again later) */
} dbtsdf_status;

/* Direction binning (Sec. III-B). */
typedef enum {
    DBTSDF_BIN_AZEL = 0,   /* eq. 2: bins_az x bins_el azimuth/elevation bins (paper: 40 x 40) */
    DBTSDF_BIN_CUBE26 = 1  /* 26 lattice directions: 8 azimuths x 3 elevations + 2 poles */
} dbtsdf_binning;

/* Shape of the shadow (occupied evidence) behind the contact voxel. */
typedef enum {
    DBTSDF_SHADOW_HEMISPHERE = 0,  /* Sec. III-B: {o : o.o <= r_s^2, o.u_b >= 0} (default) */
    DBTSDF_SHADOW_CONE = 1         /* the conical alternative of Sec. IV-A: o.u_b >= |o| cos(alpha) */
} dbtsdf_shadow_model;

/* Distance measured by the eq. 3 mask. */
typedef enum {
    DBTSDF_DIST_L2 = 0,    /* eq. 3: n = ceil(sqrt(x^2 + y^2 + z^2)) (default) */
    DBTSDF_DIST_L1 = 1     /* the L1 distance named in Sec. III-A: n = |x| + |y| + |z| */
} dbtsdf_metric;

/*
 * Kernel-set parameters (Sec. III-B).
 *   kernel_size  K, odd, 3..37 (paper: 21). With DBTSDF_DIST_L1, K <= 21 so
 *                that every mask fits 32 bits.
 *   binning      dbtsdf_binning.
 *   bins_az/el   AZEL only: bins_az even and >= 2, bins_el >= 1, product <= 65536.
 *   shadow_r2    r_s^2 in voxel^2: the shadow is {o : o.o <= r_s^2, o.u_b >= 0}
 *                (contact voxel and planar face included); negative = no shadow
 *                (the unsigned D-LIO distance field).
 *   metric       dbtsdf_metric.
 *   shadow_model dbtsdf_shadow_model (0, the hemisphere, when zero-initialised).
 *   cone_deg     DBTSDF_SHADOW_CONE only: half-angle alpha in degrees, in (0, 90].
 *                The cone is {o : o.o <= r_s^2, o = 0 or o.u_b >= |o| cos(alpha)}
 *                with cos(alpha) in fp64, taken as 0 below 1e-12 (90 degrees is
 *                the hemisphere); cube bins test (o.s)^2 >= (o.o)(s.s) cos^2(alpha)
 *                and o.s >= 0 on their integer direction s, AZEL bins
 *                o.u_b >= |o| cos(alpha) - 1e-9 in fp64 (the paper gives no
 *                aperture).
 */
typedef struct {
    uint32_t kernel_size;
    uint32_t binning;
    uint32_t bins_az;
    uint32_t bins_el;
    int32_t shadow_r2;
    uint32_t metric;
    uint32_t shadow_model;
    float cone_deg;
} dbtsdf_kernel_params;

/* Grid flags. */
#define DBTSDF_DEDUP_FIRST 0x1u    /* integrate only the first return per voxel in a scan (Sec. IV-B) */
#define DBTSDF_COUNT_TRAFFIC 0x2u  /* also count unique/changed mask words and unique shadow words */

/*
 * Grid parameters (Sec. III-A).
 *   dims           Nx, Ny, Nz; each >= K and <= 2^20; Nx*Ny*Nz*8 bytes of HBM (eq. 1).
 *   voxel_size     metres, finite and > 0.
 *   origin         map-frame coordinate of the min corner of voxel (0,0,0), finite.
 *   hit_threshold  T of eq. 6, 0..65535 (T = 0 or T > hit_max: the sign never flips).
 *   hit_max        H_max of eq. 5, 1..65535 (the paper's 8-bit counter: 255).
 *   flags          DBTSDF_DEDUP_FIRST | DBTSDF_COUNT_TRAFFIC.
 */
typedef struct {
    uint32_t dims[3];
    float voxel_size;
    float origin[3];
    uint32_t hit_threshold;
    uint32_t hit_max;
    uint32_t flags;
} dbtsdf_grid_params;

/*
 * Per-scan statistics. voxel_updates = n_integrated * K^3 (one eq. 4 AND per
 * kernel cell); shadow_updates = sum over integrated returns of |S(b)|.
 * u_mask / c_mask / u_shadow are only filled with DBTSDF_COUNT_TRAFFIC: the
 * number of distinct mask words in the union of the integrated neighbourhoods
 * (cells whose eq. 3 mask is all ones, which the AND leaves unchanged, are not
 * counted; they only occur for K = 37), of those whose value changed, and of
 * distinct words in the union of the shadows. In a batch call they are per grid and reported on the first scan of
 * that grid in the batch (zero on the others).
 * n_revisit counts the integrated returns whose voxel an earlier call had
 * already integrated (its mask reads 0): their eq. 4 window cannot lower any
 * mask, and the per-point and sort strategies skip it (the shadow counters are
 * still updated). It is a scheduling statistic of the library, not part of
 * the method: zero for the brick strategy, for kernel sets of more than 32768
 * bins, and for a grid whose planes dbtsdf_write_voxels wrote, until reset.
 */
typedef struct {
    uint64_t n_in;
    uint64_t n_invalid;       /* non-finite coordinates, or zero ray vector */
    uint64_t n_out_of_bounds; /* K^3 neighbourhood would leave the grid */
    uint64_t n_duplicate;     /* not first in its voxel within the scan */
    uint64_t n_integrated;
    uint64_t voxel_updates;
    uint64_t shadow_updates;
    uint64_t u_mask;
    uint64_t c_mask;
    uint64_t u_shadow;
    uint64_t n_revisit;
} dbtsdf_scan_stats;

/* How conflicting updates to one voxel are resolved. Results are identical. */
typedef enum {
    DBTSDF_STRATEGY_AUTO = 0,   /* the default: DBTSDF_STRATEGY_ATOMIC (dbtsdf_autotune measures instead) */
    DBTSDF_STRATEGY_BRICK = 1,  /* returns bucketed by grid brick; one workgroup owns a brick in LDS */
    DBTSDF_STRATEGY_ATOMIC = 2, /* one wavefront per return; 32-bit global atomics */
    DBTSDF_STRATEGY_SORT = 3,   /* every change a return makes to a word becomes a (voxel key, contribution)
                                   pair; the pairs are radix-sorted by key and a wavefront segmented reduction
                                   applies eq. 4 and eqs. 5-6 once per voxel, with no atomics on the planes */
    DBTSDF_STRATEGY_TILE = 4    /* returns listed by the 32x16x8 grid tiles their window reaches (a return in
                                   a voxel an earlier call integrated: the tiles its shadow reaches); one
                                   workgroup per tile takes the minimum eq. 3 distance and the shadow hit
                                   count of every word in LDS, then reads, updates and writes each touched
                                   word once with plain loads and stores (no atomics on the planes).
                                   Kernel sets with K <= 11, at most 31 bins and r_s^2 <= 9 */
} dbtsdf_strategy;

/*
 * Launch tuning of a grid. With DBTSDF_STRATEGY_BRICK, (brick, block_threads)
 * must be one of the compiled shapes: 16x8x8, 32x8x8, 64x8x8, 16x16x8,
 * 32x16x8 (256 threads), 32x16x8, 64x16x8, 32x16x16 (512 threads); a shape is
 * rejected when its LDS tiles cannot hold the kernel radius (only large K on
 * the largest shapes). apply_blocks = workgroups of the persistent apply
 * kernel (0 = as many as are resident at once).
 * chunk = most listed points one apply work unit takes from a brick; bricks
 * with more are split over several work units that merge with atomics
 * (0 = default 64, 0xFFFFFFFF = never split). With DBTSDF_STRATEGY_ATOMIC the
 * brick is ignored. DBTSDF_STRATEGY_SORT ignores the brick, takes chunk as the
 * most returns per round (0 or 0xFFFFFFFF: as many as its buffers allow), reads
 * the survivor and pair counts back in the middle of each call (so its calls
 * return once the pairs are sorted, and it never replays graphs), holds up to
 * 2^28 pairs of 12 bytes twice over in device memory (allocated on first use,
 * grown as calls need) and takes larger calls in several rounds of returns.
 * DBTSDF_STRATEGY_TILE takes brick 32x16x8 (0x0x0 or that shape) and 256
 * threads, ignores chunk, and needs a kernel set with K <= 11, at most 31
 * bins and r_s^2 <= 9 (INVALID_ARG otherwise).
 * Any valid tuning gives bit-identical grids. A new grid
 * starts with DBTSDF_STRATEGY_ATOMIC, brick 32x8x8, 256 threads, chunk 64.
 * A call that counts traffic (DBTSDF_COUNT_TRAFFIC) or spans more than 65536
 * grids runs with DBTSDF_STRATEGY_BRICK whatever the tuning says.
 */
typedef struct {
    uint32_t strategy;
    uint32_t brick[3];
    uint32_t block_threads;
    uint32_t apply_blocks;
    uint32_t chunk;
} dbtsdf_tuning;

typedef struct dbtsdf_kernel_set dbtsdf_kernel_set;
typedef struct dbtsdf_grid dbtsdf_grid;
typedef struct dbtsdf_batch dbtsdf_batch;
typedef struct dbtsdf_server dbtsdf_server;

/* Human-readable name of a status code (static storage). */
const char *dbtsdf_status_string(dbtsdf_status s);

/* Last error message recorded on the calling thread (static per thread; "" if none). */
const char *dbtsdf_last_error(void);

/* ---------------------------------------------------------------- kernel sets
 * Precomputed per-bin kernels (Sec. III-B): the eq. 3 mask of every kernel
 * cell, the shadow of every bin and the bin-centre unit vectors. Host-side.
 * *out is owned by the caller and released with dbtsdf_kernel_set_destroy.
 * Errors: INVALID_ARG (parameters, NULL), OUT_OF_MEMORY.
 */
dbtsdf_status dbtsdf_kernel_set_create(const dbtsdf_kernel_params *params, dbtsdf_kernel_set **out);

/*
 * Copy the tables out. masks: K^3 uint32 (index ((dz+R)*K + (dy+R))*K + (dx+R),
 * R = (K-1)/2); shadow: n_bins*K^3 bytes (1 = in the shadow, same cell order);
 * dirs: n_bins*3 doubles (bin-centre unit vectors; for AZEL, bin b has
 * azimuth index b % bins_az and elevation index b / bins_az, azimuth from +x
 * counter-clockwise, elevation from the nadir). Any output may be NULL.
 * *n_bins receives the bin count (may be NULL).
 */
dbtsdf_status dbtsdf_kernel_set_export(const dbtsdf_kernel_set *ks, uint32_t *masks, uint8_t *shadow,
                                       double *dirs, uint32_t *n_bins);

/* Number of bins (26 or bins_az*bins_el); 0 for NULL. */
uint32_t dbtsdf_kernel_set_n_bins(const dbtsdf_kernel_set *ks);

/* Direction bin of one ray vector d (map axes), as the device computes it; -1 on NULL. */
int32_t dbtsdf_kernel_set_bin(const dbtsdf_kernel_set *ks, float dx, float dy, float dz);

void dbtsdf_kernel_set_destroy(dbtsdf_kernel_set *ks);

/* --------------------------------------------------------------------- grids */

/* eq. 1: bytes of voxel storage = Nx*Ny*Nz*8; 0 if params is NULL. */
uint64_t dbtsdf_grid_bytes(const dbtsdf_grid_params *params);

/*
 * Allocate a grid on the current HIP device and fill the initial state
 * (Sec. III-A). The grid copies the kernel tables (the kernel set may be
 * destroyed afterwards). hip_stream is a hipStream_t (NULL = default stream)
 * that all work on this grid is enqueued on. The grid owns its planes.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE.
 */
dbtsdf_status dbtsdf_create_grid(const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks,
                                 void *hip_stream, dbtsdf_grid **out);

/*
 * As dbtsdf_create_grid, on caller-owned device planes (each Nx*Ny*Nz uint32,
 * 16-byte aligned, e.g. torch tensors). The planes are filled with the initial
 * state; they must outlive the grid and are not freed by it. The caller may
 * read them at any time but changes them only through this library (or
 * follows its own writes with dbtsdf_write_voxels or dbtsdf_reset_grid): the
 * per-point strategy relies on planes that integration alone has written
 * (see dbtsdf_write_voxels).
 */
dbtsdf_status dbtsdf_create_grid_on(const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks,
                                    void *hip_stream, void *mask_dev, void *packed_dev,
                                    dbtsdf_grid **out);

/* Device pointers of the two planes (for zero-copy views). */
dbtsdf_status dbtsdf_grid_planes(const dbtsdf_grid *g, void **mask_dev, void **packed_dev);

/* Refill the initial state (Sec. III-A) on the grid's stream. */
dbtsdf_status dbtsdf_reset_grid(dbtsdf_grid *g);

/* Read / set the launch tuning of a grid (see dbtsdf_tuning). */
dbtsdf_status dbtsdf_get_tuning(const dbtsdf_grid *g, dbtsdf_tuning *out);
dbtsdf_status dbtsdf_set_tuning(dbtsdf_grid *g, const dbtsdf_tuning *t);

/*
 * Fuse one scan (Sec. III-C, eqs. 2-6, Sec. IV-B dedup).
 *   pose     16 floats, row-major 4x4 sensor->map transform (host memory; the
 *            bottom row is ignored); must be finite.
 *   points   n x 3 fp32 (x, y, z) in the sensor frame. points_on_device = 0:
 *            host memory, copied to device staging before the call returns.
 *            points_on_device = 1: device memory that must stay valid and
 *            unmodified until dbtsdf_sync().
 *   n        number of points; 0 is a no-op. At most 2^28 per call.
 *   stats    NULL, or host memory that receives the statistics at the next
 *            dbtsdf_sync() (it must stay valid until then).
 * Non-finite and zero-range points are not errors: they are counted.
 * Front end arithmetic is fp32, one IEEE operation per step, no contraction.
 * The passes of a call are launched on the grid's stream: directly with the
 * per-point strategy (three passes), or, with the brick strategy, replayed
 * from a HIP graph captured (on a private stream of the grid) the first time
 * a call of that shape is made; the sort strategy launches directly and
 * waits for the stream twice to size its sort (see dbtsdf_tuning).
 * Errors: INVALID_ARG, OUT_OF_RANGE (n too large), OUT_OF_MEMORY, DEVICE, POISONED.
 */
dbtsdf_status dbtsdf_integrate_scan(dbtsdf_grid *g, const float pose[16], const float *points, uint64_t n,
                                    int points_on_device, dbtsdf_scan_stats *stats);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): dbtsdf_integrate_scan
 * with device points and the per-point strategy, allocating nothing. Every
 * buffer the call needs beyond the grid and the points (descriptors,
 * counters, point records, the first-return dedup table, the survivor list)
 * lives in one static device array of DBTSDF_NOALLOC_SCRATCH_BYTES per GPU,
 * set up on the first call on a device and held until the process ends.
 *   points_dev  n x 3 fp32 in device memory, valid until the passes have run.
 *   n           at most DBTSDF_NOALLOC_MAX_POINTS; more is OUT_OF_RANGE.
 *   stats       NULL: the call returns once its passes are enqueued on the
 *               grid's stream. Non-NULL: the call waits for its passes and
 *               fills *stats (traffic counts, u_mask/c_mask/u_shadow, are
 *               not taken and stay 0).
 * The grid's tuning is not used (the per-point kernels always run) and its
 * result is that of dbtsdf_integrate_scan, bit for bit. Calls on one GPU
 * share its array: calls that overlap on the device (different streams, or
 * threads) race and must be ordered by the caller. Calls on the same grid are
 * stream-ordered as usual. Errors: INVALID_ARG, OUT_OF_RANGE, DEVICE, POISONED.
 */
#define DBTSDF_NOALLOC_MAX_POINTS 131072u
#define DBTSDF_NOALLOC_SCRATCH_BYTES 11011584u
dbtsdf_status dbtsdf_integrate_scan_noalloc(dbtsdf_grid *g, const float pose[16], const float *points_dev, uint64_t n,
                                            dbtsdf_scan_stats *stats);

/*
 * dbtsdf_integrate_scan with the sequential downsampling of Sec. IV-B (DS =
 * every): only returns 0, every, 2 every, ... of the n given are taken, in
 * that order (so "first return" is among them), and the statistics count
 * those (n_in = ceil(n / every)). every = 1 is dbtsdf_integrate_scan. Host
 * points are staged whole. Errors as dbtsdf_integrate_scan; every = 0 is
 * INVALID_ARG.
 */
dbtsdf_status dbtsdf_integrate_scan_every(dbtsdf_grid *g, const float pose[16], const float *points, uint64_t n,
                                          uint32_t every, int points_on_device, dbtsdf_scan_stats *stats);

/* Motion compensation of a sweep (Sec. III-C: yaw-only or full SE(3)). */
typedef enum {
    DBTSDF_DESKEW_SE3 = 0, /* the whole rotation over the sweep */
    DBTSDF_DESKEW_YAW = 1  /* only its rotation about the map z axis */
} dbtsdf_deskew;

/*
 * The constants of a sweep from pose_start (R0, t0) to pose_end (R1, t1),
 * host memory, 4x4 row-major fp32 like the pose of dbtsdf_integrate_scan:
 * out[0..3] = the unit quaternion (w, x, y, z), w >= 0, of the rotation over
 * the sweep R1 R0^T (computed in fp64 by Shepperd's method, then rounded to
 * fp32); with DBTSDF_DESKEW_YAW that of the rotation about z taking the
 * projection of its x axis on the xy plane to where R1 R0^T takes it
 * ((1, 0, 0, 0) when the projection vanishes); out[4..6] = t1 - t0 (fp32).
 * Pure host code (no device call). Errors: INVALID_ARG (NULL, non-finite
 * pose, unknown mode).
 */
dbtsdf_status dbtsdf_deskew_constants(const float pose_start[16], const float pose_end[16], int mode, float out[7]);

/*
 * dbtsdf_integrate_scan_every for a sweep whose returns were taken while the
 * sensor moved: return j (of those taken) is transformed with the pose at its
 * time fraction tau = times[j * every] in [0, 1] between pose_start (0) and
 * pose_end (1): with q and dt the constants above, p = (1 - tau + tau q_w,
 * tau q_x, tau q_y, tau q_z), M the rotation matrix of p scaled by 2 / |p|^2,
 * R(tau) = M R0 and t(tau) = t0 + tau dt, all fp32 one operation at a time
 * (the normalised linear interpolation of the rotation; no sine or square
 * root per return). The direction for the bin is R(tau) times the point.
 * A return whose tau is outside [0, 1] or not a number is invalid (counted
 * in n_invalid). times: n floats beside the points, device memory when
 * points_on_device, else host memory (staged whole). mode: dbtsdf_deskew.
 * The passes are those of dbtsdf_integrate_scan. Errors as
 * dbtsdf_integrate_scan_every; NULL times or an unknown mode is INVALID_ARG.
 */
dbtsdf_status dbtsdf_integrate_scan_deskew(dbtsdf_grid *g, const float pose_start[16], const float pose_end[16],
                                           const float *points, const float *times, uint64_t n, uint32_t every,
                                           int mode, int points_on_device, dbtsdf_scan_stats *stats);

/*
 * Wait for all work on the grid's stream, deliver pending statistics.
 * Errors: DEVICE (the grid becomes poisoned), POISONED.
 */
dbtsdf_status dbtsdf_sync(dbtsdf_grid *g);

/*
 * Copy the box [lo, hi) (voxel indices, lo < hi <= dims) to host memory, x
 * fastest: mask_out and packed_out hold (hi-lo) products of uint32 each (either
 * may be NULL). Synchronous. Errors: INVALID_ARG, OUT_OF_RANGE, DEVICE, POISONED.
 */
dbtsdf_status dbtsdf_read_voxels(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3],
                                 uint32_t *mask_out, uint32_t *packed_out);

/*
 * Signed truncated distance of the box [lo, hi), x fastest, host int8:
 * (sign ? +1 : -1) * popcount(mask) (Sec. III-A); untouched voxels read +32.
 * Synchronous. Errors as dbtsdf_read_voxels.
 */
dbtsdf_status dbtsdf_read_distance(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], int8_t *dist_out);

/*
 * Mesh export (the pipeline's last block, Sec. III: Marching Cubes of the
 * fused map at iso = 0.0) of the signed distance that read_distance gives.
 * Takes every cube of the dual grid whose eight corner voxels lie in the box
 * [lo, hi) (lo, hi NULL: the whole grid). A corner is inside when its distance
 * is negative; a crossed edge from voxel u to u + e_a has its vertex at
 * t = d(u) / (d(u) - d(u + e_a)), coordinate o + (u + 0.5) s on the other
 * axes and o_a + (u_a + 0.5) s + t s along a (fp32, one operation at a time,
 * in that order). Saddle faces keep inside corners apart; face segments run
 * counter-clockwise seen from outside the cube and chain into loops fanned
 * from their smallest edge number (edges 4 a + rank of the lower corner among
 * those with bit a clear; corners x + 2y + 4z), or from their centre (the
 * mean of the loop's vertices) when a loop holds all four crossed edges of a
 * saddle face. Normals (right-hand rule) point to positive distance.
 * tris_dev: device memory for max_tris triangles of 9 floats (v0 xyz, v1 xyz,
 * v2 xyz), or NULL with max_tris 0 to count only. *n_tris receives the number
 * of triangles of the mesh; when it exceeds max_tris only max_tris of them are
 * written (which ones is unspecified). The order of the triangles is
 * unspecified. Runs on the grid's stream and synchronises it.
 * Errors: INVALID_ARG (NULL n_tris, NULL tris_dev with max_tris > 0),
 * OUT_OF_RANGE (box), OUT_OF_MEMORY, DEVICE, POISONED.
 */
dbtsdf_status dbtsdf_extract_mesh(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], float *tris_dev,
                                  uint64_t max_tris, uint64_t *n_tris);

/*
 * Point export (beside the mesh, the pipeline's CSV/PCL output, Sec. III):
 * the centres o + (u + 0.5) s (fp32, one operation at a time) of the occupied
 * contact voxels of the box [lo, hi) (NULL, NULL: the whole grid), i.e. those
 * a return landed in (mask 0) whose hit counter confirmed them (sign 0).
 * xyz_dev: device memory for max_points points of 3 floats, or NULL with
 * max_points 0 to count only; *n_points receives the count (when it exceeds
 * max_points only max_points are written). Points of one grid row come out in
 * x order, rows in no fixed order. Runs on the grid's stream and synchronises
 * it. Errors as dbtsdf_extract_mesh.
 */
dbtsdf_status dbtsdf_extract_points(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], float *xyz_dev,
                                    uint64_t max_points, uint64_t *n_points);

/*
 * Reconstruction-accuracy metrics (Sec. IV-A): nearest-neighbour distances
 * between a predicted point set (points on the zero level of the map, e.g.
 * the vertices of the exported mesh) and a ground-truth set.
 * Squared distances are ((qx - rx)^2 + (qy - ry)^2) + (qz - rz)^2 in IEEE
 * fp64 from the fp32 coordinates, one operation at a time in that order; a
 * nearest squared distance is the minimum of that over the whole set (exact:
 * it does not depend on the search order). "Within the tolerance t" is
 * d^2 < t * t (strict).
 *   accuracy      mean over predicted points of the distance to the nearest
 *                 ground-truth point (metres)
 *   completeness  mean over ground-truth points of the distance to the
 *                 nearest predicted point (metres)
 *   chamfer_l1    (accuracy + completeness) / 2
 *   precision     share of predicted points within t of the ground truth
 *   recall        share of ground-truth points within t of the prediction
 *   fscore        2 precision recall / (precision + recall), 0 when both are 0
 */
typedef struct dbtsdf_metrics {
    double accuracy, completeness, chamfer_l1;
    double precision, recall, fscore;
    uint64_t n_pred, n_gt, n_pred_within, n_gt_within;
} dbtsdf_metrics;

/*
 * Nearest squared distance of every query point to the reference set.
 * query_dev: n_query x 3 fp32 (x, y, z per point), ref_dev: n_ref x 3 fp32,
 * d2_dev: n_query fp64 written; all device memory of GPU `device`, owned by
 * the caller. Runs on that device's null stream and synchronises it;
 * allocates scratch (a cell grid of the reference points) for the call.
 * Errors: INVALID_ARG (NULL pointer with a nonzero count, n_ref 0 with
 * queries, a non-finite coordinate), OUT_OF_RANGE (n_query or n_ref above
 * 2^32 - 16), OUT_OF_MEMORY, DEVICE.
 */
dbtsdf_status dbtsdf_nearest_sq(int device, const float *query_dev, uint64_t n_query, const float *ref_dev,
                                uint64_t n_ref, double *d2_dev);

/*
 * The metrics above of pred_dev (n_pred x 3 fp32) against gt_dev (n_gt x 3
 * fp32), device memory of GPU `device`, at tolerance t (metres, finite,
 * >= 0), into *out (host). Sums are taken in a fixed order (repeatable bit
 * for bit). Errors as dbtsdf_nearest_sq; either set empty, NULL out or a bad
 * tolerance is INVALID_ARG.
 */
dbtsdf_status dbtsdf_surface_metrics(int device, const float *pred_dev, uint64_t n_pred, const float *gt_dev,
                                     uint64_t n_gt, double tolerance, dbtsdf_metrics *out);

/*
 * Overwrite the whole grid from host planes (Nx*Ny*Nz uint32 each, x fastest),
 * e.g. a checkpoint written from dbtsdf_read_voxels. Rejects (INVALID_ARG)
 * planes that break the representation: a mask not of the form 2^n - 1, bits
 * 16-30 of packed set, a counter above hit_max, or a sign that disagrees with
 * the counter (sign 0 iff 1 <= T <= hit_max and h >= T). Synchronous.
 * Integration relies on this: a return whose voxel an earlier call integrated
 * (its mask reads 0) has its whole eq. 4 window at least as tight already,
 * since that earlier return stamped the same masks, so the per-point strategy
 * skips the window (the shadow counters are still updated). Written planes
 * need not hold such windows, so after this call the grid integrates every
 * window in full until dbtsdf_reset_grid. A restored map therefore runs
 * slower than the map it was saved from: late in a long sequence most
 * returns land in voxels the map already holds, and each of them now loads
 * and compares its whole window (the result is the same).
 */
dbtsdf_status dbtsdf_write_voxels(dbtsdf_grid *g, const uint32_t *mask_in, const uint32_t *packed_in);

void dbtsdf_destroy_grid(dbtsdf_grid *g);

/* ---------------------------------------------------------------- profiling
 * Device-side timing with HIP events on the work's own stream. `enable` is a
 * period: 0 turns profiling off, N >= 1 times every N-th integrate call
 * (plain or batched; 1 = every call): those whose index, counted over all
 * calls on the grid (batch context) since its creation, is a multiple of N.
 * Negative is DBTSDF_ERR_INVALID_ARG. A timed call records events at its start, just
 * before the apply kernel (eqs. 4-6, the dominant kernel) and just after it;
 * the apply kernel is then launched directly between its two events, and the
 * passes before and after it are replayed from graphs (the split costs the
 * timed call some microseconds of launch gaps, which a period above 1
 * spreads thin). call time = start to the end of the apply kernel.
 * read_profile synchronises the stream and returns the accumulated
 * milliseconds and counts of the timed calls since profiling was last set.
 * Any output may be NULL. Setting resets the totals.
 */
dbtsdf_status dbtsdf_set_profiling(dbtsdf_grid *g, int enable);
dbtsdf_status dbtsdf_read_profile(dbtsdf_grid *g, double *call_ms, uint64_t *calls, double *apply_ms,
                                  uint64_t *applies);

/* ----------------------------------------------------------------- batching
 * Many scans of many grids fused by one launch sequence: one front-end pass
 * over all points, then one persistent apply kernel over every (grid, brick)
 * work item, optionally replayed from a captured HIP graph. Results are
 * identical to integrating the scans one by one in any order (the updates of
 * eqs. 4-6 commute; dedup stays per scan).
 *
 * A batch context owns a HIP stream-ordered workspace and a graph cache. All
 * grids of one call must live on the device the context was created on; the
 * context's stream is hip_stream (NULL = default stream), which must not be
 * used concurrently by another context. use_graph = 0 launches the passes one
 * by one instead of replaying graphs (graphs are captured on a private stream
 * and launched on the context's stream, the default stream included).
 */
dbtsdf_status dbtsdf_batch_create(void *hip_stream, int use_graph, dbtsdf_batch **out);

/*
 * Enqueue n_scans scans: scan i goes into grids[i] with pose poses[16*i..],
 * points[i] (n[i] x 3 fp32, device memory when points_on_device, else host
 * memory copied before return), statistics into stats[i] at dbtsdf_batch_sync
 * (stats may be NULL). The same grid may appear several times. Points on the
 * device must stay valid until dbtsdf_batch_sync(). Total points <= 2^28.
 */
dbtsdf_status dbtsdf_batch_integrate(dbtsdf_batch *b, uint32_t n_scans, dbtsdf_grid *const *grids,
                                     const float *poses, const float *const *points, const uint64_t *n,
                                     int points_on_device, dbtsdf_scan_stats *stats);

/*
 * The same for callers without a batch context: n_scans scans into grids[i]
 * with poses[16*i..] and device points[i] (n[i] x 3 fp32), in one launch
 * sequence on a context the library keeps per device (made on first use,
 * calls through it serialised). Ordered after earlier work on each grid's
 * stream and before later work there. With stats (n_scans entries) the call
 * returns once the batch has finished and the statistics are filled in;
 * with stats NULL it returns after enqueueing. Errors as dbtsdf_batch_integrate.
 */
dbtsdf_status dbtsdf_integrate_batch(uint32_t n_scans, dbtsdf_grid *const *grids, const float *poses,
                                     const float *const *points, const uint64_t *n, dbtsdf_scan_stats *stats);

/*
 * dbtsdf_batch_integrate for motion-compensated sweeps (as
 * dbtsdf_integrate_scan_deskew, every = 1): scan i runs from poses_start[16*i..]
 * to poses_end[16*i..], return j at time fraction times[i][j]; times[i] lives
 * where the points do (host arrays are copied before return). mode:
 * dbtsdf_deskew, for every scan of the call. Errors as dbtsdf_batch_integrate;
 * NULL times, a non-finite end pose or an unknown mode is INVALID_ARG.
 */
dbtsdf_status dbtsdf_batch_integrate_deskew(dbtsdf_batch *b, uint32_t n_scans, dbtsdf_grid *const *grids,
                                            const float *poses_start, const float *poses_end, int mode,
                                            const float *const *points, const float *const *times,
                                            const uint64_t *n, int points_on_device, dbtsdf_scan_stats *stats);

/* Wait for the batch context's stream and deliver statistics. */
dbtsdf_status dbtsdf_batch_sync(dbtsdf_batch *b);

/* Number of graph captures and graph replays so far (either may be NULL). */
dbtsdf_status dbtsdf_batch_graph_stats(const dbtsdf_batch *b, uint64_t *captures, uint64_t *replays);

/* Profiling of a batch context (see dbtsdf_set_profiling). */
dbtsdf_status dbtsdf_batch_set_profiling(dbtsdf_batch *b, int enable);
dbtsdf_status dbtsdf_batch_read_profile(dbtsdf_batch *b, double *call_ms, uint64_t *calls, double *apply_ms,
                                        uint64_t *applies);

void dbtsdf_batch_destroy(dbtsdf_batch *b);

/* ------------------------------------------------------------------ tuning
 * Time each candidate tuning on the grid with the given scans (device points),
 * on a scratch copy of the grid (the grid itself is not changed), keep the
 * fastest, and return it in *best (may be NULL). Every candidate is checked to
 * give a bit-identical scratch grid; a mismatch returns DEVICE.
 */
dbtsdf_status dbtsdf_autotune(dbtsdf_grid *g, uint32_t n_scans, const float *poses,
                              const float *const *points_dev, const uint64_t *n, dbtsdf_tuning *best);

/* ----------------------------------------------------------------- serving
 * A request loop that keeps many grids resident in HBM and fuses scans as they
 * arrive (continuous batching): a scheduler thread takes every ready scan up
 * to the batch limits, integrates them with one batched launch on one of
 * n_streams streams while earlier batches are still running, and stamps each
 * scan's completion when its batch's event fires. Scans of one map are never
 * in flight twice at once, so per-map order is kept (results do not depend on
 * it anyway). New maps are admitted only while their eq. 1 bytes fit in the
 * memory budget.
 */
typedef struct {
    uint32_t n_streams;          /* >= 1 concurrent batches (default 2) */
    uint32_t max_batch_scans;    /* scans per batch (default 64) */
    uint64_t max_batch_points;   /* points per batch (default 4M) */
    uint64_t memory_budget;      /* bytes of grid storage admitted; 0 = free device memory minus 8 GiB */
    uint32_t queue_capacity;     /* pending scans before submit returns BUSY (default 4096) */
    uint32_t use_graph;          /* replay batches from captured graphs */
} dbtsdf_server_config;

typedef struct {
    uint64_t ticket;         /* from dbtsdf_server_submit */
    uint32_t map_id;
    uint32_t status;         /* dbtsdf_status of the scan */
    uint64_t t_arrival_ns;   /* as given at submit */
    uint64_t t_launch_ns;    /* host clock when its batch was enqueued */
    uint64_t t_done_ns;      /* host clock when its batch's completion was observed */
    uint32_t batch_scans;    /* scans in the batch it rode in */
    dbtsdf_scan_stats stats;
} dbtsdf_completion;

dbtsdf_status dbtsdf_server_create(const dbtsdf_server_config *cfg, dbtsdf_server **out);

/* Admit a map (allocates its grid). OUT_OF_MEMORY when the budget is exceeded. */
dbtsdf_status dbtsdf_server_add_map(dbtsdf_server *s, const dbtsdf_grid_params *params,
                                    const dbtsdf_kernel_set *ks, uint32_t *map_id);

/* Release a map's grid (waits for its in-flight work). */
dbtsdf_status dbtsdf_server_remove_map(dbtsdf_server *s, uint32_t map_id);

/* The grid of an admitted map (owned by the server), e.g. for readout after drain. */
dbtsdf_status dbtsdf_server_map_grid(dbtsdf_server *s, uint32_t map_id, dbtsdf_grid **g);

/*
 * Queue one scan (host points, copied into pinned staging before return).
 * t_arrival_ns is the caller's arrival stamp on the CLOCK_MONOTONIC clock
 * (dbtsdf_now_ns). BUSY when the queue is full.
 */
dbtsdf_status dbtsdf_server_submit(dbtsdf_server *s, uint32_t map_id, const float pose[16], const float *points,
                                   uint64_t n, uint64_t t_arrival_ns, uint64_t *ticket);

/*
 * Queue one motion-compensated sweep (as dbtsdf_integrate_scan_deskew):
 * pose_start and pose_end host 4x4 fp32, mode a dbtsdf_deskew, n points and
 * n time fractions in [0, 1] (host, copied before return). A launch holds
 * only requests of one kind (plain scans, or sweeps of one mode); scans of
 * one map still complete in arrival order. Errors as dbtsdf_server_submit;
 * a non-finite end pose, NULL times or an unknown mode is INVALID_ARG.
 */
dbtsdf_status dbtsdf_server_submit_sweep(dbtsdf_server *s, uint32_t map_id, const float pose_start[16],
                                         const float pose_end[16], int mode, const float *points, const float *times,
                                         uint64_t n, uint64_t t_arrival_ns, uint64_t *ticket);

/* Move up to max finished scans into out; *n_out receives the count. Non-blocking. */
dbtsdf_status dbtsdf_server_poll(dbtsdf_server *s, dbtsdf_completion *out, uint32_t max, uint32_t *n_out);

/* Block until every submitted scan has completed (completions stay pollable). */
dbtsdf_status dbtsdf_server_drain(dbtsdf_server *s);

/* Admitted bytes and the budget (either may be NULL). */
dbtsdf_status dbtsdf_server_memory(const dbtsdf_server *s, uint64_t *admitted, uint64_t *budget);

void dbtsdf_server_destroy(dbtsdf_server *s);

/* CLOCK_MONOTONIC in nanoseconds (the server's clock). */
uint64_t dbtsdf_now_ns(void);

#ifdef __cplusplus
}
#endif
#endif /* DBTSDF_H */
