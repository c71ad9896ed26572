/*
 * hull3d.h -- C ABI of the MI355X (gfx950) divide-and-conquer 3-d convex hull.
 *
 * The method is the paper's: points sorted by x (Sec. 2), each block's lower
 * hull kept as a "movie" -- the time-ordered insert/delete events of a 2-d
 * kinetic hull, one event per 3-d face (Sec. 2, the kinetic reformulation) --
 * and movies merged pairwise, level by level, bottom-up (Sec. 2, the movie
 * array and merge step; Sec. 3, Fig. "main_loop_figure" and Fig.
 * "kernel_variables").  The upper hull is the lower hull of the points with z
 * negated.  All predicates are exact on the integer lattice, with ties broken
 * by a symbolic perturbation indexed by the input position i:
 *   (x + e1*i, y + e2*i^2, z + e3*i^3),  1 >> e1 >> e2 >> e3 > 0,
 * so the result is the unique face set of the perturbed points' hull (every
 * face a triangle, F = 2V - 4; degenerate inputs give one specific
 * triangulation, possibly with zero-area faces).
 *
 * Conventions (all entry points):
 *  - Pointers named d_* are device pointers owned by the caller.  The library
 *    allocates nothing and keeps no state between calls.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the
 *    default stream).  The return value reports argument errors and launch
 *    failures only; errors that depend on the data are written to d_info[0]
 *    on the device.
 *  - Points are int32 (x, y, z) rows, C-contiguous [n, 3], |coord| <= 2^29,
 *    n <= 2^26.
 *  - Faces are int32 rows of input indices (0-based), oriented counter-
 *    clockwise seen from outside (outward right-hand normal).  Row order is
 *    unspecified.  n < 3 gives no face; n = 3 gives the triangle twice, once
 *    per orientation.
 *  - Calls on different streams are independent if each has its own
 *    workspace.
 *  - A HIP error left pending on the calling thread by earlier, unrelated
 *    HIP calls is cleared on entry (it is not reported as this call's
 *    failure); hull_last_hip_error() gives the HIP code behind a HULL_EHIP.
 */
#ifndef HULL3D_H
#define HULL3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (return values and d_info[0]). */
#define HULL_OK 0
#define HULL_EINVAL (-1)     /* null pointer, n out of range, capacity < 2n */
#define HULL_EWORKSPACE (-2) /* workspace smaller than hull_workspace_bytes() */
#define HULL_ERANGE (-3)     /* a coordinate outside the entry point's range (reported in
                                d_info[0]): |c| > 2^29 for int32 rows; see the wide and
                                float entry points for theirs */
#define HULL_EHIP (-4)       /* HIP runtime or launch failure */
#define HULL_EINTERNAL (-5)  /* an internal consistency bound tripped (d_info[0]) */

/* Static description of a status code. */
const char* hull_strerror(int32_t code);

/* The hipError_t behind the last HULL_EHIP returned on this host thread (0
 * if none yet). */
int32_t hull_last_hip_error(void);

/* Workspace kinds for hull_workspace_bytes. */
#define HULL_WS_STANDARD 0 /* hull_lower, hull_full (int32 rows) */
#define HULL_WS_WIDE 1     /* hull_lower_wide, hull_full_wide (int64 rows) */
#define HULL_WS_F32 2      /* hull_full_f32, hull_lower_f32 (float rows) */

/* Bytes of device workspace that the entry points of kind `flags` (one of
 * HULL_WS_*) need for n points (host, synchronous).  HULL_EINVAL for another
 * flag value, n < 0 or n > 2^26. */
int32_t hull_workspace_bytes(int64_t n, int32_t flags, size_t* bytes);

/* Lower hull: the faces whose outward normal points to negative z (under the
 * perturbation; every face is lower or upper).
 *   d_xyz   device int32 [n, 3]                    (read)
 *   d_faces device int32 [cap, 3], cap >= 2n      (written: first F rows)
 *   d_info  device int64 [2]: status, F           (written)
 *   d_ws    device workspace of ws_bytes bytes    (scratch)
 * The kinetic merge of the paper, run once (Sec. 2; Sec. 3). */
int32_t hull_lower(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                   void* d_ws, size_t ws_bytes, void* stream);

/* Full hull: lower faces followed by upper faces, F = 2V - 4 (n >= 3).  The
 * upper faces are the lower faces of (x, y, -z) with the z perturbation
 * negated too, so both halves close into one surface. */
int32_t hull_full(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, void* stream);

/* hull_full, with HIP events recorded on `stream` at phase boundaries, for
 * timing each kernel phase:
 *   events[0]              on entry
 *   events[1]              after the sort
 *   events[2k], [2k+1]     around the merge kernel of level k = 1..L,
 *                          L = ceil(log2 n)
 *   events[2L+2]           after the face extraction
 * `events` is a host array of nevents >= 2L+3 hipEvent_t handles that the
 * caller created (and destroys); otherwise the same as hull_full. */
int32_t hull_full_timed(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                        int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream,
                        void* const* events, int32_t nevents);

/* The same two calls on the wide coordinate range: int64 rows [n, 3] with
 * |x|, |y| <= 2^30 and |z| <= 2^42 (beyond the standard range of 2^29; for
 * instance lifted points (x, y, x^2 + y^2) with |x|, |y| <= 2^20).  Same
 * method, same perturbation and the same result definition; the orientation
 * products are taken in int128, and exact ties of the double filter go to
 * the full 256-bit cascade.  A coordinate outside the range gives HULL_ERANGE
 * in d_info[0].  Workspace: hull_workspace_bytes(n, HULL_WS_WIDE).  The
 * paper keeps float coordinates (Sec. 3, Fig. "point_datatypes"); the wide
 * range is what float input snapped to a 30-bit lattice needs. */
int32_t hull_lower_wide(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                        int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream);
int32_t hull_full_wide(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                       int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream);

/* Float input (the paper's single-precision coordinates, Sec. 3, Fig.
 * "point_datatypes"): every coordinate of the float32 rows [n, 3] is scaled
 * by the one power of two s = 2^(bits - E), E the least integer with
 * max |c| <= 2^E over all 3n coordinates (E = 0 if all are zero), and rounded
 * to the nearest integer, ties to even; the faces are those of the exact
 * perturbed hull of these lattice points (as hull_full_wide / hull_lower_wide
 * on them).  Scaling by a power of two is exact, so the only rounding is the
 * last step: floats within a factor 2^(bits - 24) of the largest magnitude
 * keep their value exactly.  bits in [1, 30] (HULL_EINVAL otherwise).  A NaN
 * or infinite coordinate gives HULL_ERANGE in d_info[0].
 * Workspace: hull_workspace_bytes(n, HULL_WS_F32). */
int32_t hull_full_f32(const float* d_xyz, int64_t n, int32_t bits, int32_t* d_faces, int64_t cap,
                      int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream);
int32_t hull_lower_f32(const float* d_xyz, int64_t n, int32_t bits, int32_t* d_faces, int64_t cap,
                       int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream);

/* hull_full for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same call
 * without a workspace argument.  Its scratch memory is a fixed 64 MiB device
 * array of the library (one per GPU, held until the process ends), so n is
 * limited to the sizes whose hull_workspace_bytes(n, HULL_WS_STANDARD) fits
 * in 64 MiB; larger n returns HULL_EWORKSPACE before launching anything.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race and must not be
 * made.  Uses the current device (the stream must belong to it). */
int32_t hull_full_noalloc(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                          int64_t* d_info, void* stream);

/* Merge schedule of a batched call (every field < 0, or 0 for walk_segment,
 * takes the library default):
 *   serial_levels  merge levels 1..serial_levels run one lane per merge (the
 *                  paper's kernel, Sec. 3); the levels above split each merge
 *                  into time segments walked in parallel (default 10)
 *   walk_segment   child events per walk segment, >= 4 (default 4)
 *   fused_levels   ignored on input (pass 0 or -1); hull_schedule_defaults
 *                  writes the number of LDS-staged lowest levels here
 *   wave_from      lane-serial levels from this one on run one merge per
 *                  group of wave_lanes lanes instead of one per lane (the
 *                  six candidates of an iteration on six lanes, child movies
 *                  through LDS); 0: the default (level 4 for calls of up to
 *                  2^16 points in all, 5 up to 2^18, one level later per
 *                  doubling, level 8 from 2^21 points), negative: no level
 *   wave_lanes     lanes per merge at level wave_from: 8, 16, 32 or 64,
 *                  doubling with every level above (merges halve), up to
 *                  wave_lanes_max (0: the default, 8)
 *   wave_lanes_max the most lanes per merge: 8, 16, 32 or 64, at least
 *                  wave_lanes (0: the default, 64; environment
 *                  HULL_WAVE_LANES_MAX).  Batches with many long merges on
 *                  the top lane-serial levels keep more merges in flight
 *                  with fewer lanes each. */
typedef struct hull_schedule_t {
  int32_t serial_levels;
  int32_t walk_segment;
  int32_t fused_levels;
  int32_t wave_from;
  int32_t wave_lanes;
  int32_t wave_lanes_max;
} hull_schedule_t;

/* The schedule the library uses when a call passes none (or leaves a field
 * at its default; wave_from as for the largest calls, 2^21 points and more):
 * the built-in defaults, overridden by the environment
 * variables HULL_SERIAL_LEVELS, HULL_WALK_SEGMENT, HULL_WAVE_LEVEL and
 * HULL_WAVE_LANES when set.  On output, fused_levels is the number of lowest
 * lane-serial levels that stage each merge's points and links in LDS (a
 * separate kernel from the other lane-serial levels; default 3, at most 4,
 * environment HULL_LDS_LEVELS).  Above them, lane-serial merges of blocks up
 * to 128 points and lane-group merges keep only their working links in LDS
 * (HULL_LDS_LINKS=0: in global memory), except on lane-group levels of at
 * most 1024 merges in all (environment HULL_PTS_LDS_MERGES), where a merge's
 * points join its links in LDS when a workgroup's share fits.  None of this
 * changes a result.
 * Host, synchronous. */
int32_t hull_schedule_defaults(hull_schedule_t* out);

/* Bytes of device workspace for hull_full_batched over H hulls of
 * total_points points in all (host, synchronous).  total_points is at most
 * 2^28 (whose workspace, about 924 bytes per point, fits one GPU's memory);
 * more returns HULL_EINVAL, as does hull_full_batched. */
int32_t hull_workspace_bytes_batched(int64_t total_points, int64_t H, size_t* bytes);

/* Full hulls of H independent point clouds in one launch sequence: every
 * merge level of every hull runs in the same kernels (the level loop of
 * Sec. 3 over a device-built list of the merges of all hulls).
 *   d_xyz          device int32 [N, 3], N = h_offsets[H]; cloud h is rows
 *                  [offsets[h], offsets[h+1]), each of at most 2^26 points
 *   d_offsets      device int64 [H + 1], offsets[0] = 0, non-decreasing
 *   h_offsets      host copy of the same offsets (read during the call)
 *   d_faces        device int32 [cap, 3], cap >= 2N (written): the faces of
 *                  cloud h are rows [face_offsets[h], face_offsets[h+1]),
 *                  lower then upper, indices local to the cloud; a cloud
 *                  of fewer than 3 points has none
 *   d_face_offsets device int64 [H + 1] (written)
 *   d_info         device int64 [2]: status, total faces (written)
 *   schedule       NULL = defaults
 * The perturbation index of a point is its index within its own cloud, so
 * each cloud's faces equal those of hull_full on that cloud alone. */
int32_t hull_full_batched(const int32_t* d_xyz, const int64_t* d_offsets, const int64_t* h_offsets,
                          int64_t H, int32_t* d_faces, int64_t cap, int64_t* d_face_offsets,
                          int64_t* d_info, void* d_ws, size_t ws_bytes,
                          const hull_schedule_t* schedule, void* stream);

/* Intermediate movies, for inspection and tests: sorts, runs `level` merge
 * levels (level < 0: all) of run 0 (lower) or 1 (upper) and writes, for
 * every block of width 2^level from rank 0, its movie events at offset
 * 2 * (block start):
 *   d_ev        device int32 [2n, 4]: (left, middle, right rank, is_insertion)
 *   d_block_len device int32 [n]: event count at each block start
 *   d_order     device int32 [n]: input index of each rank
 * Same workspace as hull_full. */
int32_t hull_movies(const int32_t* d_xyz, int64_t n, int32_t run, int32_t level, int32_t* d_ev,
                    int32_t* d_block_len, int32_t* d_order, int64_t* d_info, void* d_ws,
                    size_t ws_bytes, void* stream);

/* Volume and surface area of H closed hull surfaces (FP32), for clouds given
 * as float positions:
 *   d_p        device float [N, 3]; cloud h is rows [pt_off[h], pt_off[h+1])
 *   d_pt_off   device int64 [H + 1]
 *   d_faces    device int32 [F, 3]: outward faces, indices local to the cloud
 *              (as hull_full returns them); cloud h owns face rows
 *              [face_off[h], face_off[h+1])
 *   d_face_off device int64 [H + 1]
 *   d_V, d_A   device float [H] (written)
 * V = 1/6 sum_f (a - c).((b - c) x (d - c)) with c = the cloud's point 0,
 * A = 1/2 sum_f |(b - a) x (d - a)|; per-face FP32 terms, compensated
 * per-thread sums and a fixed-order tree reduction (deterministic).  One
 * workgroup per cloud. */
int32_t hull_volume_area_fwd(const float* d_p, const int64_t* d_pt_off, const int32_t* d_faces,
                             const int64_t* d_face_off, int32_t H, float* d_V, float* d_A,
                             void* stream);

/* Gradient of sum_h (gV[h] V_h + gA[h] A_h) with respect to the positions,
 * on the fixed face set (faces carry no gradient):
 *   dV/dp = 1/6 sum of the face normals (b - a) x (d - a) around p,
 *   dA/da = 1/2 (b - d) x unit normal, summed over the faces (a, b, d) at a
 *           (0 for zero-area faces).
 * d_gV / d_gA: device float [H] (either may be NULL = 0); d_grad_p: device
 * float [N, 3], fully overwritten.  Contributions are added with float
 * atomics, so the last bits may depend on the execution order. */
int32_t hull_volume_area_bwd(const float* d_p, const int64_t* d_pt_off, const int32_t* d_faces,
                             const int64_t* d_face_off, int32_t H, const float* d_gV,
                             const float* d_gA, float* d_grad_p, void* stream);

/* Bytes of device workspace for hull_face_adjacency on F faces (host,
 * synchronous). */
int32_t hull_adjacency_workspace_bytes(int64_t F, size_t* bytes);

/* Face adjacency (half-edge twins) of closed, consistently oriented surfaces,
 * as hull_full and hull_full_batched return them: the connectivity of an
 * edge-list structure (the paper's future work, Sec. "Conclusion").
 *   d_faces    device int32 [F, 3]: face rows; edge k of row f runs from
 *              vertex k to vertex (k + 1) mod 3
 *   d_face_off device int64 [H + 1] face offsets of the clouds, and
 *   d_pt_off   device int64 [H + 1] their point offsets (vertex indices are
 *              within the cloud); both NULL for a single surface (H ignored)
 *   d_adj      device int32 [F, 3] (written): adj[f][k] = the row of the face
 *              holding the reverse edge (vertex k+1 -> vertex k) in the same
 *              cloud, -1 if none
 *   d_info     device int64 [2] (written): status (HULL_OK; HULL_ERANGE: a
 *              vertex index outside its cloud; HULL_EINTERNAL: a directed
 *              edge used twice, not a 2-manifold) and the number of edges
 *              without a twin (0 for a closed surface)
 *   d_ws       workspace of hull_adjacency_workspace_bytes(F) bytes
 * F may be at most (2^31 - 3) / 3 (half-edge ids 3f + k are int32); larger F
 * returns HULL_EINVAL here and from hull_adjacency_workspace_bytes.
 * A hash table of directed edges in the workspace: one insertion pass, one
 * lookup pass (deterministic result). */
int32_t hull_face_adjacency(const int32_t* d_faces, int64_t F, const int64_t* d_face_off,
                            const int64_t* d_pt_off, int64_t H, int32_t* d_adj, int64_t* d_info,
                            void* d_ws, size_t ws_bytes, void* stream);

/* Bytes of device workspace for hull_delaunay on n points (host,
 * synchronous). */
int32_t hull_delaunay_workspace_bytes(int64_t n, size_t* bytes);

/* 2-d Delaunay triangulation by lifting: the lower hull of (x, y, x^2 + y^2)
 * (the hull method of Sec. 2 and 3 unchanged; Sec. "Conclusion" names such
 * follow-on algorithms).
 *   d_xy    device int32 [n, 2], |x|, |y| <= 2^20 (lifted z = x^2 + y^2 up to
 *           2^41: the wide range of hull_lower_wide, which runs the lower
 *           hull; otherwise HULL_ERANGE in d_info[0])
 *   d_tris  device int32 [cap, 3], cap >= 2n (written: first T rows):
 *           triangles of input indices, counter-clockwise in the plane
 *   d_info  device int64 [2]: status, T
 *   d_ws    workspace of hull_delaunay_workspace_bytes(n) bytes
 * Ties (cocircular or collinear points, duplicates) are decided by the hull's
 * symbolic perturbation: the result is the Delaunay triangulation of the
 * perturbed points (unique; zero-area triangles possible for degenerate
 * input; T = 2n - h - 2 with h points on the perturbed convex hull). */
int32_t hull_delaunay(const int32_t* d_xy, int64_t n, int32_t* d_tris, int64_t cap, int64_t* d_info,
                      void* d_ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HULL3D_H */
