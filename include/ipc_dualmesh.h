/* Dual-mesh mapping of PhyVisGen (arXiv 2609.25653, Sec. III-D, Eq. (6)-(7)):
 * the fine render mesh of a deformable object is L levels of Loop
 * subdivision of its coarse simulation mesh.  Every level is linear in the
 * positions, so the whole subdivision is one sparse matrix
 *     W = S^(L) ... S^(1)   (N_f x N_c, Eq. (6)),
 * built once, and the fine states of every frame are X^f_t = W X^c_t
 * (Eq. (7)).  The library builds W on the host at creation and applies it
 * to many frames in one launch on the GPU.
 *
 * Rules of one level (Loop's scheme; the paper gives no weights): an edge
 * shared by two triangles gets 3/8 of each end and 1/8 of each opposite
 * corner, a boundary edge its midpoint; an old interior vertex of valence n
 * keeps 1 - n beta of itself and beta of each neighbour, beta = (5/8 -
 * (3/8 + cos(2 pi / n) / 4)^2) / n; an old vertex on two boundary edges
 * keeps 3/4 of itself and 1/8 of each boundary neighbour; a vertex in no
 * triangle keeps its position.
 *
 * Numbering (part of the interface): the old vertices keep their indices;
 * edges are numbered in the order in which they are first met when the
 * triangles are scanned in order, each triangle (a, b, c) contributing
 * (a, b), (b, c), (c, a); the vertex of edge e gets index n_old + e.
 * Triangle (a, b, c) with edge vertices ab, bc, ca becomes, in this order,
 * (a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca).
 *
 * Errors: every call returns an IPC_* status of ipc.h; messages from
 * ipc_dualmesh_last_error (NULL handle: the last failed create).
 */
#ifndef IPC_DUALMESH_H
#define IPC_DUALMESH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipc_dualmesh ipc_dualmesh;

/* Build W for `levels` (0 <= levels <= 6) levels of Loop subdivision of the
 * triangle mesh tri_host[n_tri][3] (vertex indices in [0, n_vert)), and the
 * fine triangles.  Host work only: device memory is taken at the first
 * ipc_dualmesh_apply, on hip_stream (nullable: the null stream).  Rejected
 * with IPC_E_INVALID: an index out of range, a triangle with a repeated
 * vertex, an edge in more than two triangles, a vertex on more than two
 * boundary edges, or more than 2^31 - 1 fine vertices, triangles or
 * nonzeros.  The arrays are copied; *out owns everything. */
int ipc_dualmesh_create(const int32_t *tri_host, int32_t n_tri, int32_t n_vert, int32_t levels, void *hip_stream,
                        ipc_dualmesh **out);
void ipc_dualmesh_destroy(ipc_dualmesh *m);
const char *ipc_dualmesh_last_error(const ipc_dualmesh *m);

enum {
    IPC_DM_NCOARSE = 0,   /* N_c                                               */
    IPC_DM_NFINE = 1,     /* N_f                                               */
    IPC_DM_NTRI = 2,      /* fine triangles (4^L n_tri)                        */
    IPC_DM_NNZ = 3,       /* nonzeros of W                                     */
    IPC_DM_MAXROW = 4     /* largest row of W                                  */
};
int ipc_dualmesh_query(const ipc_dualmesh *m, int what, int64_t *v);

/* Host copies: the fine triangles (tri_host[NTRI][3]); W in CSR form with
 * ascending columns per row (row_ptr[NFINE + 1], col[NNZ], val[NNZ];
 * any pointer may be NULL). */
int ipc_dualmesh_fine_tris(const ipc_dualmesh *m, int32_t *tri_host);
int ipc_dualmesh_weights(const ipc_dualmesh *m, int32_t *row_ptr, int32_t *col, double *val);

/* Eq. (7) for n_frames frames in one launch: xf_dev[f][i][k] =
 * sum_j W[i][j] xc_dev[f][j][k] for f < n_frames, i < N_f, k < 3 (device
 * arrays of n_frames x N_c x 3 and n_frames x N_f x 3 doubles, frame-major,
 * caller-owned).  Stream-ordered on the creation stream; returns before the
 * work is done. */
int ipc_dualmesh_apply(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames);

/* The same product for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * this entry point calls no hipMalloc, hipFree or other allocating routine.
 * W is staged in a fixed device array of 16 MiB per GPU that the library
 * holds until the process ends; a W that needs more (its CSR arrays, plus
 * the per-block column lists when every block fits the staged kernel, each
 * rounded up to 256 bytes) is rejected with IPC_E_CAPACITY.  Every call on
 * one GPU shares that array: it keeps the W of the last call (a call with the
 * same handle copies nothing, another handle's call copies its W from host
 * memory first), so calls that overlap on one GPU, from several host threads
 * or on different streams, race.  Arguments, results and errors are those of
 * ipc_dualmesh_apply; the calling thread's current device must be the one
 * the creation stream belongs to. */
int ipc_dualmesh_apply_noalloc(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames);

/* Duration of one ipc_dualmesh_apply launch, from `reps` back-to-back
 * launches between two HIP events on the creation stream; bytes = the
 * launch's algorithmic bytes (12 per nonzero of W and 4 per row pointer,
 * read once; 24 per coarse vertex read and 24 per fine vertex written, per
 * frame). */
int ipc_dualmesh_time(ipc_dualmesh *m, const double *xc_dev, double *xf_dev, int32_t n_frames, int32_t reps,
                      double *avg_us, double *bytes);

#ifdef __cplusplus
}
#endif

#endif
