/*
 * sfg.h -- C ABI of libsfg, the MI355X (gfx950) implementation of the
 * data-parallel hot path of SF-GRASS (Zhang, Zhao, Feng, "SF-GRASS:
 * Solver-Free Graph Spectral Sparsification", ICCAD 2020).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers unless the comment says (host).  The caller
 *   owns all memory; no entry point keeps a pointer after it returns.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is enqueued on it in order.  Entry points that return host scalars
 *   (marked "synchronises") wait for the stream before returning.
 * - Graphs are canonical undirected edge lists: u[e] < v[e], sorted by
 *   (u, v), no duplicates, node ids in [0, n), weights finite and > 0.  The
 *   edge id is the list index; every tie-break uses it.
 * - Blocks of vectors are n-by-k, row-major (node-major): element (p, c)
 *   at p*k + c.
 * - Status codes are returned; sfg_last_error() gives a message for the
 *   last non-OK status on the calling thread.  Asynchronous device faults
 *   surface as SFG_EHIP at the next call that checks the stream.  No C++
 *   exception crosses the ABI.
 * - The primitives (sfg_laplacian_csr, sfg_csr_select, sfg_smooth,
 *   sfg_edge_scores, sfg_select_topk and the affinity / coarsening calls)
 *   allocate nothing: the caller passes a workspace of at least
 *   sfg_workspace_bytes() bytes.  sfg_sparsify, sfg_spanning_tree,
 *   sfg_kappa_estimate and sfg_pcg allocate their
 *   buffers themselves, stream-ordered, in chunks of at least 256 MB.  When
 *   a call completes (its stream drained) its chunks go to a per-device
 *   cache of at most 16 GiB that later calls reuse, held until the process
 *   ends; a call that fails frees its chunks (stream-ordered) instead.  The
 *   device's default pool of stream-ordered memory is set to keep up to
 *   16 GiB of freed memory for reuse.
 * - Sizes: nnz = 2*(number of edges in the graph) must be < 2^31.
 */
#ifndef SFG_H_
#define SFG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFG_OK = 0,
    SFG_EINVAL = 1,        /* bad argument or malformed edge list */
    SFG_ENOTCONN = 2,      /* graph (or candidate sparsifier) is not connected */
    SFG_ENOMEM = 3,        /* device allocation failed (the calls that allocate) */
    SFG_EHIP = 4,          /* HIP runtime error; message has the HIP error string */
    SFG_EWORKSPACE = 5,    /* workspace smaller than sfg_workspace_bytes() */
    SFG_EUNSUPPORTED = 6,  /* valid request the library does not support (e.g. k > 64) */
    SFG_ENUMERIC = 7       /* NaN/Inf met in scores */
} sfg_status;

typedef enum { SFG_F64 = 0, SFG_F32 = 1, SFG_F16 = 2, SFG_BF16 = 3 } sfg_dtype;

/* Compressed sparse rows of the adjacency A of a weighted graph.  The
 * Laplacian L = D - A (Sec. 2.1) is implicit: deg holds D.  Columns are
 * ascending in every row.  A view: owns nothing. */
typedef struct {
    int64_t n;             /* rows (nodes) */
    int64_t nnz;           /* stored entries = 2 * edges */
    const int32_t *rowptr; /* [n+1] */
    const int32_t *col;    /* [nnz] */
    const void *val;       /* [nnz] of vt: edge weight */
    const int32_t *eid;    /* [nnz] edge id of each entry (may be NULL if unused) */
    const void *deg;       /* [n] of vt: weighted degree */
    sfg_dtype vt;          /* SFG_F64 or SFG_F32 */
} sfg_csr;

/* Operation codes for sfg_workspace_bytes. */
typedef enum {
    SFG_OP_LAPLACIAN_CSR = 0,
    SFG_OP_SMOOTH = 1,
    SFG_OP_SELECT_TOPK = 2,
    SFG_OP_AFFINITY = 3,
    SFG_OP_COARSEN = 4,
    SFG_OP_MPNN_FORWARD = 5,   /* n nodes, t = activation dtype */
    SFG_OP_MPNN_TRAIN = 6,     /* n nodes, m = scored edges */
    SFG_OP_COLOR = 7,          /* n nodes */
    SFG_OP_TREE_ORDER = 8,     /* n nodes, m edges */
    SFG_OP_TREE_SOLVE = 9,     /* n nodes, k columns */
    SFG_OP_CSR_SELECT = 10,    /* n nodes, m = edges of the whole graph */
    SFG_OP_MPNN_NORM = 11,     /* no sizes: a fixed 512 bytes */
    SFG_OP_SMOOTH_ORDERED = 12 /* n nodes, k columns, t = storage dtype */
} sfg_op;

/* Which graph's embedding scores the candidates (Sec. 3.5 derives the score
 * from eigenvectors of the current sparsifier; Alg. 1 embeds the graph). */
typedef enum { SFG_EMBED_SPARSIFIER = 0, SFG_EMBED_GRAPH = 1 } sfg_embed;
typedef enum { SFG_SMOOTH_JACOBI = 0, SFG_SMOOTH_GAUSS_SEIDEL = 1 } sfg_smoother;

/* Workspace (bytes) needed by an operation.  For SFG_OP_LAPLACIAN_CSR, m is
 * the edge count; for SFG_OP_SMOOTH, n, k and t (the storage dtype); for
 * SFG_OP_SELECT_TOPK, m is the candidate count; for SFG_OP_AFFINITY, n, k;
 * for SFG_OP_COARSEN, n, m, k. */
size_t sfg_workspace_bytes(int op, int64_t n, int64_t m, int32_t k, sfg_dtype t);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *sfg_last_error(void);

/*
 * Build the CSR of the adjacency and the degree vector of the graph
 * (Sec. 2.1: A(p,q) = w(p,q); D(p,p) = sum of the weights at p).
 *   n, m        nodes, edges of the canonical edge list u, v, w (wt = F64|F32)
 *   mask        optional [m] uint8: only edges with mask[e] != 0 are included
 *               (NULL = all), e.g. the spanning tree or current sparsifier
 *   rowptr      out [n+1] int32
 *   col, eid    out [nnz] int32, nnz = 2 * included edges; columns ascend in a
 *               row, so entries of a row are in ascending edge id
 *   val         out [nnz] of wt (the edge weight)
 *   deg         out [n] of wt; summed in FP64 in ascending edge id, then
 *               stored in wt
 *   nnz_out     (host, may be NULL) receives nnz; synchronises when non-NULL
 * Errors: SFG_EINVAL on bad sizes/dtypes, SFG_EWORKSPACE.
 */
sfg_status sfg_laplacian_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                             const void *w, sfg_dtype wt, const uint8_t *mask,
                             int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg,
                             int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream);

/*
 * The CSR of a subgraph of G (the edges e with mask[e] != 0; L = D - A as in
 * Sec. 2.1), taken from G's CSR instead of the edge list: row p keeps, in
 * their stored order, the entries whose edge id is in the mask, and its
 * degree is their sum, added in FP64 in column order and rounded once.  The
 * result is bit-identical to sfg_laplacian_csr with the same mask (same
 * rowptr, col, val, eid and deg).  Used where G's CSR exists already (the
 * surrogate aggregates over G and embeds on the spanning tree).
 *   G        device CSR of the whole graph as sfg_laplacian_csr builds it
 *            (eid required), F64 or F32
 *   mask     [m] uint8, edge e kept iff mask[e] != 0 (m = the number of edges
 *            G was built from; every eid of G must index it)
 *   rowptr   out [n+1]; col, val (G's dtype), eid: out, room for the kept
 *            entries (2 x kept edges; G->nnz always suffices); deg out [n]
 *   nnz_out  host, may be NULL: if given, the call synchronises and returns
 *            rowptr[n]
 * Workspace: sfg_workspace_bytes(SFG_OP_CSR_SELECT, n, m, 0, 0) with m =
 * G->nnz / 2.  Errors: SFG_EINVAL (null pointers, a CSR without eid, an odd
 * nnz, a weight type other than F64 or F32), SFG_EWORKSPACE.
 */
sfg_status sfg_csr_select(const sfg_csr *G, const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val,
                          int32_t *eid, void *deg, int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream);

/*
 * Local spectral embedding (Sec. 3.2): make the k random vectors x0
 * orthogonal to the all-one vector (subtract each column's mean), then apply `sweeps` damped
 * Jacobi relaxations of L x = 0:
 *     x_p <- (1 - omega) x_p + omega * (sum_q A_pq x_q) / D_pp
 * with the row sum taken in ascending column order.
 * Column mean: the column is summed in double-double arithmetic (Knuth's
 * two-sum, about 106 significant bits), the double-double total rounded once
 * to FP64 and divided by n.  That equals the exactly rounded sum divided by n
 * unless the column cancels to within about 2^-100 of the magnitude of its
 * partial sums (the error of the double-double sum then reaches the FP64
 * rounding boundary); columns of random starting vectors are far from that.
 *   H          graph to smooth (vt F64 when storage is F64, else F32)
 *   k          1..64 vectors; sweeps >= 0; 0 < omega <= 1 (0.5 damps the
 *              top of the spectrum of bipartite graphs)
 *   x0         [n*k] FP64, not modified
 *   storage    element type of the iterates: F64 (FP64 arithmetic) or
 *              F32/F16/BF16 (FP32 arithmetic, rounding to nearest even on
 *              every store)
 *   final_f32  when storage is F16/BF16: store the last iterate in FP32
 *   x          out [n*k] of storage (of F32 when final_f32)
 * Errors: SFG_EINVAL, SFG_EUNSUPPORTED (k > 64 or an unsupported
 * combination), SFG_EWORKSPACE.
 */
sfg_status sfg_smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega,
                      const double *x0, sfg_dtype storage, int32_t final_f32, void *x,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * sfg_smooth with the rows taken in a given order, several sweeps per pass
 * over the block where the graph allows: the same result, bit for bit.  The
 * rows are split into blocks of 64 consecutive entries of `order`.  A layout
 * pass gives each block its h-hop neighbourhood (h = 2 in FP64, 3 in FP32,
 * fewer when a block exceeds the LDS capacities below) and a local copy of
 * the rows it needs.  For each block a workgroup then loads the current iterate of the
 * block's rows and of that neighbourhood into LDS, forms up to h sweeps there
 * (sweep j for the rows within h - j hops of the block) and writes the last
 * one for the block only, so the block X is read about once and written once
 * per h sweeps.  Every row is formed with sfg_smooth's arithmetic (entries in
 * stored order, the same epilogue, every intermediate iterate rounded to the
 * storage type).  The order decides how small the neighbourhoods are: a
 * spanning tree's preorder (sfg_tree_order) keeps them to a few hundred rows
 * on meshes and power grids.
 *   order         [n] int32 (device): a permutation of the nodes (checked
 *                 whenever the passes run; unused, and not read, otherwise)
 *   per_pass_out  (host, may be NULL): the sweeps each pass took, 2 to 4; 1 if
 *                 the call ran sfg_smooth instead: sweeps x k x (bytes of a
 *                 storage value) under 320 (a narrow block's few sweeps do
 *                 not repay the layout pass), k not a multiple of 4 or
 *                 over 128 bytes per row (F16/BF16: over 16 columns), fewer
 *                 than 2 sweeps, a reduced-precision row over 256 entries
 *                 (sfg_smooth sums those by lane groups), or a block whose
 *                 2-hop layout exceeds the capacities (168 rows in all, 112
 *                 within one hop, 288 local entries; 4 hops: 288, 224 within
 *                 three hops, 512; 3 hops: 224, 160, 384).  The environment
 *                 variable SFG_SWEEP_HOPS (2, 3 or 4, read at every call) caps
 *                 h and takes the passes at any width; 0 forces sfg_smooth
 *   other arguments as sfg_smooth
 * Workspace: sfg_workspace_bytes(SFG_OP_SMOOTH_ORDERED, n, 0, k, storage).
 * Synchronises once per layout tried (to learn whether every block fits).
 * Errors: those of sfg_smooth; SFG_EINVAL when the passes would run and order
 * is not a permutation.
 */
sfg_status sfg_smooth_ordered(const sfg_csr *H, const int32_t *order, int32_t k, int32_t sweeps, double omega,
                              const double *x0, sfg_dtype storage, int32_t final_f32, void *x, int32_t *per_pass_out,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * Random test vectors for the embedding (Sec. 3.2 smooths random vectors),
 * drawn on the device: x0[i][c] (row-major, n-by-k, FP64) standard normal from
 * the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * SC'11) with Box-Muller.  Element pair j (elements 2j, 2j+1) takes counter
 * (lo32 j, hi32 j, block, 0) and key (lo32 seed, hi32 seed); with output words
 * r0..r3, u1 = ((r0:r1) >> 11) 2^-53, u2 = ((r2:r3) >> 11) 2^-53,
 * rho = sqrt(-2 log(1 - u1)), z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2).
 * The integer part is exact; the logarithm and trigonometric functions are
 * the device math library's (within a few ulp of a host libm).
 *   x0   out [n*k] FP64 (device)
 * Errors: SFG_EINVAL.
 */
sfg_status sfg_random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *x0, void *stream);

/*
 * Multicolouring for the Gauss-Seidel reading of the smoother (Sec. 3.2
 * relaxes L x = 0 by Gauss-Seidel steps).  Jones-Plassmann rounds with the
 * fixed priority (h(p), p), h(x) the integer mixer x ^= x>>16, x *= 0x7feb352d,
 * x ^= x>>15, x *= 0x846ca68b, x ^= x>>16 (32-bit): in round r each uncoloured
 * node whose priority exceeds that of all its uncoloured neighbours takes the
 * smallest colour unused by neighbours coloured in earlier rounds.
 *   H           graph (its structure only)
 *   color       out [n] int32 colour of each node (adjacent nodes differ)
 *   class_rows  out [n] int32: the nodes of colour 0, then 1, ..., each class
 *               in ascending node order
 *   class_ptr   out [n + 1] int32 (device): the first ncolors + 1 entries are
 *               the class offsets into class_rows
 *   ncolors     (host) out: number of colours
 * Workspace: sfg_workspace_bytes(SFG_OP_COLOR, n, 0, 0, 0).  Synchronises
 * once per round.  Errors: SFG_EINVAL, SFG_EWORKSPACE, SFG_EHIP.
 */
sfg_status sfg_color(const sfg_csr *H, int32_t *color, int32_t *class_rows, int32_t *class_ptr, int32_t *ncolors,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * Gauss-Seidel reading of the smoother (Sec. 3.2): centre x0 as sfg_smooth
 * does, then `sweeps` sweeps, each updating the colour classes in order, in
 * place, every row with sfg_smooth's arithmetic over the current values:
 *     x_p <- (1 - omega) x_p + omega * (sum_q A_pq x_q) / D_pp
 * (omega = 1: plain Gauss-Seidel).  Rows of one class are never adjacent, so
 * the order inside a class does not matter.
 *   class_rows, class_ptr, ncolors   from sfg_color on the same H
 *   storage    F64 or F32 (H's values of the same type); x out [n*k]
 * Workspace: sfg_workspace_bytes(SFG_OP_SMOOTH, n, 0, k, storage).
 * Synchronises once.  Errors: SFG_EINVAL, SFG_EUNSUPPORTED, SFG_EWORKSPACE.
 */
sfg_status sfg_smooth_gs(const sfg_csr *H, const int32_t *class_rows, const int32_t *class_ptr, int32_t ncolors,
                         int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage, void *x,
                         void *ws, size_t ws_bytes, void *stream);

/*
 * Edge scores (Eq. 18 with the smoothed block in place of eigenvectors;
 * Alg. 1's edge distortion): s_e = w_e * sum_c (x_pc - x_qc)^2 over the k
 * columns, c ascending.
 *   x, xt      smoothed block [n*k] (F64, F32, F16 or BF16)
 *   ne         number of scored edges
 *   cand       optional [ne] edge ids into u, v, w (NULL: edge i is scored)
 *   u, v, w    edge list (wt = F64 or F32)
 *   score, st  out [ne]: F64 (requires xt = F64 and wt = F64, FP64
 *              arithmetic) or F32 (FP32 arithmetic)
 */
sfg_status sfg_edge_scores(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t ne,
                           const int32_t *cand, const int32_t *u, const int32_t *v,
                           const void *w, sfg_dtype wt, void *score, sfg_dtype st, void *stream);

/*
 * Top-k selection (Alg. 1, "include top few edges with large distortion"):
 * order the ne scores by value descending, then position ascending (callers
 * keep candidates in ascending edge id, so this is edge id ascending), and
 * mark the first k.
 *   score, st  [ne] F64 or F32 values (any sign; NaN is an error)
 *   sel        out [ne] uint8: 1 if chosen else 0
 *   tau        out (device, 1 double): the k-th largest score (+inf if k = 0)
 *   tau_host   (host, may be NULL) receives tau; synchronises when non-NULL
 * Errors: SFG_EINVAL when k > ne; SFG_ENUMERIC on a NaN (reported through
 * tau_host, or as a NaN tau when tau_host is NULL).
 */
sfg_status sfg_select_topk(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel,
                           double *tau, double *tau_host, void *ws, size_t ws_bytes, void *stream);

/*
 * sfg_select_topk without a workspace and without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments (minus the
 * workspace), same kernels, same results.  Its scratch (selection state,
 * digit histogram, the keys a radix pass copies, per-tile tie counts) is a device array of
 * 128 MiB (134217728 bytes) in the library, one copy per GPU, held from the
 * first call on that GPU until the process ends.  The first call on a device
 * looks up that copy's address (hipGetSymbolAddress) with the device current;
 * later calls only launch kernels.  The current device must be the one that
 * `stream` belongs to.
 *   ne     accepted while sfg_workspace_bytes(SFG_OP_SELECT_TOPK, 0, ne, 0,
 *          st) <= 134217728, i.e. up to about 16.7 million scores
 * Every call on a GPU uses that GPU's one array, and each call clears what it
 * needs: calls that overlap on one GPU (two streams, or two host threads)
 * race on it and must be serialised by the caller.
 * Errors: SFG_EUNSUPPORTED when ne is above the limit (nothing is launched),
 * otherwise those of sfg_select_topk.
 */
sfg_status sfg_select_topk_noalloc(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel,
                                   double *tau, double *tau_host, void *stream);

/*
 * Maximum-weight spanning tree (the MST the paper uses in place of a
 * low-stretch tree, Sec. 3.4): the unique tree that Kruskal's rule picks
 * under the order (weight descending, edge id ascending).
 *   allowed    optional [m] uint8 restricting the usable edges (NULL = all);
 *              with a restriction the result is a spanning forest
 *   in_tree    out [m] uint8: 1 for tree edges
 *   n_comp     (host) receives the number of components of the forest;
 *              synchronises
 * Runs Boruvka rounds on the device (integer atomics only, deterministic).
 * Errors: SFG_ENOMEM, SFG_EHIP.  (Allocates internally: see the conventions.)
 */
sfg_status sfg_spanning_tree(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                             const void *w, sfg_dtype wt, const uint8_t *allowed,
                             uint8_t *in_tree, int64_t *n_comp, void *stream);

/*
 * Node affinity of the algebraic-distance type used to form aggregation
 * sets (Sec. 3.2): with xb = x minus its column means,
 *     a_pq = (xb_p . xb_q)^2 / (|xb_p|^2 |xb_q|^2),   0 if a norm is 0.
 *   x, xt      smoothed block [n*k] (F64 or F32)
 *   aff        out [m] of at (F64 requires xt F64; else F32)
 */
sfg_status sfg_affinity(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t m,
                        const int32_t *u, const int32_t *v, void *aff, sfg_dtype at,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * One spectral-coarsening step (Sec. 3.2-3.3, Eqs. 3-5): aggregation sets
 * from the affinities, then the Galerkin coarse graph L_c = H+^T L H+.
 * Aggregation rule (the paper leaves it open): every node points to the
 * neighbour with the largest (affinity, weight, -id); aggregates are the
 * connected components of these pointers, numbered by smallest member.
 *   G          CSR of the graph (with eid); vt F64 or F32
 *   m,u,v,w,wt its canonical edge list
 *   aff, at    [m] edge affinities (F64 or F32)
 *   agg        out [n] aggregate id of each node
 *   n_coarse   (host) out: number of aggregates; synchronises
 *   m_coarse   (host) out: number of coarse edges
 *   cu,cv,cw   out [<= m] canonical coarse edge list (cw of wt: sums of
 *              fine weights, added in ascending fine edge id, in FP64)
 *   crep       out [<= m] per coarse edge, the heaviest fine edge between
 *              the two aggregates (ties: smallest id), kept by the
 *              backward mapping of Sec. 3.4
 */
sfg_status sfg_coarsen(const sfg_csr *G, int64_t m, const int32_t *u, const int32_t *v,
                       const void *w, sfg_dtype wt, const void *aff, sfg_dtype at,
                       int32_t *agg, int64_t *n_coarse, int64_t *m_coarse, int32_t *cu,
                       int32_t *cv, void *cw, int32_t *crep, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Spanning tree rooted at node 0, in depth-first preorder (views; owns
 * nothing).  The walk from the root crosses every tree edge once down and
 * once up; at each node it takes the neighbours in ascending id order,
 * starting after the neighbour it came from (the root starts at its smallest
 * neighbour).  A subtree is the contiguous preorder range [i, i + size[i]).
 * Used by the condition-number estimate (Eq. 2) as the preconditioner of
 * solves with the sparsifier Laplacian.
 */
typedef struct {
    int64_t n;
    const int32_t *order;  /* [n] node at preorder position i; order[0] = 0 */
    const int32_t *parent; /* [n] preorder position of the parent; -1 at the root */
    const int32_t *size;   /* [n] nodes in the subtree */
    const double *pw;      /* [n] weight of the edge to the parent; 0 at the root */
    const int32_t *tdown;  /* [n] walk step (0 .. 2n-3) entering the node; -1 at the root */
    const int32_t *tup;    /* [n] walk step leaving it; -1 at the root */
} sfg_tree;

/*
 * Preorder layout of the spanning tree formed by the edges with keep[e] == 1
 * (the marking sfg_sparsify gives its tree).
 *   n, m, u, v       canonical edge list; w of wt (must be SFG_F64)
 *   keep             [m] uint8; exactly n - 1 edges equal 1
 *   order, parent, size, tdown, tup  out [n] int32; pw out [n] double
 *   ws               >= sfg_workspace_bytes(SFG_OP_TREE_ORDER, n, m, 0, SFG_F64)
 * Synchronises.  Errors: SFG_EINVAL (count of marked edges is not n - 1,
 * bad sizes, null pointer), SFG_ENOTCONN (the marked edges do not form a
 * spanning tree), SFG_EWORKSPACE, SFG_EHIP.
 */
sfg_status sfg_tree_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                          const uint8_t *keep, int32_t *order, int32_t *parent, int32_t *size, double *pw,
                          int32_t *tdown, int32_t *tup, void *ws, size_t ws_bytes, void *stream);

/*
 * x = L_T^+ b for each of the k columns (the pseudo-inverse of the tree
 * Laplacian, Sec. 2.1): b is projected onto the complement of the all-one
 * vector, the system is solved exactly (net demand below each edge, then
 * potentials down from the root) and x has zero column means.
 *   T      tree from sfg_tree_order
 *   b, x   n-by-k FP64, node order; x may alias b
 *   ws     >= sfg_workspace_bytes(SFG_OP_TREE_SOLVE, n, 0, k, SFG_F64)
 * Asynchronous.  Errors: SFG_EINVAL (k outside 1..64, null pointer),
 * SFG_EWORKSPACE.
 */
sfg_status sfg_tree_solve(const sfg_tree *T, int32_t k, const double *b, double *x, void *ws, size_t ws_bytes,
                          void *stream);

/* Parameters of the condition-number estimate (host struct). */
typedef struct {
    int32_t k;             /* block width, 1..32 and <= n - 1 (0 = 8) */
    int32_t steps;         /* subspace-iteration steps, 1..64 (0 = 6) */
    double tol;            /* inner solves: stop a column when ||r|| <= tol ||rhs|| (0 = 1e-1: the power grid's
                              estimate moves by 1e-4 against 1e-2, with 40% fewer iterations) */
    int32_t max_iter;      /* inner solves: iteration cap per solve (0 = 20000) */
    uint64_t seed;         /* with y0 == NULL: starting block sfg_random_block(n, k, seed, block) */
    uint32_t block;
} sfg_kappa_params;

typedef struct {
    double kappa;          /* estimate after the last step */
    double ritz[64];       /* largest Ritz value after each step */
    int32_t steps;
    int64_t inner_iters;   /* preconditioned CG iterations over all steps */
    int32_t max_inner;     /* most iterations of one solve */
    int32_t unconverged;   /* solves that reached max_iter */
    float ms;              /* wall time of the call */
} sfg_kappa_report;

/*
 * Estimate of the relative condition number kappa(L_G, L_P) of Eq. 2 for a
 * sparsifier P of G (P = the edges with keep[e] != 0, kept with G's
 * weights).  Since L_P <= L_G the smallest eigenvalue of the pencil is at
 * least 1, so kappa <= lambda_max; the estimate is the largest Ritz value of
 * the pencil on the subspace after `steps` steps of Y <- L_P^+ L_G Y, which
 * never exceeds lambda_max (Courant-Fischer) and approaches it from below.
 * Solves with L_P run preconditioned conjugate gradients, the preconditioner
 * being the exact solve with P's spanning tree (edges with keep[e] == 1).
 *   n, m, u, v, w    canonical edge list of G, w of wt (F64 or F32)
 *   keep             [m] uint8: 0 not in P, 1 tree edge of P, 2 other edge of P
 *   kp               (host) parameters
 *   y0               n-by-k FP64 starting block, or NULL (drawn from kp->seed)
 *   rep              (host, may be NULL) per-step values and iteration counts
 *   kappa            (host) out: the estimate
 * Allocates its buffers internally (see the conventions).
 * Synchronises.  Errors: SFG_EINVAL, SFG_ENOTCONN (the edges marked 1 are not
 * a spanning tree), SFG_ENUMERIC (the block lost rank), SFG_ENOMEM, SFG_EHIP.
 */
sfg_status sfg_kappa_estimate(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                              sfg_dtype wt, const uint8_t *keep, const sfg_kappa_params *kp, const double *y0,
                              double *kappa, sfg_kappa_report *rep, void *stream);

/* Report of sfg_pcg (host). */
typedef struct {
    int64_t iters;         /* outer CG iterations */
    int64_t inner_iters;   /* tree-preconditioned CG iterations of all preconditioner solves */
    double relres;         /* ||r|| / ||b|| at the end */
    float ms;              /* wall time of the call */
    int32_t converged;     /* relres <= tol */
    int32_t inner_capped;  /* a preconditioner solve reached its iteration cap */
} sfg_pcg_report;

/*
 * The sparsifier's downstream use in the paper's evaluation (Sec. 4, Table 3):
 * conjugate gradients on L_G x = b grounded at node 0 (row and column 0
 * removed, x_0 = 0), preconditioned by the sparsifier: every preconditioner
 * application solves the grounded L_P system, by the tree-preconditioned
 * conjugate gradients of sfg_kappa_estimate to a relative residual of 1e-6
 * (in effect an exact solve for an outer tolerance of 1e-3 or more; an FP64
 * solve of a large tree Laplacian cannot go much below that in residual).  Stops when ||r|| <= tol ||b|| or after
 * max_iter iterations.  FP64 throughout.
 *   u, v, w, wt  the graph's canonical edge list (F64 or F32 weights)
 *   keep     [m] uint8: sparsifier edges != 0, its spanning tree marked 1
 *            (the output of sfg_sparsify)
 *   b        device [n] FP64 right-hand side; b[0] is ignored
 *   x        device [n] FP64 out (x[0] = 0), may be NULL
 *   tol      in (0, 1); max_iter >= 1
 *   rep      host, may be NULL
 * Allocates stream-ordered and synchronises (a host check per iteration).
 * Errors: SFG_EINVAL (arguments; the edges marked 1 not a spanning tree),
 * SFG_EUNSUPPORTED (2m >= 2^31).
 */
sfg_status sfg_pcg(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                   const uint8_t *keep, const double *b, double *x, double tol, int32_t max_iter,
                   sfg_pcg_report *rep, void *stream);

/* Parameters of sfg_sparsify (host struct). */
typedef struct {
    int32_t levels;        /* 1 = spanning tree + one scoring pass; >1 = Alg. 1 hierarchy */
    int32_t k;             /* vectors per embedding, 1..64 */
    int32_t sweeps;        /* smoothing sweeps per embedding */
    double omega;          /* damping, 0 < omega <= 1 */
    double frac;           /* recovered fraction f of each level's candidates: k_sel = ceil(f * n_cand) */
    int32_t embed;         /* sfg_embed */
    sfg_dtype storage;     /* iterate storage: F64, F32, F16, BF16 */
    int32_t final_f32;     /* F16/BF16: last iterate in FP32 */
    double band;           /* F16/BF16/F32: relative margin m of FP64 re-scoring around the threshold (0 = none) */
    int32_t rounds;        /* single level: multi-round densification, 1..16 (0 = 1).  The budget
                              ceil(frac * off-tree edges) is split into near-equal quotas; round r smooths
                              block r of x0 on the current sparsifier (tree + edges added so far; its
                              Laplacian is the one the perturbation analysis of Sec. 3.5 is about) and adds
                              its quota's top-scored edges outside it.  x0 then holds rounds * n * k values
                              and the report has one entry per round. */
    int32_t smoother;      /* sfg_smoother: damped Jacobi (default) or multicolour Gauss-Seidel; Gauss-Seidel
                              needs F64 or F32 storage and no band */
    uint64_t seed;         /* with x0 == NULL: blocks drawn on the device by sfg_random_block(seed, index) */
    double sigma;          /* > 0: sigma-driven stopping (single level).  Starting from the tree, while the
                              condition-number estimate exceeds sigma^2 (Eq. 2) and fewer than `rounds`
                              batches (0 = 16) were added, add the next ceil(frac * off-tree edges) top-scored
                              edges, scored on the sparsifier grown so far; batch r smooths block r of x0.
                              Estimate j starts from sfg_random_block(n, est.k, seed, 64 + j). */
    sfg_kappa_params est;  /* estimate parameters (seed and block are ignored here) */
    const struct sfg_surrogate *surrogate;   /* host, may be NULL: see sfg_surrogate */
    double cand_frac;      /* with a surrogate: fraction of the off-tree edges scored exactly (0 < cand_frac <= 1) */
} sfg_params;

/* A trained edge-criticality model (not in the paper) that prunes the candidates
 * of a single-level sparsify.  Callers: those who trade a little recall of the
 * plain selection for skipping exact scores of most off-tree edges.  With
 * sfg_params.surrogate set, sfg_sparsify (levels = 1, one round, no sigma,
 * Jacobi, the sparsifier embedding, no band, F32 or F64 storage):
 *   1. G's CSR and the spanning tree's, FP32 weights;
 *   2. the cheap embedding: the first kc columns of x0, centred and smoothed
 *      tc times on the tree (omega 1/2, BF16 storage, FP32 last iterate);
 *   3. node and edge features (sfg_mpnn_features with `norm`) and one BF16
 *      inference (sfg_mpnn_forward) over the off-tree edges;
 *   4. the top ceil(cand_frac * off-tree edges) by prediction (ties: lower
 *      edge id) are scored exactly as the plain path scores them (k vectors,
 *      `sweeps` sweeps on the tree, storage and omega of sfg_params);
 *   5. of those, the top min(ceil(frac * off-tree edges), scored) are kept.
 * If a parameter or normalisation value is not finite, the plain path runs
 * instead and the level report says so (surrogate_fallback = 1). */
typedef struct sfg_surrogate {
    const float *params;   /* device [sfg_mpnn_param_count()] FP32 */
    const float *norm;     /* device [24] FP32: node feature means, inverse stds, edge means, inverse stds */
    int32_t kc;            /* vectors of the cheap embedding, 1..k */
    int32_t tc;            /* its sweeps, >= 0 */
} sfg_surrogate;

/* Per-level report (host). */
typedef struct {
    int64_t n, m;          /* level graph size */
    int64_t n_cand;        /* off-subgraph candidates */
    int64_t k_sel;         /* edges recovered */
    double tau;            /* k_sel-th largest score */
    int64_t band;          /* edges re-scored in FP64 (precision form) */
    int64_t band_above;    /* edges accepted above the band */
    int32_t band_rounds;   /* margin doublings needed */
    float ms_smooth, ms_score, ms_select, ms_other;
    int64_t cone_rows;     /* row updates spent on FP64 re-scoring (sum over sweeps) */
    int32_t precision_fallback;   /* F16/BF16/F32 with a band: 1 when the re-scoring cone predicted for the
                                     expected band exceeded a quarter of the full pass, so the level ran the
                                     FP64 path instead (same selection, no reduced-precision pass) */
    int32_t node_order;   /* numbering the level was swept in: 0 the input's, 1 the spanning tree's preorder.
                             Single level (Jacobi smoother): taken when the call plans at least 512 sweep
                             launches of 8-column parts over all its batches, n >= 65536, and more than a
                             quarter of the scoring graph's entries lie over 4096 rows from their own row.
                             Hierarchy (levels > 1): per level, the preorder of a spanning tree of G_l, for the
                             sweeps on G_l and on the level's sparsifier, when n_l >= 65536, the level's block
                             of k vectors exceeds 96 MiB (256 MiB on the coarse levels, whose spanning tree is
                             computed for it) and more than half of G_l's entries lie over 4096 rows from their
                             own row.  The environment variable SFG_NODE_ORDER=0 / 1 forces
                             either.  Results are bit-identical either way: rows keep their entry order */
    int64_t n_scored;      /* candidates scored exactly (n_cand, or the surrogate's share) */
    int32_t surrogate_fallback;   /* a surrogate was given but was not usable: the plain path ran */
    int32_t sweeps_per_pass;      /* Jacobi sweeps the level's scoring smoothing took per pass over the block: 1,
                                     or 2 to 4 when the level was swept in the tree's preorder and
                                     sfg_smooth_ordered's passes paid (same bits either way) */
} sfg_level_report;

typedef struct {
    int32_t levels;
    sfg_level_report level[16];   /* index 0 = finest */
    int32_t n_kappa;              /* sigma mode: estimates made (batches added + 1) */
    double kappa[17];             /* sigma mode: estimate of the tree, then after each batch */
    int64_t kappa_inner_iters;    /* sigma mode: inner iterations of all estimates */
    float ms_kappa;               /* sigma mode: time spent estimating */
} sfg_report;

/*
 * Spectral sparsifier P of G (the problem of Sec. 2.2 and Alg. 1):
 * levels = 1: maximum-weight spanning tree, embed (sparsifier = the tree, or
 *   the graph), score the off-tree edges, add the top ceil(f * n_cand); with
 *   rounds R > 1 that budget is added in R near-equal quotas, each after
 *   re-embedding on the sparsifier grown so far (x0 holds R blocks).
 * levels > 1: Alg. 1 -- coarsen G_0..G_{levels-1}, P_last = G_last, then for
 *   each finer level map the sparsifier back (per-aggregate spanning trees and
 *   the heaviest fine edge of each coarse sparsifier edge) and add the top
 *   f of that level's off-subgraph edges.
 *   x0         random blocks, FP64: level l uses rows [0, N_l) of the n-by-k
 *              block at x0 + l*n*k  (caller draws levels*n*k values; with
 *              rounds R > 1, block r for round r); NULL: block i is drawn
 *              on the device by sfg_random_block(n, k, p->seed, i)
 *   keep       out [m] uint8: 0 not in P, 1 in P before the final additions
 *              (the tree, or the mapped sparsifier), 2 recovered at level 0
 *              (in any round)
 *   rep        (host, may be NULL) per-level report (per round when R > 1)
 * Synchronises.  Errors: SFG_EINVAL, SFG_ENOTCONN, SFG_ENOMEM, SFG_EHIP,
 * SFG_EUNSUPPORTED.
 */
sfg_status sfg_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                        sfg_dtype wt, const sfg_params *p, const double *x0, uint8_t *keep,
                        sfg_report *rep, void *stream);

/*
 * Learned edge-criticality surrogate (not in the paper: an addition that
 * predicts which candidates the scores of Eq. 18 will rank highest, so that
 * most of them can be pruned before exact scoring).  Two message-passing
 * layers of width 32 over G, with the row-normalised aggregation D^-1 A of
 * Sec. 3.2's smoothing, then an edge head:
 *   H1 = relu([X | D^-1 A X | 1] W1),  H2 = relu([H1 | D^-1 A H1 | 1] W2),
 *   yhat_e = [relu([|H2_p - H2_q| | H2_p * H2_q | f_e | 1] W3) | 1] . w4
 * Parameters: one F32 vector [W1 (17x32) | W2 (65x32) | W3 (69x32) | w4 (33)],
 * row-major, sfg_mpnn_param_count() values.  The graph CSR must be F32.
 */
int64_t sfg_mpnn_param_count(void);

/* Features from a cheap smoothed block xc (n x kc, F32):
 *   node (n x 8): 1, log D_G, log D_T, log deg_G, log deg_T, log |xc_p|^2,
 *                 log local energy sum_q w_pq |xc_p - xc_q|^2 / D_p on G, on T
 *   edge (ne x 4): log w, log w |xc_p - xc_q|^2, min and max of log D_T at the ends
 * standardised as (f - mean) * inv_std with norm = [node means (8), node
 * inverse stds (8), edge means (4), edge inverse stds (4)] (NULL: raw;
 * node feature 0 stays 1).  cand (NULL = all edges) selects the edges. */
sfg_status sfg_mpnn_features(const sfg_csr *G, const sfg_csr *T, const float *xc, int32_t kc, int64_t ne,
                             const int32_t *cand, const int32_t *u, const int32_t *v, const float *w,
                             const float *norm, float *node_feat, float *edge_feat, void *stream);

/* Inference: predictions pred[ne] for the candidate edges; activations are
 * stored as act (F32 or BF16) with FP32 arithmetic.  Workspace:
 * sfg_workspace_bytes(SFG_OP_MPNN_FORWARD, n, 0, 0, act). */
sfg_status sfg_mpnn_forward(const sfg_csr *G, const float *params, const float *node_feat, int64_t ne,
                            const int32_t *cand, const int32_t *u, const int32_t *v, const float *edge_feat,
                            sfg_dtype act, float *pred, void *ws, size_t ws_bytes, void *stream);

/* Training step core, FP32: forward, loss = mean_e (pred_e - target_e)^2
 * (device scalar), and its gradient grad[param_count] with respect to the
 * parameters.  Deterministic (no floating-point atomics).  Workspace:
 * sfg_workspace_bytes(SFG_OP_MPNN_TRAIN, n, ne, 0, SFG_F32). */
sfg_status sfg_mpnn_loss_grad(const sfg_csr *G, const float *params, const float *node_feat, int64_t ne,
                              const int32_t *cand, const int32_t *u, const int32_t *v, const float *edge_feat,
                              const float *target, float *pred, float *loss, float *grad, void *ws,
                              size_t ws_bytes, void *stream);

/* Adam update (Kingma & Ba) with bias correction, step >= 1, in place on
 * params, m, v (all F32, n values). */
sfg_status sfg_mpnn_adam(float *params, const float *grad, float *m, float *v, int64_t n, int64_t step,
                         double lr, double beta1, double beta2, double eps, void *stream);

/* Standardisation of a training set of `ngraphs` graphs (host arrays of
 * device pointers): per column, the mean and the population standard
 * deviation over all rows of all graphs, summed in FP64 in a fixed order
 * (deterministic), in two passes (means, then squared deviations).
 *   node_feat[i]  device n_i x 8 F32 raw node features (sfg_mpnn_features with
 *                 norm = NULL), node_rows[i] = n_i >= 1
 *   edge_feat[i]  device e_i x 4 F32 raw edge features; target[i] device e_i F32
 *                 targets; edge_rows[i] = e_i >= 1
 *   norm          out, device 24 F32 in the layout sfg_mpnn_features takes:
 *                 node means, node 1/max(std, 1e-6), edge means, edge
 *                 1/max(std, 1e-6); node feature 0 (the constant) gets 0 and 1
 *   ystat         out, device 2 doubles: target mean and standard deviation (1
 *                 when every target is equal)
 *   ws            >= sfg_workspace_bytes(SFG_OP_MPNN_NORM, 0, 0, 0, 0) bytes
 * Errors: SFG_EINVAL, SFG_EWORKSPACE. */
sfg_status sfg_mpnn_fit_norm(int32_t ngraphs, const float *const *node_feat, const int64_t *node_rows,
                             const float *const *edge_feat, const float *const *target, const int64_t *edge_rows,
                             float *norm, double *ystat, void *ws, size_t ws_bytes, void *stream);

/* out[i] = (y[i] - ystat[0]) / ystat[1], in FP64 and rounded to F32 (the
 * standardised training targets); out may alias y. */
sfg_status sfg_mpnn_standardize(const float *y, int64_t n, const double *ystat, float *out, void *stream);

/* What a model file records besides its parameters and normalisation. */
typedef struct {
    int32_t kc;            /* vectors of the cheap embedding, 1..64 */
    int32_t tc;            /* its sweeps, 0..1000 */
    double y_mean, y_std;  /* target standardisation the model was trained with */
} sfg_mpnn_meta;

/* Model file of the surrogate, so that a C caller can store and reuse a
 * trained model.  Version 1, little-endian: magic "SFGMPNN1"; uint32 version,
 * parameter count, normalisation count (24); int32 kc, tc; uint32 0; double
 * y_mean, y_std; the F32 parameters (sfg_mpnn_param_count()) and the 24 F32
 * normalisation values; then the 64-bit FNV-1a hash of every byte before it.
 *   params, norm   device F32 arrays (read by save, written by load)
 *   meta           host
 * Both synchronise.  sfg_mpnn_load checks the magic, the version, the shapes,
 * the length, the hash, the cheap-embedding ranges and that every value is
 * finite, and writes nothing to the outputs unless all hold.
 * Errors: SFG_EINVAL (unreadable or unwritable file, or a failed check; the
 * message says which), SFG_EHIP. */
sfg_status sfg_mpnn_save(const char *path, const float *params, const float *norm, const sfg_mpnn_meta *meta,
                         void *stream);
sfg_status sfg_mpnn_load(const char *path, float *params, float *norm, sfg_mpnn_meta *meta, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SFG_H_ */
