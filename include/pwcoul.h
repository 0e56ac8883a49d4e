/*
 * pwcoul.h -- C ABI of libpwcoul, the MI355X (gfx950) library for two-electron
 * Coulomb integrals over box planewaves reconstructed from O(N^{2/3})
 * per-direction tables.
 *
 * Method (Pederson, arxiv 1502.08043):
 *   basis       phi_n(r) = L^{-3/2} exp(2 pi i n.r / L), r in [0, L]^3, all
 *               n in Z^3 with |n|^2 <= n2max (Sec. II, the cutoff on |I|).
 *   integral    <ij|kl> = Int Int phi_i*(r) phi_j*(r') phi_k(r) phi_l(r')
 *               / |r - r'| d^3r d^3r'   (Eq. 2; free-space Coulomb between
 *               densities confined to the box; bra conjugated, i and k share r).
 *   quadrature  Laplace transform of the Coulomb kernel, split at alpha_c,
 *               t = alpha^{-1/2} on the tail, Gauss quadrature on both pieces
 *               (Eqs. 5-13), giving Q nodes (beta_q, W_q) with
 *               beta = 4 alpha / L^2 and
 *                 <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q
 *                           tau_q(m_x, m'_x) tau_q(m_y, m'_y) tau_q(m_z, m'_z)
 *               (Eq. 14), m = n_k - n_i, m' = n_l - n_j per direction.
 *   table       tau_q(m, m') = beta_q^{-1/2} Int_0^1 Int_0^1
 *               exp(-(xi - xi')^2 / beta_q) exp(2 pi i (m xi + m' xi')) dxi dxi'
 *               (Eq. 8 after the p integral, reduced coordinates), one real
 *               table of (4 nmax + 1)^2 entries per node serving all three
 *               directions of the cube (Sec. III: planewave products are
 *               planewaves, so only index differences matter); a rectangular
 *               box has one table per direction (pwc_table_create_box).
 *   energies    uniform electron gas, one spin channel (Sec. III):
 *               E_H =  1/2 sum_{i,j} f_i f_j <ij|ij>,
 *               E_x = -1/2 sum_{i,j} f_i f_j <ij|ji>  (i = j included).
 *
 * Conventions for every call:
 *   - Units are atomic units, L in bohr.  Results scale as 1/L.
 *   - Basis indices are 0-based in the canonical order: ascending
 *     (|n|^2, n_x, n_y, n_z), so a Fermi sphere |n|^2 <= r2 is an index prefix.
 *   - "d_" pointers are device (HBM) pointers on the current HIP device and
 *     stay owned by the caller; "h_" pointers are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked async only enqueue work on it.
 *   - No exception crosses the ABI.  Argument errors are returned at once and
 *     nothing is enqueued.  Errors found by kernels (an index out of range)
 *     set an error word in the table that pwc_sync() reports and clears; the
 *     affected outputs are NaN and the others are valid.
 *   - A table is immutable after creation and may be read from several
 *     streams at once; pwc_table_destroy() must not race with its use.
 */
#ifndef PWCOUL_H
#define PWCOUL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every entry point is exported; the library is built with hidden visibility. */
#if defined(__GNUC__)
#define PWC_API __attribute__((visibility("default")))
#else
#define PWC_API
#endif

typedef enum {
    PWC_OK = 0,
    PWC_ERR_ARG = 1,     /* invalid argument (null pointer, bad size, bad mesh) */
    PWC_ERR_RANGE = 2,   /* a basis index outside [0, N) was seen by a kernel */
    PWC_ERR_NOMEM = 3,   /* device or host allocation failed */
    PWC_ERR_DEVICE = 4,  /* HIP runtime error */
    PWC_ERR_BUSY = 5,    /* server: queue full or shutting down */
    PWC_ERR_STATE = 6,   /* server: unknown ticket, or object in the wrong state */
    PWC_ERR_IO = 7,      /* table file missing, unreadable, corrupt or inconsistent */
    PWC_ERR_LIMIT = 8    /* a size beyond a fixed limit of the call (pwc_reconstruct_noalloc) */
} pwc_status;

typedef enum {
    PWC_FP64 = 0,   /* FP64 tables, FP64 node products and accumulation */
    PWC_MIXED = 1,  /* FP32 hi/lo split tables; node products and sums in
                       float-float (error-free FP32 transformations), final
                       scaling and energy reductions in FP64 */
    PWC_FP32 = 2    /* one FP32 table (W^(1/3) tau rounded once: 4 bytes an
                       entry, half the bytes the node passes read); node
                       products and sums of four nodes in FP32, accumulated in
                       FP64.  Error at most about 4.2e-7 of the sum of the
                       node terms' magnitudes (seven FP32 roundings per term):
                       for work at six places.  Reconstruction of planewave
                       tables only (PWC_ERR_ARG elsewhere). */
} pwc_precision;

/*
 * How the pair sums of pwc_energies* evaluate <ij|ji>.  Both give the same sum
 * up to rounding.
 *   NODESUM: the Q-node sum of Eq. 14 for every pair, from the diagonal
 *            entries tau_q(m, -m) (the paper's O(M^2 Q) evaluation).
 *   KTABLE:  <ij|ji> depends only on |n_j - n_i| per direction (sorted,
 *            for a cube); the node sums K(a, b, c) = sum_q W_q D_q(a) D_q(b)
 *            D_q(c), a <= b <= c <= 4 nmax for a cube and every a, b, c for a
 *            box, are formed once at table creation and each pair reads one
 *            entry.  Available when the entries fit in LDS: C(4 nmax + 3, 3)
 *            for a cube (nmax <= 23), (4 nmax + 1)^3 for a box (nmax <= 6 ...
 *            13, i.e. n2max <= 195).
 *   AUTO:    KTABLE when available, else NODESUM.
 */
typedef enum {
    PWC_PAIR_AUTO = 0,
    PWC_PAIR_NODESUM = 1,
    PWC_PAIR_KTABLE = 2
} pwc_pair_algo;

typedef enum {
    PWC_MESH_GEOMETRIC = 0,      /* "Mesh 2" of Sec. III / Table I */
    PWC_MESH_TWO_INTERVAL = 1,   /* "Mesh 1" of Sec. III / Table I */
    PWC_MESH_GEOMETRIC_ROOT = 2  /* Mesh 2's pieces in sqrt(beta), tail exact for
                                    polynomials in t^2 (Sec. II after Eq. 14) */
} pwc_mesh_kind;

/*
 * Quadrature mesh on the Laplace variable (Eqs. 11-14, Sec. III).
 * Interval 1 is [0, beta_c] with beta_c = 4 alpha_c / L^2; the tail
 * [beta_c, inf) is integrated in t = beta^{-1/2} on (0, beta_c^{-1/2}] and
 * each tail node maps back to beta = 1/t^2 with weight 2 w / t^3.
 *   GEOMETRIC:    interval 1 is cut at beta_c * ratio^{-k}, k = n_sub-1 .. 1,
 *                 into n_sub pieces with q_sub Gauss-Legendre points each;
 *                 plus q_tail tail points.  Q = n_sub * q_sub + q_tail.
 *                 Table I's Mesh 2 is n_sub = 8, ratio = 5.
 *   TWO_INTERVAL: q_sub points on interval 1 and q_tail on the tail
 *                 (Table I's Mesh 1 has q_sub = q_tail = Q).
 *   GEOMETRIC_ROOT: the pieces of GEOMETRIC, each integrated by q_sub
 *                 Gauss-Legendre points in s = beta^{1/2} (node s^2, weight
 *                 2 s w; near beta = 0 the integrand is a series in
 *                 beta^{1/2}), and a tail rule in t exact for polynomials in
 *                 t^2 up to degree 4 q_tail - 2 (the positive half of the
 *                 2 q_tail-point Gauss-Legendre rule on [-t_c, t_c]; the
 *                 paper notes that a rule for polynomials in x^2 is twice as
 *                 efficient).  Q = n_sub * q_sub + q_tail.  On the
 *                 9171-planewave basis, n_sub = 4, ratio = 7, q_sub = 8,
 *                 q_tail = 4 (Q = 36) is within 1e-9 of the converged
 *                 integrals, where GEOMETRIC needs 88 to 112 nodes.
 * alpha_c <= 0 selects alpha_c = L^2 / 4, i.e. beta_c = 1 for every box: the
 * tables are then independent of L and <ij|kl>(L) = <ij|kl>(1) / L exactly.
 * This is the reading of the paper's "alpha_c = 1" that reproduces Table I.
 * alpha_c > 0 is taken literally (fixed alpha_c in bohr^2).
 */
typedef struct {
    int kind;        /* pwc_mesh_kind */
    int n_sub;       /* GEOMETRIC(_ROOT): number of pieces of interval 1, 1..32 */
    double ratio;    /* GEOMETRIC(_ROOT): ratio of successive piece edges, > 1 */
    int q_sub;       /* Gauss-Legendre points per piece of interval 1, 1..256 */
    int q_tail;      /* Gauss-Legendre points on the tail, 1..256 */
    double alpha_c;  /* split point (bohr^2); <= 0 selects beta_c = 1 */
} pwc_mesh;

/* Maximum sizes accepted by pwc_table_create. */
#define PWC_MAX_N2MAX 624    /* nmax <= 24, table dimension 4 nmax + 1 <= 97 */
#define PWC_MAX_NODES 512
/* ... and by pwc_table_create_gauss (n1^3 basis functions fit an int32). */
#define PWC_GAUSS_MAX_N1 1290
#define PWC_GAUSS_MAX_PAIRS 8192

typedef struct pwc_table pwc_table;
typedef struct pwc_server pwc_server;

/* Library version string (static storage). */
PWC_API const char *pwc_version(void);

/* Human-readable name of a status code (static storage, never NULL). */
PWC_API const char *pwc_status_str(pwc_status s);

/*
 * Default mesh for a node count: GEOMETRIC with n_sub = 8, ratio = 5,
 * q_tail = 8 and q_sub = (n_nodes - 8) / 8.  Requires n_nodes >= 16 and
 * n_nodes % 8 == 0, else PWC_ERR_ARG.  Writes *out (host).
 */
PWC_API pwc_status pwc_mesh_default(int n_nodes, pwc_mesh *out);

/* Number of nodes Q of a mesh; PWC_ERR_ARG if the mesh is invalid. */
PWC_API pwc_status pwc_mesh_count(const pwc_mesh *mesh, int *n_nodes);

/*
 * Host-only set-up, no device needed.  pwc_mesh_build writes the nodes
 * beta_q and weights W_q (q = 0..Q-1, FP64, Eqs. 11-13: Gauss-Legendre in
 * beta on interval 1, in t = beta^{-1/2} on the tail) that a table of box side
 * L (the reference length of a box) built with `mesh` uses; PWC_ERR_ARG for an
 * invalid mesh or L <= 0.  pwc_basis_enumerate writes *N and, unless h_n is
 * NULL, the canonical basis |n|^2 <= n2max ([N][3] int32, ascending
 * (|n|^2, n_x, n_y, n_z)); 1 <= n2max <= PWC_MAX_N2MAX.
 */
PWC_API pwc_status pwc_mesh_build(const pwc_mesh *mesh, double L, double *h_beta, double *h_W);
PWC_API pwc_status pwc_basis_enumerate(int n2max, int32_t *h_n, int64_t *N);

/*
 * Build the tables for a cube of side L > 0 (pwc_table_create_box for a
 * rectangular box) and the basis |n|^2 <= n2max
 * (1 <= n2max <= PWC_MAX_N2MAX) on the mesh `mesh` (NULL: the default mesh
 * for n_nodes).  If mesh is given, n_nodes must be 0 or equal its node count.
 * Basis, mesh and index maps are formed on the host in FP64; the 1-D
 * primitives and every table layout are computed by HIP kernels on `stream`
 * (FP64).  The call returns once that work is queued: every later call that
 * takes the table and a stream first makes that stream wait for the table's
 * construction, so the table may be used on any stream at once, with no
 * synchronization by the caller.  The handle owns all of its device memory
 * (see pwc_table_info) and must be released with pwc_table_destroy.  *out is
 * NULL on failure.
 */
PWC_API pwc_status pwc_table_create(double L, int n2max, int n_nodes, const pwc_mesh *mesh,
                            void *stream, pwc_table **out);

/*
 * A rectangular box with sides (Lx, Ly, Lz).  The derivation (Sec. II)
 * counts planewaves in a box among the separable bases but works the
 * formulas out for the cube only; writing 1/r as a Gaussian integral
 * (Eqs. 5-6), direction d factorises as in a cube of side L_d, so on the
 * reference mesh beta = 4 alpha / L0^2, L0 = (Lx Ly Lz)^(1/3), direction d
 * reads its own tables at the node beta_q / rho_d^2, rho_d = L_d / L0, and
 *   <ij|kl> = (1/(sqrt(pi) L0)) sum_q W_q tau^x_q tau^y_q tau^z_q.
 * alpha_c of a mesh refers to L0.  The basis is the same |n|^2 <= n2max set
 * of integer vectors.  Equal sides give exactly the table of
 * pwc_table_create.  The exchange kernel table of a box has (K+1)^3 entries
 * (no sorting across directions) and is kept when it fits on chip.  Errors
 * and ownership as pwc_table_create.
 */
PWC_API pwc_status pwc_table_create_box(double Lx, double Ly, double Lz, int n2max, int n_nodes,
                                        const pwc_mesh *mesh, void *stream, pwc_table **out);

/*
 * Tables for a separable basis of s-type Gaussians (Sec. II: products of
 * one-dimensional Gaussians are the other common separable basis; the paper
 * works the formulas out for planewaves only).  One-dimensional functions
 * f_u(x) = (2 a_u / pi)^{1/4} exp(-a_u (x - A_u)^2), u < n1, from h_exp
 * (a_u > 0, bohr^-2) and h_center (A_u, bohr), host arrays [n1]; the same set
 * along x, y and z, and every product is a basis function:
 * I = (l n1 + m) n1 + n is f_l(x) f_m(y) f_n(z), N = n1^3.
 * <ij|kl> = Int Int g_i(r) g_k(r) g_j(r') g_l(r') / |r - r'| (the functions
 * are real).  Writing 1/r = pi^{-1/2} Int s^{-1/2} exp(-s r^2) ds with
 * s = 1/(beta L^2), the factor of direction d is the closed form
 *   tau_q(x, y) = c_x c_y pi / sqrt(p_x p_y beta_q + (p_x + p_y)/L^2)
 *                 exp(-p_x p_y (P_x - P_y)^2 / (p_x p_y beta_q L^2 + p_x + p_y)),
 * for the one-dimensional pair products f_u f_v = c exp(-p (x - P)^2) of
 * (i, k) (x) and (j, l) (y), and <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q
 * tau_q tau_q tau_q (Eq. 14).  L is a reference length for the mesh
 * (beta = 4 alpha / L^2); about the extent of the centers serves well.  A
 * pair (u, v) is kept when exp(-(a_u a_v/(a_u + a_v))(A_u - A_v)^2) >= eps
 * (0 <= eps < 1): the band of eta N^{1/3} products of Sec. II; an integral
 * that needs a dropped pair is zero.  Tables: the full FP64 [Q][P1][P1]
 * (pwc_table_copy; P1 kept pairs) and the folded pairs of pairs with the
 * weights, FP64 and split FP32.  pwc_reconstruct (both precisions, any n,
 * async) and pwc_sync, pwc_table_copy, pwc_mesh_nodes, pwc_table_info
 * (N = n1^3) and pwc_table_destroy take such a table; the planewave calls
 * (energies, value table, layouts, files, basis vectors, no-allocation and
 * profiled reconstruction) return PWC_ERR_ARG.  PWC_ERR_ARG for invalid
 * inputs, PWC_ERR_RANGE if more than PWC_GAUSS_MAX_PAIRS pairs are kept.
 * pwc_gauss_info reports n1, the kept pairs and eps (PWC_ERR_ARG for a
 * planewave table).  Mesh, stream and ownership as pwc_table_create.
 */
PWC_API pwc_status pwc_table_create_gauss(const double *h_exp, const double *h_center, int n1,
                                          double L, double eps, int n_nodes, const pwc_mesh *mesh,
                                          void *stream, pwc_table **out);
PWC_API pwc_status pwc_gauss_info(const pwc_table *t, int *n1, int *n_pairs, double *eps);

/*
 * Free a table.  NULL is accepted.  The call does not wait for the device:
 * its device blocks (and its value table) go to a per-device cache of the
 * library together with events recorded after the last work each stream
 * queued on the table (every call that takes the table and a stream records
 * one), and a later table of the same device reuses a block only once all
 * of those events have completed (a block serves a table at most 1/8
 * smaller than itself); the cache keeps at most 4 GiB.  If the table was
 * used on more than 32 streams, or on a stream under graph capture, the
 * call waits for the device instead.  pwc_table_free_values waits for the
 * device before its block enters the cache.
 * pwc_release_cached_memory waits for the current device and returns the
 * cached blocks, the pinned upload buffers whose copies are done and the
 * value-table build's block lists (formed once per cutoff and shape); it must
 * not run while another thread calls into the library.
 */
PWC_API pwc_status pwc_table_destroy(pwc_table *t);
PWC_API pwc_status pwc_release_cached_memory(void);

/*
 * Sizes of a table: basis size N, nmax = floor(sqrt(n2max)), node count Q and
 * the device bytes it holds.  Any output pointer may be NULL.
 */
PWC_API pwc_status pwc_table_info(const pwc_table *t, int64_t *N, int *nmax, int *n_nodes,
                          size_t *device_bytes);

/*
 * Small quadruple lists skip the node passes: pwc_reconstruct evaluates a
 * list of n <= direct_max quadruples with four lanes per quadruple reading
 * the tables from global memory (Eq. 14 over all nodes in one launch);
 * longer lists run the node-pass kernels.  The two agree to rounding.  The
 * default is 524288 for a table whose node sums run fused (pwc_table_fused
 * for PWC_FP64; about where the two take equal time on MI355X) and 1048576,
 * the largest, for the others, whose separate node passes the direct kernel
 * outruns up to that size; 0 sends every list through the node passes.  n
 * must lie in [0, 1048576] (PWC_ERR_ARG otherwise).  Must not overlap a reconstruction that uses the
 * same table.
 */
PWC_API pwc_status pwc_table_set_direct_max(pwc_table *t, int64_t n);

/*
 * Reconstruction layout of a table for precision p (Eq. 14 evaluated in node
 * passes; each precision has its own default): lanes = G lanes of a
 * wavefront share one quadruple; words = W 16-byte words (two nodes, four
 * for PWC_FP32) per lane; nodes_per_pass = 2 G W (4 G W) nodes of every folded table entry
 * are held on chip per pass; passes = ceil(Q / (2 G W)); entry_bytes = size
 * of one decoded quadruple in the reconstruction's scratch stream (4 when the
 * table has at most 1024 folded entries per node, else 8).  Any output
 * pointer may be NULL.
 */
PWC_API pwc_status pwc_table_layout(const pwc_table *t, pwc_precision p, int *lanes, int *words,
                                    int *nodes_per_pass, int *passes, int *entry_bytes);

/*
 * *fused = 1 when a node-pass reconstruction of precision p on this table
 * runs fused: the one-lane layout (lanes 1, words 8) whose slab, basis and
 * fold map fit in one workgroup's LDS, every pass in one launch with the
 * partial sums in registers and no decoded stream (pwc_reconstruct and
 * pwc_reconstruct_noalloc; pwc_reconstruct_profile always runs the separate
 * launches, whose results agree to the rounding of the order of each
 * quadruple's node terms, bit for bit with one node range); else 0.
 */
PWC_API pwc_status pwc_table_fused(const pwc_table *t, pwc_precision p, int *fused);

/*
 * Force the reconstruction layout of every precision: (lanes, words) = (16, 1), (8, 2), (8, 1),
 * (4, 2), (2, 4), (1, 8) or (4, 1); (0, 0) restores the default choice.  A
 * PWC_FP32 pass covers 4 lanes x words nodes (four per 16-byte word), twice the
 * others; where that would run past the table's node padding (Q rounded up
 * to 32) PWC_FP32 keeps its default layout.  Results agree
 * between layouts to rounding; only speed differs.  PWC_ERR_ARG for other
 * pairs, PWC_ERR_RANGE if the per-pass slab of that layout does not fit on
 * chip (the layout is then unchanged).  Must not overlap a reconstruction
 * that uses the same table.
 */
PWC_API pwc_status pwc_table_set_layout(pwc_table *t, int lanes, int words);

/*
 * Value table.  <ij|kl> depends on a quadruple only through its three folded
 * table entries, one per direction (Sec. III: only index differences matter,
 * and tau_q(m, m') = tau_q(m', m) = tau_q(-m, -m')).  A cube's directions
 * share one table, so its distinct integrals are indexed by the sorted entry
 * triple: E (E + 1) (E + 2) / 6 values for E folded entries (E = 729 for
 * nmax = 13: 6.5e7 values, 0.52 GB); a box has E1^3.
 * pwc_table_build_values evaluates once by Eq. 14 over all nodes (FP64)
 * each of them that a quadruple of the basis can read (with m = n_k - n_i,
 * m' = n_l - n_j: |m|^2 + |m'|^2 <= 8 n2max, about half of them; the others
 * are left unwritten) into a device allocation of its own, asynchronously on
 * `stream`: work queued after it on that stream sees the values, work on
 * another stream must wait for it first (an event or a synchronize).  From
 * then on pwc_reconstruct with PWC_FP64 reads one value per
 * quadruple instead of summing nodes, for any n; PWC_MIXED keeps its node
 * sums.  The values agree with the node sums to rounding.  PWC_ERR_NOMEM if
 * the allocation fails (the table is then unchanged); a second call is a
 * no-op.  pwc_table_values_info sets *built (1 or 0) and *bytes, the size
 * the values take or would take (either pointer may be NULL);
 * pwc_table_free_values releases them (no-op if not built).  While built,
 * pwc_table_info's device_bytes includes them.  None of these calls may
 * overlap a reconstruction that uses the same table.
 */
PWC_API pwc_status pwc_table_build_values(pwc_table *t, void *stream);
PWC_API pwc_status pwc_table_values_info(const pwc_table *t, int *built, size_t *bytes);
PWC_API pwc_status pwc_table_free_values(pwc_table *t);

/*
 * Table persistence.  The 1-D tables of Eq. 8 depend only on the box, the
 * cutoff and the mesh, so a built table can be kept and reused.
 * pwc_table_save writes the mesh nodes and weights and the FP64 tables
 * tau_q(m, m') (the layout of pwc_table_copy) with the box sides,
 * cutoff and mesh fields and a checksum to `path` (synchronous; PWC_ERR_IO
 * if the file cannot be written).  pwc_table_load reads such a file and
 * creates the table from it without recomputing the 1-D integrals; the
 * folded, split-FP32, diagonal and kernel tables are derived on the device as
 * in pwc_table_create.  It returns PWC_ERR_IO for a missing, truncated,
 * corrupt (checksum) or inconsistent file, before any device work.  *out is
 * NULL on failure.
 */
PWC_API pwc_status pwc_table_save(const pwc_table *t, const char *path);
PWC_API pwc_status pwc_table_load(const char *path, void *stream, pwc_table **out);

/* Reference length (cube side, or (Lx Ly Lz)^(1/3) of a box), cutoff and
 * mesh of a table.  Any output pointer may be NULL. */
PWC_API pwc_status pwc_table_params(const pwc_table *t, double *L, int *n2max, pwc_mesh *mesh);

/* The three box sides of a table: sides[3] (host). */
PWC_API pwc_status pwc_table_box(const pwc_table *t, double *sides);

/* Canonical basis vectors: h_n[3 * i + d] = n_d of basis function i (host). */
PWC_API pwc_status pwc_basis(const pwc_table *t, int32_t *h_n);

/* Mesh nodes beta_q and weights W_q, q = 0..Q-1 (host, FP64). */
PWC_API pwc_status pwc_mesh_nodes(const pwc_table *t, double *h_beta, double *h_W);

/*
 * Copy the FP64 tables into the caller's device buffer, layout
 * d_dst[((d * Q + q) * nd + (m + 2 nmax)) * nd + (m' + 2 nmax)] = tau^d_q(m, m'),
 * nd = 4 nmax + 1, m, m' in [-2 nmax, 2 nmax], d < 1 for a cube (one table
 * serves every direction) and d < 3 for a box.  Async on `stream`.
 */
PWC_API pwc_status pwc_table_copy(const pwc_table *t, double *d_dst, void *stream);

/*
 * Reconstruct <ij|kl> (Eq. 14) for n quadruples.  d_quads is int32 [n][4]
 * holding (i, j, k, l) per row, 16-byte aligned; d_out is double [n], 8-byte
 * aligned.  Async on `stream`.  n = 0 is a no-op.  An index outside [0, N)
 * makes that output NaN and sets the table's error word (see pwc_sync).
 * p = PWC_FP64, PWC_MIXED or PWC_FP32.  An FP64 call on a table with its
 * value table built reads one value per quadruple; otherwise lists of at
 * most direct_max quadruples run the direct kernel and longer ones the node
 * passes (pwc_table_set_direct_max).  With the one-lane layout, when its
 * slab and the decode's basis and fold map fit in one workgroup's LDS
 * (pwc_table_fused), the passes run fused in one launch that keeps no
 * decoded stream; the results are those of the separate launches, bit for
 * bit.
 */
PWC_API pwc_status pwc_reconstruct(const pwc_table *t, const int32_t *d_quads, int64_t n,
                           double *d_out, pwc_precision p, void *stream);

/*
 * The node-pass reconstruction (whatever the direct-kernel size, and with or
 * without a value table; always as separate launches, never fused) that
 * also reports how long each of its launches took on `stream` (HIP events
 * between the launches), then waits for the stream.  h_ms[0] is the
 * standalone decode launch (near zero when the first pass decodes the
 * stream itself) and h_ms[1 .. P] are the P passes (first slab of at most
 * 2^27 quadruples).  *n_stages = 1 + P; PWC_ERR_ARG if max_stages < 1 + P.
 * Results are identical to pwc_reconstruct's with direct_max = 0.
 */
PWC_API pwc_status pwc_reconstruct_profile(const pwc_table *t, const int32_t *d_quads, int64_t n,
                                           double *d_out, pwc_precision p, void *stream,
                                           double *h_ms, int max_stages, int *n_stages);

/* Largest quadruple count of one pwc_reconstruct_noalloc call. */
#define PWC_NOALLOC_MAX_QUADS 8388608

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The node
 * passes of pwc_reconstruct (whatever the direct-kernel size, and with or
 * without a value table: the same kernels and results as pwc_reconstruct
 * with direct_max = 0) whose decoded-quadruple stream lives in a fixed
 * device array of the library (64 MiB per device, held until the process
 * ends) instead of a per-call allocation (a table whose passes run fused
 * keeps no such stream); no call allocates or frees device or host
 * memory.  Arguments, layouts, errors and ownership as
 * pwc_reconstruct; async on `stream`.  n > PWC_NOALLOC_MAX_QUADS returns
 * PWC_ERR_LIMIT with nothing enqueued (split longer lists into calls of at
 * most that many).  Every call on one device shares that device's array:
 * two calls whose work may overlap on the device (different streams with
 * no ordering between them, or several host threads) race and give wrong
 * results; calls on one stream, or ordered by events, are safe.  Nothing in
 * the array needs clearing between calls.
 */
PWC_API pwc_status pwc_reconstruct_noalloc(const pwc_table *t, const int32_t *d_quads, int64_t n,
                                           double *d_out, pwc_precision p, void *stream);

/*
 * Uniform-electron-gas energies of one spin channel (Sec. III) for the M
 * occupied orbitals d_occ (int32 basis indices [M]) with occupations d_f
 * (double [M], NULL = all ones):
 *   d_out[0] = E_H =  1/2 sum_{i,j} f_i f_j <ij|ij>
 *   d_out[1] = E_x = -1/2 sum_{i,j} f_i f_j <ij|ji>
 * Exchange integrals read only the diagonal entries tau_q(m, -m).  The pair
 * sum visits each unordered pair once (the summand is symmetric in i, j) and
 * reduces block partials in a fixed order, so results are bitwise
 * reproducible.  Async on `stream`; d_out is double [2] on the device.
 * M = 0 writes zeros.
 */
PWC_API pwc_status pwc_energies_async(const pwc_table *t, const int32_t *d_occ, const double *d_f,
                              int64_t M, pwc_precision p, double *d_out, void *stream);

/*
 * pwc_energies_async with an explicit pair-sum algorithm (PWC_ERR_ARG if
 * PWC_PAIR_KTABLE is asked for a table that does not keep the kernel table).
 * pwc_energies_async is this call with PWC_PAIR_AUTO.
 */
PWC_API pwc_status pwc_energies_ex(const pwc_table *t, const int32_t *d_occ, const double *d_f,
                                   int64_t M, pwc_precision p, pwc_pair_algo algo,
                                   double *d_out, void *stream);

/* Same as pwc_energies_async, then waits and writes h_out[2] = {E_H, E_x}. */
PWC_API pwc_status pwc_energies(const pwc_table *t, const int32_t *d_occ, const double *d_f,
                        int64_t M, pwc_precision p, double *h_out, void *stream);

/*
 * Wait for `stream`, then report and clear the table's kernel error word:
 * PWC_ERR_RANGE if any index seen since the last pwc_sync was out of range,
 * PWC_ERR_DEVICE on a runtime error, else PWC_OK.
 */
PWC_API pwc_status pwc_sync(const pwc_table *t, void *stream);

/* ------------------------------------------------------------------------
 * Serving: a persistent request loop with continuous batching.
 *
 * A scheduler thread owns `max_inflight` HIP streams ("slots") and a cache
 * of resident tables keyed by (Lx, Ly, Lz, n2max, mesh).  Submitted requests
 * wait in a FIFO; whenever a slot is free and the request's table plus
 * scratch fit in the HBM budget, the request is admitted: its table is
 * reused or built (least-recently-used tables that no queued or running
 * request holds are evicted to make room) and its kernels are launched on
 * the slot's stream, so work of different requests and tables overlaps on
 * the device.  A small reconstruction (at most the table's direct-kernel
 * size, pwc_table_set_direct_max: the default of each table the server
 * builds) admitted from the head of the queue takes along up to 23
 * later queued small reconstructions whose tables are resident, and one
 * launch of the direct kernel serves them all, each with its own table,
 * precision, buffers and error word.  A request whose table alone exceeds the budget fails with
 * PWC_ERR_NOMEM; otherwise requests wait for memory rather than fail.  Each
 * request computes every output with exactly the arithmetic of
 * pwc_reconstruct / pwc_energies_ex on the same table, so its result does
 * not depend on what else is in flight.
 *
 * Buffers named in a request (d_idx, d_f, d_out) are owned by the caller and
 * must stay valid and unmodified until pwc_server_wait (or a successful
 * pwc_server_poll) returns for its ticket.  If a kernel sees an index out of
 * range, the request reports PWC_ERR_RANGE.  Every request has an error word
 * of its own (the table's word, which pwc_sync reads, is not touched), so
 * the report reaches only the request that held the bad index, whatever
 * else ran at the same time on that table.
 * ------------------------------------------------------------------------ */
typedef enum { PWC_REQ_RECONSTRUCT = 0, PWC_REQ_ENERGIES = 1 } pwc_request_kind;

typedef struct {
    int kind;             /* pwc_request_kind */
    double L;             /* box side (along x for a rectangular box) */
    int n2max;            /* basis cutoff */
    int n_nodes;          /* default mesh for this node count, used if !has_mesh */
    int has_mesh;
    pwc_mesh mesh;
    int prec;             /* pwc_precision */
    int algo;             /* energies: pwc_pair_algo */
    const int32_t *d_idx; /* reconstruct: quadruples [n][4]; energies: occupied [n] */
    int64_t n;
    const double *d_f;    /* energies: occupations [n] or NULL */
    double *d_out;        /* reconstruct: [n]; energies: [2] = {E_H, E_x} */
    void *ready_event;    /* hipEvent_t or NULL: recorded by the caller after the
                             last work that writes d_idx / d_f or touches d_out;
                             the server's kernels for this request wait for it on
                             the device.  It must stay valid until the result is
                             collected.  With NULL the buffers must already be
                             idle when the request is submitted. */
    double Ly, Lz;        /* box sides along y and z for a rectangular box
                             (pwc_table_create_box, with L along x); 0 and 0
                             for a cube of side L */
} pwc_request;

typedef struct {
    pwc_status status;
    double e_h, e_x;      /* energies requests (also left in d_out) */
    double queue_ms;      /* submit -> launch */
    double latency_ms;    /* submit -> completion seen by the scheduler */
    int table_built;      /* 1 if this request had to build its table */
} pwc_result;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t table_builds, evictions;
    int resident_tables;
    size_t resident_bytes;
    double p50_ms, p99_ms, max_ms;    /* latency over completed requests */
    double wall_s;                    /* first submit -> last completion */
    double integrals_per_s, pairs_per_s;
    uint64_t launches;                /* kernel groups enqueued (one per slot use) */
    uint64_t batched;                 /* requests that rode in another's direct launch */
} pwc_server_stats;

/* Create a server for the current device.  hbm_budget_bytes > 0 bounds the
 * bytes of resident tables plus per-request scratch; 1 <= max_inflight <= 64. */
PWC_API pwc_status pwc_server_create(size_t hbm_budget_bytes, int max_inflight,
                                     pwc_server **out);

/* Queue a request (non-blocking).  Argument errors return at once. */
PWC_API pwc_status pwc_server_submit(pwc_server *s, const pwc_request *r, uint64_t *ticket);

/* PWC_OK and *res if the request has finished (its entry is then released),
 * PWC_ERR_BUSY if not yet, PWC_ERR_STATE for an unknown ticket. */
PWC_API pwc_status pwc_server_poll(pwc_server *s, uint64_t ticket, pwc_result *res);

/* Block until the request has finished; then as pwc_server_poll.  Each
 * ticket is collected once: a second thread waiting on the same ticket gets
 * PWC_ERR_STATE when the first collects it. */
PWC_API pwc_status pwc_server_wait(pwc_server *s, uint64_t ticket, pwc_result *res);

/* Counters and latency percentiles since creation (or the last reset). */
PWC_API pwc_status pwc_server_get_stats(pwc_server *s, pwc_server_stats *st);
PWC_API pwc_status pwc_server_reset_stats(pwc_server *s);

/* Drain every queued request, stop the scheduler, free every table. */
PWC_API pwc_status pwc_server_destroy(pwc_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PWCOUL_H */
