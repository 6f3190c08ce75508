/*
 * spde.h -- C interface of the MI355X (gfx950) SPDE field sampler.
 *
 * The library draws Gaussian random fields with exponential (Matern nu = 1/2)
 * covariance by the method of Osborn et al., "Scalable hierarchical PDE
 * sampler for generating spatially correlated random fields using
 * non-matching meshes" (arXiv:1712.06758):
 *
 *   1. the reaction-diffusion SPDE (kappa^2 - Laplacian) u = g W is discretised
 *      with lowest-order Raviart-Thomas fluxes and piecewise-constant cells on
 *      a structured box with sigma.n = 0 on the boundary (Sec. "Mixed finite
 *      element discretization", eq. reac_diff_weak), giving the saddle-point
 *      system eq. linsys / linsys_blocks
 *         [M  B^T       ] [sigma]   [ 0                 ]
 *         [B  -kappa^2 W] [u    ] = [ -g W^{1/2} xi     ],  xi ~ N(0, I);
 *   2. that system is solved with block-preconditioned MINRES whose
 *      preconditioner is blkdiag(diag(M), V), V one geometric-multigrid V-cycle
 *      on the approximate Schur complement kappa^2 W + B diag(M)^-1 B^T
 *      (the approximate Schur complement of eq. ldu with the kappa^2 W term);
 *   3. the cell field is projected onto a non-matching tetrahedral mesh,
 *      u_tet = Pi u, Pi = W_h^-1 G (Sec. "L2-Projection", eq. proj_op);
 *   4. coarse samples of the same event use the restricted noise of
 *      eq. ml-linsys (F_{l+1} = P^T F_l).
 *
 * Geometry and ordering
 *   The box is the unit cube [0,1]^3 with n^3 cubic cells, h = 1/n.
 *   Cells:  c = i + n*(j + n*k)                       (x fastest)
 *   Faces (external arrays, 3 n^2 (n+1) entries per sample):
 *           x-faces  i + (n+1)*(j + n*k),              i in 0..n
 *           y-faces  n^2(n+1) + i + n*(j + (n+1)*k),   j in 0..n
 *           z-faces  2 n^2(n+1) + i + n*(j + n*k),     k in 0..n
 *   A face value is the normal flux component along +x, +y or +z.
 *   Boundary faces carry sigma.n = 0 and are written as 0.
 *
 * Memory
 *   Pointers named *_dev are device pointers, *_host host pointers.  All
 *   device memory is owned by the caller; the library never allocates device
 *   memory.  It allocates a small pinned host buffer per context for the
 *   convergence poll.
 *
 * Errors
 *   Every entry point returns spde_status.  No exception crosses the
 *   interface.  spde_last_error() gives a thread-local description of the
 *   last non-OK status.  Handles are not thread-safe: use one handle per host
 *   thread at a time.
 */
#ifndef SPDE_H
#define SPDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spde_ctx* spde_handle;

typedef enum {
    SPDE_OK       = 0,   /* success                                                   */
    SPDE_ENOTCONV = 1,   /* max_iter reached for some sample; all outputs are written */
    SPDE_EINVAL   = -1,  /* invalid argument (size, range, null pointer, order)       */
    SPDE_ENOMEM   = -2,  /* bound workspace too small for the request                 */
    SPDE_EHIP     = -3,  /* a HIP runtime call failed                                 */
    SPDE_EFAILED  = -4   /* breakdown or non-finite value in some sample: that
                            sample's outputs are NaN, the others are valid           */
} spde_status;

typedef enum {
    SPDE_FP64  = 0,      /* everything in float64                                     */
    SPDE_MIXED = 1       /* float32 multigrid preconditioner inside float64 MINRES;
                            residuals, inner products, recurrences, transfer in f64  */
} spde_precision;

/* ---- set-up ------------------------------------------------------------ */

/* Create a sampler for the unit box with n^3 cells and SPDE coefficients
 * kappa, g (Sec. "Mixed finite element discretization"; for unit marginal
 * variance with nu = 1/2 in 3-D, g^2 = 8 pi kappa).
 * n must be a power of two with 4 <= n <= 1024; kappa > 0; g > 0.
 * Host-only: touches no GPU.  *out receives the handle (NULL on error). */
spde_status spde_setup_box(int n, double kappa, double g, spde_handle* out);

/* Choose precision, MINRES relative tolerance (on the preconditioned residual
 * norm, from a zero initial guess), iteration cap and the largest batch.
 * rtol in (0, 1); 1 <= max_iter <= 100000; 1 <= max_batch <= 4096.
 * Invalidates any bound workspace.  Host-only. */
spde_status spde_configure(spde_handle h, spde_precision prec, double rtol,
                           int max_iter, int max_batch);

/* Device workspace size in bytes needed by the current configuration.  On a
 * handle with a bound workspace the query leaves that binding in use. */
size_t spde_workspace_bytes(spde_handle h);

/* Bind a caller-owned device buffer of at least spde_workspace_bytes() bytes,
 * 256-byte aligned.  The buffer must outlive every call that uses the handle.
 * Selects the current HIP device as the handle's device. */
spde_status spde_bind_workspace(spde_handle h, void* dev_ptr, size_t bytes);

/* ---- L2 projection onto a tetrahedral mesh (Sec. "L2-Projection") ------- */

/* Build Pi = W_h^-1 G on the host for a tet mesh lying inside [0,1]^3:
 * Pi[t, c] = vol(tet t intersect cell c) / vol(tet t), exact overlap volumes
 * by convex clipping (eq. proj_op with P0 spaces on both meshes).
 *   xyz_host  [n_vert][3] float64 vertex coordinates
 *   tet_host  [n_tet][4]  int32 vertex indices
 * Outputs a CSR matrix in host memory allocated by the library:
 *   *row_ptr_host [n_tet+1] int64, *col_host [nnz] int32 (ascending per row),
 *   *val_host [nnz] float64; release each with spde_free_host().
 * Returns SPDE_EINVAL for a vertex outside [0,1]^3, a degenerate tet or an
 * index out of range.  Host-only; runs on all hardware threads. */
spde_status spde_build_transfer(spde_handle h, int64_t n_vert, const double* xyz_host,
                                int64_t n_tet, const int32_t* tet_host,
                                int64_t** row_ptr_host, int32_t** col_host,
                                double** val_host, int64_t* nnz);

/* Pi of the coupled coarse box ((n_fine/2)^3) onto the same tet mesh, from Pi
 * of the n_fine^3 box (eq. recursive_l2_projection, G_{l+1} = G_l P with the
 * box hierarchy's P0 injection P; the tet mesh is not coarsened):
 * Pi_c[t, I] = sum over the 8 children c of coarse cell I of Pi_f[t, c],
 * exact since a tet's overlap with I is the sum of its overlaps with the
 * children.  Input CSR in host memory (columns in [0, n_fine^3)); outputs as
 * spde_build_transfer (ascending columns, release with spde_free_host).
 * n_fine even in [2, 1024].  SPDE_EINVAL on a malformed matrix.  Host-only. */
spde_status spde_transfer_coarsen(int n_fine, int64_t n_rows, const int64_t* row_ptr_host,
                                  const int32_t* col_host, const double* val_host,
                                  int64_t** row_ptr_c, int32_t** col_c, double** val_c,
                                  int64_t* nnz_c);

/* Build the same Pi on the device, bit for bit equal to spde_build_transfer
 * (the same clipping arithmetic, no fused multiply-adds, the same order of
 * the pieces).  Two calls, so that the caller allocates every buffer:
 *   1. spde_build_transfer_device_rows writes the row pointers
 *      row_ptr_dev [n_tet+1] int64 and returns the entry count in *nnz (host);
 *      it synchronises `stream`.
 *   2. The caller allocates col_dev [nnz] int32 and val_dev [nnz] float64;
 *      spde_build_transfer_device_fill writes them (asynchronous on `stream`),
 *      given the row_ptr_dev of call 1 and the same mesh.
 *   n         cells per box edge, in [2, 1024]
 *   xyz_dev   [n_vert][3] float64 vertex coordinates (device)
 *   tet_dev   [n_tet][4]  int32 vertex indices (device)
 * n_vert in [4, 2^31), n_tet in [1, 2^31).  Returns SPDE_EINVAL, naming the
 * first offending tet, for a vertex index out of range, a vertex outside
 * [0,1]^3 or a degenerate tet (only vertices that some tet references are
 * checked); row_ptr_dev is then undefined.  No device memory is allocated. */
spde_status spde_build_transfer_device_rows(int n, int64_t n_vert, const double* xyz_dev, int64_t n_tet,
                                            const int32_t* tet_dev, int64_t* row_ptr_dev, int64_t* nnz,
                                            void* stream);
spde_status spde_build_transfer_device_fill(int n, int64_t n_vert, const double* xyz_dev, int64_t n_tet,
                                            const int32_t* tet_dev, const int64_t* row_ptr_dev,
                                            int32_t* col_dev, double* val_dev, void* stream);

/* Register a device copy of Pi (CSR as produced above).  The arrays are
 * borrowed, not copied: they must stay valid while the handle samples. */
spde_status spde_set_transfer(spde_handle h, int64_t n_tet, int64_t nnz,
                              const int64_t* row_ptr_dev, const int32_t* col_dev,
                              const double* val_dev);

/* Visiting order of the transfer SpMM.  The product takes the rows in chunks
 * of spde_transfer_chunk_rows() consecutive rows (so that each sample's
 * values are stored contiguously) and visits the chunks in an order that
 * keeps neighbouring chunks together in time, so that the box cells they
 * share are still cached: order_host [ceil(n_rows / chunk)] receives the
 * chunk indices sorted by the cell of each chunk's first entry (16 x 16-cell
 * tiles of the (x, y) plane, then z, then y, then x).  n in [1, 1024] is the
 * box edge of the matrix's columns; row_ptr/col as built above (host).
 * Host-only. */
int spde_transfer_chunk_rows(void);
spde_status spde_transfer_chunk_order(int n, int64_t n_rows, const int64_t* row_ptr_host,
                                      const int32_t* col_host, int32_t* order_host);

/* Register a device copy of such a chunk order for the handle's transfer
 * (borrowed; NULL: the chunks in index order).  Must follow spde_set_transfer.
 * Results do not depend on the order: each row's sum is formed the same way
 * wherever it runs. */
spde_status spde_set_transfer_chunk_order(spde_handle h, const int32_t* order_dev);

/* Row units of the LDS-staged transfer product (eq. proj_op, u_tet = Pi u).
 * The rows are grouped in units of spde_transfer_unit_rows() consecutive rows
 * (a chunk holds a whole number of units).  For each unit: the distinct box
 * cells its entries reference, ascending, and for each entry the index of its
 * column in that list.  The product then loads each unit's cells once into
 * LDS and forms all of the unit's rows from there.
 *   row_ptr_host  [n_rows + 1] int64, col_host [nnz] int32: Pi as built above
 *   unit_ptr_host [n_units + 1] int64 out, n_units = ceil(n_rows / unit rows):
 *                 offsets of each unit's list in unit_cells_host
 *   unit_cells_host [unit_ptr_host[n_units]] int32 out (NULL: first call)
 *   local_col_host  [nnz] uint16 out (NULL: first call); 65535 for a column
 *                 outside [0, n_cols) (the product skips it, as spde_csr_apply)
 *   max_cells, max_entries out: the largest count of cells / entries of a unit
 * Two calls: the first (both list pointers NULL) writes unit_ptr_host and the
 * maxima, the second fills the lists.  Host arrays, caller-owned; no device
 * call.  SPDE_EINVAL for null pointers, n_rows < 1, n_cols < 1 or row pointers
 * that decrease or leave [0, nnz]; SPDE_ENOMEM if host memory runs out. */
int spde_transfer_unit_rows(void);
spde_status spde_transfer_units(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr_host,
                                const int32_t* col_host, int64_t* unit_ptr_host, int32_t* unit_cells_host,
                                uint16_t* local_col_host, int32_t* max_cells, int32_t* max_entries);

/* Register device copies of spde_transfer_units' lists for the handle's
 * transfer (borrowed: they must stay valid while the handle samples; they must
 * come from the registered matrix).  The transfer product of the sampling
 * calls then uses the LDS-staged kernel for sample blocks of 32 or 64 samples
 * whose largest unit fits its LDS budget (60 KiB per block), and the chunked
 * gather otherwise.  Results are bitwise those of the gather: each row's sum
 * runs over its entries in the same order.  spde_set_transfer clears the
 * registration; NULL pointers clear it too. */
spde_status spde_set_transfer_units(spde_handle h, const int64_t* unit_ptr_dev, const int32_t* unit_cells_dev,
                                    const uint16_t* local_col_dev, int32_t max_cells, int32_t max_entries);

/* ---- the sampler --------------------------------------------------------- */

/* Draw `batch` field samples from the noise vectors xi_dev [batch][n^3]:
 * solve eq. linsys for each right-hand side, then project.
 *   u_tet_dev  [batch][n_tet]      Pi u            (nullable if no transfer set)
 *   u_box_dev  [batch][n^3]        box cell field  (nullable)
 *   sigma_dev  [batch][3n^2(n+1)]  flux sigma = -M^-1 B^T u (nullable)
 *   stream     hipStream_t to run on (NULL = default stream)
 *   iters_host [batch] MINRES iterations per sample, refinement passes
 *              included (nullable)
 *   relres_host[batch] true relative residual ||F - A U|| / ||F|| with the
 *              flux recovered from u (nullable; computing it costs one extra
 *              pass, so NULL skips it unless sigma_dev is requested)
 * Blocks the host until the solve has converged (it polls per-sample
 * convergence flags every few iterations); the projection and the optional
 * outputs are enqueued on `stream` before returning.  Samples are
 * independent: each result is bitwise the same alone or in any batch.
 * Returns SPDE_ENOTCONV if some sample hit max_iter (outputs written),
 * SPDE_EFAILED on breakdown, SPDE_ENOMEM if batch > max_batch. */
spde_status spde_sample(spde_handle h, int batch, const double* xi_dev,
                        double* u_tet_dev, double* u_box_dev, double* sigma_dev,
                        void* stream, int* iters_host, double* relres_host);

/* Warm-started coupled fine solve (the MLMC coupling of levels l and l+1):
 * as spde_sample, but MINRES starts from U0 = P u_c, the coarse solution
 * u_coarse_dev [batch][(n/2)^3] (float64, cell order of the (n/2)^3 box)
 * injected into its 8 children.  The true residual r0 = F - A U0 (flux
 * recovered from U0) is solved for by one correction solve that adds to U0,
 * stopped at the relative tolerance rtol ||F|| / max ||r0|| (within
 * [rtol, 0.5]), so the result has the accuracy of a cold solve.  iters_host
 * counts the correction solve's iterations.  White noise puts most of the load
 * at the grid scale, which the coarse field cannot represent, so the start
 * saves few iterations (measured: under one at these sizes).  u_coarse_dev is
 * read only; u_coarse_count is the number of float64 values the caller passes
 * there and must equal batch (n/2)^3.  Errors as spde_sample, and SPDE_EINVAL
 * if xi_dev or u_coarse_dev is NULL or u_coarse_count is not batch (n/2)^3.
 * Iterative refinement (spde_set_refinement) follows the correction solve as
 * in spde_sample. */
spde_status spde_sample_warm(spde_handle h, int batch, const double* xi_dev, const double* u_coarse_dev,
                             int64_t u_coarse_count, double* u_tet_dev, double* u_box_dev,
                             double* sigma_dev, void* stream, int* iters_host, double* relres_host);

/* Noise of the coupled coarse sample (eq. ml-linsys, F_{l+1} = P^T F_l):
 * xi_c[I] = 8^{-1/2} * sum of xi_f over the 8 children of coarse cell I.
 *   xi_f_dev [batch][n_fine^3] -> xi_c_dev [batch][(n_fine/2)^3]
 * n_fine even and >= 2.  Asynchronous on `stream`. */
spde_status spde_restrict_noise(int n_fine, int batch, const double* xi_f_dev,
                                double* xi_c_dev, void* stream);

/* ---- spatially varying coefficients -----------------------------------------
 * The SPDE (kappa(x)^2 - Laplacian) u = g(x) W with cell-wise kappa and g: the
 * method's space-dependent correlation length and marginal variance (the
 * advantage over circulant embedding named in Sec. "Introduction").  The
 * (2,2) block of eq. linsys_blocks becomes -diag(kappa_c^2) W and the load
 * -diag(g_c) W^{1/2} xi; every sample of the handle uses the same fields.
 *   kappa_dev [n^3], g_dev [n^3]: caller-owned device arrays in cell order,
 *     read by every later sampling call (keep them alive and unchanged while
 *     the handle samples); NULL = the constant of spde_setup_box.  Values must
 *     be finite, kappa > 0 and g >= 0 (not checked: a non-finite value makes
 *     the samples fail with SPDE_EFAILED).
 *   kappa_ref: the reaction coefficient of the multigrid preconditioner S~
 *     (the operator always uses the cell values).
 *     0 with a kappa field (the recommended form): the multigrid takes the
 *       cell-wise kappa.  The finest level's reaction diagonal is
 *       kappa_c^2 h^3; each coarser level's is the Galerkin one, the sum of the
 *       8 children's (the coarse kappa^2 is the children's mean, eq.
 *       ml-linsys).  The smoother's diagonal is the cell's, and its Chebyshev
 *       interval comes from kappa_min.  The level diagonals are built, once, by
 *       the next sampling, V-cycle or slot-reset call.  That call synchronises
 *       its stream and returns SPDE_EINVAL if some kappa_c is not positive and
 *       finite.
 *     > 0: one constant kappa_ref in the whole hierarchy, e.g.
 *       sqrt(kappa_min kappa_max).  This takes more iterations as the contrast
 *       grows.
 *     0 without a kappa field keeps the setup kappa.
 * The preconditioner stays symmetric positive definite in both forms, so the
 * solution does not depend on the choice; only the iteration count does.
 * Coupled coarse samples (eq. ml-linsys): the Galerkin coarse reaction block
 * has kappa_c^2 = mean of the 8 children's kappa^2; the coarse load equals the
 * restricted one when g is constant on each coarse cell.
 * Call between sampling calls (not while slots iterate).  Host-only: returns
 * SPDE_EINVAL for a negative or non-finite kappa_ref. */
spde_status spde_set_coefficients(spde_handle h, const double* kappa_dev, const double* g_dev,
                                  double kappa_ref);

/* ---- counter-based noise --------------------------------------------------
 * The noise xi of eq. linsys can be drawn on the device instead of being read
 * from memory (the paper draws it on the host with a parallel pseudo-random
 * library, Sec. "Implementation details").  Every value is a pure function of
 * (seed, event, grid, cell), so a field is reproducible from its key alone.
 *   Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
 *   Field of event e on the n^3 box: key (seed, e), counter (c >> 2, n, 0, 0)
 *     for cell c; the call's four 64-bit words x0..x3 give, by Box-Muller,
 *     xi[4b + 0, 1] from (x0, x1) and xi[4b + 2, 3] from (x2, x3), with
 *     u = ((x_a >> 11) + 1) 2^-53, t = (x_b >> 11) 2^-53,
 *     (xi_a, xi_b) = sqrt(-2 ln u) (cos 2 pi t, sin 2 pi t).
 *   Coupled field (coupled = 1): the noise of the coarse sample of event e
 *     (eq. ml-linsys), i.e. spde_restrict_noise applied to the event's
 *     (2n)^3 field; drawing it directly gives bitwise the same values.
 * Raw words are integers (bitwise reproducible); normals use the device's
 * float64 log, sqrt and sincos (a few ulp from any other libm). */

/* Like spde_sample, with the noise of events event0 .. event0 + batch - 1
 * drawn inside the initialisation kernel (nothing is read for xi).
 * n must be divisible by 4 (coupled = 0) or even (coupled = 1); relres_host
 * draws the noise again into workspace.  Errors as spde_sample. */
spde_status spde_sample_seeded(spde_handle h, int batch, uint64_t seed, uint64_t event0,
                               int coupled, double* u_tet_dev, double* u_box_dev,
                               double* sigma_dev, void* stream, int* iters_host,
                               double* relres_host);

/* Write the noise of events event0 .. event0 + batch - 1 on the n^3 box:
 * xi_dev [batch][n^3].  n in [2, 1024], divisible by 4 (coupled = 0) or even
 * (coupled = 1); batch in [1, 65535].  Asynchronous on `stream`. */
spde_status spde_noise(int n, int coupled, uint64_t seed, uint64_t event0, int batch,
                       double* xi_dev, void* stream);

/* Raw generator output for the counters (ctr0 + b, ctr1, 0, 0) under the key
 * (seed, event): out_dev [nblocks][4] uint64, b < nblocks (1 <= nblocks <= 2^36).
 * For checking the generator against its definition.  Asynchronous. */
spde_status spde_philox4x64(uint64_t seed, uint64_t event, uint64_t ctr0, uint64_t ctr1,
                            int64_t nblocks, uint64_t* out_dev, void* stream);

/* ---- continuous batching (serving) ---------------------------------------
 * The slots [0, max_batch) of a handle are independent MINRES instances on the
 * same box.  A caller may start a new sample in an idle slot at any time while
 * other slots iterate; every slot's arithmetic is independent of the others,
 * so a sample's result is bitwise the same whichever slots share its launches.
 * Slot states returned by spde_slots_poll:
 *   0 iterating, 1 converged, 2 stopped at max_iter, 3 failed, 4 idle. */

/* Mark slots [0, nslots) idle.  Call once before using the slot interface. */
spde_status spde_slots_reset(spde_handle h, int nslots, void* stream);

/* Start a sample in `slot` from the noise xi_dev [n^3] (the slot must be idle
 * or finished).  Asynchronous on `stream`. */
spde_status spde_slot_start(spde_handle h, int slot, const double* xi_dev, void* stream);

/* Like spde_slot_start, with the noise of `event` (coupled: the coarse noise
 * of the event) drawn inside the initialisation kernel; see spde_noise. */
spde_status spde_slot_start_seeded(spde_handle h, int slot, uint64_t seed, uint64_t event,
                                   int coupled, void* stream);

/* Enqueue `iters` MINRES iterations over slots [0, nslots); idle and finished
 * slots are skipped on the device.  Asynchronous on `stream`. */
spde_status spde_slots_step(spde_handle h, int nslots, int iters, void* stream);

/* Blocking: copy the states and iteration counts of slots [0, nslots) to the
 * host arrays (nullable). */
spde_status spde_slots_poll(spde_handle h, int nslots, int* state_host, int* iters_host,
                            void* stream);

/* Write the field of a converged slot to u_box_dev [n^3] (nullable: discard)
 * and mark the slot idle.  Asynchronous on `stream`. */
spde_status spde_slot_finish(spde_handle h, int slot, double* u_box_dev, void* stream);

/* Stateless CSR SpMM y[b] = A x[b] for b < batch (the transfer apply with an
 * explicit matrix, Sec. "L2-Projection", eq. proj_op).  x [batch][n_cols],
 * y [batch][n_rows]; column indices outside [0, n_cols) are skipped; the
 * row chunks are visited in chunk_order_dev (see spde_transfer_chunk_order)
 * when it is not NULL, else in index order.  Each row sums its entries in
 * their stored order, the same for every batch.
 * The samples are processed in blocks of up to 64, each block first staged
 * sample-minor (x_t[col][s]) so that one gather of a column brings the whole
 * block: work_dev (256-byte aligned, caller-owned, at least
 * spde_csr_apply_work_bytes(n_cols, batch) bytes) holds the staged block; it
 * may be NULL for batch 1, which needs none.  SPDE_EINVAL for bad sizes, a null
 * array or a work buffer that is too small.  Asynchronous on `stream`; the
 * work buffer is in use until the call's work on the stream has finished. */
size_t spde_csr_apply_work_bytes(int64_t n_cols, int batch);
spde_status spde_csr_apply(int64_t n_rows, int64_t nnz, const int64_t* row_ptr_dev,
                           const int32_t* col_dev, const double* val_dev, int64_t n_cols,
                           int batch, const double* x_dev, double* y_dev,
                           const int32_t* chunk_order_dev /* nullable */, void* work_dev,
                           size_t work_bytes, void* stream);

/* The same product without a work buffer, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the staged sample block lives in a device array
 * of the library, spde_csr_apply_noalloc_max_bytes() = 64 MiB, that each GPU
 * holds from the call's first use on it until the process ends.  The call
 * allocates nothing; it accepts the sizes whose staged block fits that array
 * (spde_csr_apply_work_bytes(n_cols, batch) <= 64 MiB, e.g. 64 samples of a
 * 32^3 box or 32 of a 64^3 box; batch 1 always) and returns SPDE_EINVAL with
 * the sizes for larger ones.  Arguments, results (bitwise those of
 * spde_csr_apply) and other errors as spde_csr_apply.  All calls on one GPU
 * share the array: calls that overlap on that GPU (other streams or host
 * threads) race and must be serialised by the caller.  Asynchronous on
 * `stream`. */
size_t spde_csr_apply_noalloc_max_bytes(void);
spde_status spde_csr_apply_noalloc(int64_t n_rows, int64_t nnz, const int64_t* row_ptr_dev,
                                   const int32_t* col_dev, const double* val_dev, int64_t n_cols,
                                   int batch, const double* x_dev, double* y_dev,
                                   const int32_t* chunk_order_dev /* nullable */, void* stream);

/* ---- operators exposed for verification -------------------------------- */

/* y = A x with A the saddle-point matrix of eq. linsys_blocks on the full
 * external face/cell layout (boundary face entries of x are ignored, of y
 * written as 0).  x_sigma/y_sigma [batch][3n^2(n+1)], x_u/y_u [batch][n^3].
 * Needs a bound workspace; batch <= max_batch.  Asynchronous on `stream`. */
spde_status spde_apply_operator(spde_handle h, int batch, const double* x_sigma_dev,
                                const double* x_u_dev, double* y_sigma_dev,
                                double* y_u_dev, void* stream);

/* The production operator pass on a given direction:
 *   y = A blkdiag(P_f diag(M), I) x,
 * i.e. A applied to z = (P_f diag(M) x_sigma, x_u), where P_f is the handle's
 * face block of the MINRES preconditioner (spde_set_face_preconditioner:
 * diag(M)^-1, or the truncated Neumann series of M^-1 about its diagonal) and
 * x_u enters in the multigrid precision (rounded to float32 in mixed
 * precision), exactly as the solver's fused Lanczos pass forms A z.  Layouts
 * and conditions as spde_apply_operator.  For checking the solver's own
 * kernel instances against an explicit matrix. */
spde_status spde_apply_operator_precond(spde_handle h, int batch, const double* x_sigma_dev,
                                        const double* x_u_dev, double* y_sigma_dev, double* y_u_dev,
                                        void* stream);

/* z = V r: one V-cycle of the configured precision on the approximate Schur
 * complement (the u-block of the preconditioner).  r, z [batch][n^3].
 * Asynchronous on `stream`. */
spde_status spde_apply_vcycle(spde_handle h, int batch, const double* r_dev,
                              double* z_dev, void* stream);

/* u_tet = Pi u_box with the registered transfer.  [batch][n^3] -> [batch][n_tet],
 * batch <= max_batch.  Stages the samples in the bound workspace (as
 * spde_csr_apply does in its work buffer), so it must not overlap a running
 * solve or iterating slots of the same handle.  Asynchronous on `stream`. */
spde_status spde_apply_transfer(spde_handle h, int batch, const double* u_box_dev,
                                double* u_tet_dev, void* stream);

/* ---- execution options and instrumentation ----------------------------- */

/* Replay MINRES iterations from captured HIP graphs (1, default) or launch
 * kernels one by one (0).  Results are bitwise identical either way. */
spde_status spde_set_graphs(spde_handle h, int enable);

/* Streams per spde_sample call: 2 runs a batch of 8 or more as two halves,
 * the second on a stream of the library's own, so that the kernels of one half
 * overlap those of the other; 1 (default) runs the batch as one.  The halves
 * meet at every convergence poll and the call returns when both are done; the
 * caller's stream sees the whole call as ordered work.  Results are bitwise
 * identical either way.  EINVAL for other values. */
spde_status spde_set_split(spde_handle h, int ways);

/* Face (flux) block of the MINRES preconditioner: 0 = diag(M)^-1;
 * 1 (default) = the truncated Neumann series q (I - S + S^2) of M^-1 along each
 * grid line (M = (1/q)(I + S) on a line, q = 3/(2h^3)).  Both are symmetric
 * positive definite; 1 takes about 20 % fewer iterations at no extra memory
 * traffic.  The multigrid V-cycle on the approximate Schur complement
 * kappa^2 W + B diag(M)^-1 B^T is the cell block in both cases. */
spde_status spde_set_face_preconditioner(spde_handle h, int kind);

/* Iterative refinement around the solve, in float64: after MINRES, the true
 * residual r = F - A U is formed with the flux recovered from U (so only its
 * cell row is nonzero); while ||r|| / ||F|| > target for a sample, and at most
 * max_passes times, A d = r is solved by the same preconditioned MINRES and
 * U += d for the samples above the target.  A sample's pass stops at the
 * relative tolerance 0.5 target / (its residual), kept within [rtol, 0.5].  This lets the mixed
 * precision (float32 multigrid) reach residuals far below its rtol.
 * target = 0 (default) turns refinement off; target in [0, 1), max_passes in
 * [0, 16].  Applies to spde_sample, spde_sample_seeded and spde_sample_warm
 * (not to the continuous-batching slots).  relres_host then reports the final residual at
 * no extra cost; a sample may stay above the target when max_passes runs out. */
spde_status spde_set_refinement(spde_handle h, double target, int max_passes);

/* A HIP stream whose kernels run only on the compute units whose bits are set
 * in mask[0 .. n_words) (host array, read during the call; bit i of word w:
 * mask position 32 w + i of the current device); default priority.  The
 * runtime deals consecutive mask positions out to the XCDs in turn, and fails
 * (SPDE_EHIP) for a mask that leaves an XCD with no compute unit.  For a server
 * that keeps some compute units free of its long kernels, so that short kernels
 * on other streams start at once.  Results do not depend on the mask, only
 * speed.  n_words in [1, 64], stream_out non-null, mask not all zero, else
 * SPDE_EINVAL.  The caller owns the stream: spde_stream_destroy releases it,
 * once no work, event or memory pool refers to it any more. */
spde_status spde_stream_create_cu_mask(int n_words, const uint32_t* mask, void** stream_out);
spde_status spde_stream_destroy(void* stream);

/* Autotuning of the multigrid tile shapes (default on).  When on, the first
 * sample or V-cycle call of a handle times every admissible tile shape of each
 * per-level kernel at max_batch and keeps the fastest; the choice is shared by
 * all handles of the process with the same device architecture, n, precision
 * and batch class of max_batch (1, 2..15, 16+), and is appended to the file named by the environment variable
 * SPDE_TUNE_CACHE (if set), from which later processes read it; with
 * SPDE_TUNE_VERBOSE=1 every timed shape is printed to stderr.  Off: fixed
 * default tiles.  Results depend on the tiles only through the rounding of
 * per-block partial sums (a few ulps): with the same tiles (spde_get_tiles after
 * a call, spde_set_tiles in another handle or process, or a shared
 * SPDE_TUNE_CACHE) a seeded sample is reproduced bit for bit. */
spde_status spde_set_autotune(spde_handle h, int enable);

/* Tile shape ids of the per-level multigrid kernels (level 0 = finest):
 *   3-D tiles (x*y*z cells):   0: 16x8x8  1: 8x8x8  2: 32x8x4  3: 16x16x4
 *                              4: 32x4x4  5: 16x8x4  (float64 up-kernels: 1, 4, 5 only)
 *   2.5-D columns x planes:    6: 32x8 x 32  7: 16x16 x 32  8: 32x8 x 16  9: 32x8 x 64
 *   pipelined 2.5-D columns:  10: 32x8 x 32 11: 16x16 x 32 12: 32x8 x 64 13: 16x16 x 64
 *                             14: 32x8 x 128 15: 16x16 x 128 16: 32x8 x 16 17: 16x16 x 16
 * spde_set_tiles fixes the shapes of one level (or all levels with level = -1)
 * and turns autotuning off for the handle; spde_get_tiles reads them. */
spde_status spde_set_tiles(spde_handle h, int level, int down_shape, int up_shape);
spde_status spde_get_tiles(spde_handle h, int level, int* down_shape, int* up_shape);

/* Iterations per convergence poll (default 8; 1..256). */
spde_status spde_set_poll_interval(spde_handle h, int iters);

/* Per-kernel timing with HIP events on the sampling stream; accumulated times
 * and algorithmic bytes are read with spde_timing_get().
 *   enable = 1: every kernel class; kernels are launched one by one (no
 *               graphs) with an event pair around each launch.
 *   enable = 2: the operator pass only: in each poll block the passes
 *               0, 3, 6, ... run on their own, bracketed by an event pair,
 *               and everything between them replays as captured graphs.
 *   enable = 0 stops and keeps the totals; -1 clears the totals (the mode
 *   is kept). */
spde_status spde_timing(spde_handle h, int enable);
int         spde_kernel_count(void);
const char* spde_kernel_name(int id);
spde_status spde_timing_get(spde_handle h, int id, double* total_ms, int64_t* launches,
                            double* bytes_per_launch);

/* Number of multigrid levels and the box edge of the coarsest level handled
 * by per-level kernels (levels below it run in one persistent launch). */
spde_status spde_info(spde_handle h, int* levels, int* persistent_top_n,
                      int* device_lds_bytes);

/* ---- teardown ------------------------------------------------------------ */

void        spde_free_host(void* p);
void        spde_destroy(spde_handle h);
const char* spde_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPDE_H */
