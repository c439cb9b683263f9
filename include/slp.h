/*
 * slp.h — smooth part of the single-layer potential by non-uniform FFT on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Exl & Schrefl, "Non-uniform FFT for the finite element computation of
 * the micromagnetic scalar potential". For a closed triangulated surface with
 * nodes x_i and a density g sampled at the three quadrature points of every
 * triangle, the library evaluates at every node
 *
 *   phi_s(x_i) = 1/(4 pi) sum_k w_k g_k K_F(x~_i - y~_k),
 *   K_F(xi)    = Re sum_{l in I_n} c_l(N_s) e^{2 pi i l.xi},
 *
 * the smooth part of the split kernel (Sec. 2.2, eq. approx2 and smooth_phi)
 * with N_s an exponential sum for 1/r (Sec. 3.3) and its Fourier coefficients
 * on the torus (eq. Fcoeff). It is computed as in eq. (convtheo) /
 * (BEM_NFFT_compact2): Gaussian gridding of the charges w_k g_k on the
 * oversampled grid (Sec. 3.1, eq. gridding), 3-D FFT (eq. FFT), deconvolution
 * and multiplication by c_l (eq. deconv, Alg. 1), inverse FFT and
 * interpolation at the nodes (type-2 NFFT).
 *
 * Conventions for every entry point:
 *  - Return value: SLP_OK (0) or a negative slp_status. No exception crosses
 *    the ABI. slp_last_error() returns a message for the calling thread's last
 *    failure (valid until that thread's next call).
 *  - "stream" is a hipStream_t (NULL = the legacy default stream). Work is
 *    enqueued asynchronously; the host returns before the device finishes.
 *  - Pointers documented as "host" are read during the call only. Pointers
 *    documented as "device" must stay valid until the stream has passed the
 *    work that reads or writes them. The library never frees caller memory.
 *  - A context (slp_geom) may be used by one stream at a time.
 *  - Index conventions: triangles are 0-based node triples, counter-clockwise
 *    seen from outside; quadrature point s (0..2) of triangle j has the long
 *    index k = j + s*M (eq. naive_gridding) and barycentric weight 2/3 on
 *    vertex s, 1/6 on the other two; its weight is |S_j|/3.
 */
#ifndef SLP_H
#define SLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLP_OK = 0,
  SLP_EINVAL = -1,    /* invalid argument, shape or parameter */
  SLP_ENOMEM = -2,    /* device or host allocation failed; nothing was created */
  SLP_EDEVICE = -3,   /* a HIP call failed (message names it) */
  SLP_EBUSY = -4,     /* server: no slot or memory free for the request now */
  SLP_ENOTREADY = -5  /* server: request not finished yet */
} slp_status;

typedef enum { SLP_FP64 = 0, SLP_FP32 = 1 } slp_precision;

/* Parameters of one geometry (Alg. 1, Require line: n in 2N^3, alpha >= 2,
 * cut-off m; and the exponential sum of Sec. 3.3). */
/* Window of the gridding and the NFFT (Sec. 3.2). Gaussian: exp(-tau^2 / b)
 * in grid units, b = 2 alpha m / ((2 alpha - 1) pi). Kaiser-Bessel (eq. KBfct):
 * sinh(b sqrt(m^2 - tau^2)) / sqrt(m^2 - tau^2) for |tau| <= m, b = pi (2 - 1/alpha),
 * whose error decays much faster in m (eq. error_bound_nufft). Both are
 * truncated to the 2m grid points floor(t) - m + 1 .. floor(t) + m per axis;
 * the deconvolution uses each window's Fourier coefficients (eq. cFB for KB). */
typedef enum { SLP_WINDOW_GAUSS = 0, SLP_WINDOW_KB = 1 } slp_window;

typedef struct {
  int32_t grid[3];        /* oversampled grid N_q = alpha * n_q; n_q even; power of two, 8..2048 */
  int32_t alpha;          /* oversampling factor alpha >= 2 (the paper fixes 2) */
  int32_t m;              /* window cut-off: 2m grid points per axis, 1 <= m <= 8 */
  int32_t precision;      /* slp_precision: FP32 runs gridding, FFT and interpolation in
                             FP32 with the per-node sum in FP64; kernel tables are built
                             in FP64 either way */
  const double *es_w;     /* host [es_terms]: exponential-sum weights omega_t (physical units) */
  const double *es_gamma; /* host [es_terms]: exponents gamma_t, 1/r ~ sum omega_t e^{-gamma_t r^2} */
  int32_t es_terms;       /* number of terms S (>= 1) */
  int32_t window;         /* slp_window: SLP_WINDOW_GAUSS (0) or SLP_WINDOW_KB (1), Sec. 3.2 */
  double eta2;            /* keep term t iff (pi n_q/2)^2 s_q^2 / gamma_t >= eta2 on every axis
                             (Sec. 5, eq. error_est3: eta^2 bounds the Fourier tail); 37 by default */
  int32_t seg_share;      /* gridding work split (no effect on the result beyond rounding
                             order): a tile holding more than 1.5 x seg_share sources is cut
                             into pieces of about seg_share sources, each gridded by its own
                             workgroup into its own block. 0 = automatic (the chip's
                             workgroup slots shared out evenly, at least 300 sources, 150
                             for FP64 with m = 8); otherwise
                             64 <= seg_share <= 2^24 (EINVAL outside). A timing autotuner
                             sets it; the automatic value is reported in slp_geom_info. */
  int32_t reduce_cells;   /* cells per thread of the gridding's block sum (no effect on the
                             result: each cell adds its terms in one fixed order either way):
                             1 (workgroups of 512 threads) or 2 (of 256); 0 = automatic, 2
                             where the region has 2048 tiles or more (times the densities of
                             a batched call), else 1; fused multi-geometry batches take the
                             automatic rule over all their items. EINVAL outside 0..2. A timing
                             autotuner sets it; the value in effect for one density is
                             reported in slp_geom_info. */
} slp_params;

typedef struct slp_geom slp_geom;   /* opaque; owns device tables and work buffers */

/* Geometry facts computed at setup (for tests and reports). */
typedef struct {
  double centre[3];       /* body centre c (bounding-box midpoint) */
  double scale[3];        /* x~ = s (x - c); s_q N_q equal on all axes, body in [-0.2, 0.2]^3 */
  double window_b;        /* window shape b: Gaussian 2 alpha m / ((2 alpha - 1) pi) (grid
                             units), Kaiser-Bessel pi (2 - 1/alpha) (eq. KBfct) */
  int64_t n_nodes, n_tris, n_src;
  int64_t n_targets;      /* evaluation points (n_nodes unless set up with targets) */
  int32_t terms_kept;     /* S' after the eta2 truncation */
  int32_t lo[3];          /* first grid index of the region touched by any stencil */
  int32_t extent[3];      /* its length per axis */
  int32_t tiles[3];       /* 8^3 tiles covering the region */
  int64_t device_bytes;   /* device memory held by the context */
  int64_t seg_share;      /* sources per gridding piece in effect (see slp_params) */
  int64_t n_segments;     /* gridding workgroups (padded blocks) per density */
  int32_t reduce_cells;   /* block-sum cells per thread for one density (see slp_params) */
} slp_geom_info;

/* Setup phase of Alg. 1 for one surface (Sec. 3.1-3.3). Scales the body into
 * (-0.2, 0.2)^3 of the torus, forms the quadrature sources, bins sources and
 * nodes by grid tiles, builds the Fourier coefficients of the kept
 * exponential-sum terms (eq. Fcoeff, FP64 on the device) and the combined
 * multiplier table, and allocates every work buffer.
 *   out     : receives the new context (NULL on failure)
 *   nodes   : host float64 [n_nodes][3], physical coordinates
 *   tris    : host int32 [n_tris][3], 0-based
 *   p       : host, see slp_params
 * Errors: EINVAL for non-finite coordinates, out-of-range node indices,
 * degenerate triangles, unsupported grid/m/alpha, or a stencil that would wrap
 * around the torus (m too large for the grid); ENOMEM; EDEVICE. */
int slp_setup_geometry(slp_geom **out, const double *nodes, int64_t n_nodes,
                       const int32_t *tris, int64_t n_tris, const slp_params *p,
                       void *stream);

/* As slp_setup_geometry, but the potential is evaluated at the given points
 * instead of the boundary nodes: the paper evaluates phi at every node of the
 * tetrahedral volume mesh (Sec. 2, Tables 3-4), which only changes the target
 * list of the interpolation. The body (its nodes) still sets the scaling.
 *   targets : host float64 [n_targets][3], physical coordinates
 * Errors as slp_setup_geometry; EINVAL also for non-finite targets and for
 * targets whose stencil would leave the grid (far outside the body's box). */
int slp_setup_geometry_targets(slp_geom **out, const double *nodes, int64_t n_nodes,
                               const int32_t *tris, int64_t n_tris, const double *targets,
                               int64_t n_targets, const slp_params *p, void *stream);

/* Device bytes slp_setup_geometry would hold for these arguments, computed on
 * the host without touching a device (same validation and errors). Used for
 * admission by memory. */
int slp_geometry_device_bytes(const double *nodes, int64_t n_nodes, const int32_t *tris,
                              int64_t n_tris, const slp_params *p, int64_t *bytes);

/* Density for the next slp_eval_single_layer on this context.
 *   dens : device float64 [3 * n_tris], density at the quadrature points in
 *          long-index order k = j + s*M. Only the pointer is recorded: the
 *          gridding of the next evaluation forms the charges q_k = w_k g_k
 *          (eq. naive_gridding) from it, so it must stay valid until that
 *          evaluation has run on its stream. */
int slp_set_density(slp_geom *g, const double *dens, void *stream);

/* Density of the paper's P1 ansatz (Sec. 2): g = m.n - dphi1/dn with m.n
 * projected onto element-wise constants by its integral mean over each flat
 * triangle (for affine m the mean of the three vertex values, dotted with the
 * unit outward normal from the vertex order), and dphi1/dn constant per
 * triangle. Every quadrature source of triangle j carries g_j. The density is
 * formed on `stream` in a buffer the context owns (allocated at setup) and
 * replaces any pointer recorded by slp_set_density for the next evaluation.
 *   m_nodes  : device float64 [n_nodes][3], nodal magnetisation (caller's node order)
 *   dphi1_dn : device float64 [n_tris], interior normal derivative of phi_1 per
 *              triangle, or NULL for zero (divergence-free m: phi_1 = 0)
 * Both need only stay valid until the call's kernel has run on `stream`. */
int slp_set_density_from_m(slp_geom *g, const double *m_nodes, const double *dphi1_dn,
                           void *stream);

/* phi_s at every target for the charges of the last slp_set_density
 * (computation phase of Alg. 1, smooth part).
 *   phi : device float64 [n_targets] (= n_nodes unless the context was set up
 *         with separate targets), written in the caller's order, physical
 *         units (the 1/(4 pi) of the Newton kernel included). */
int slp_eval_single_layer(slp_geom *g, double *phi, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as slp_eval_single_layer (same kernels, same result up to the
 * rounding order of the gridding's block accumulation), but every work buffer
 * of the evaluation (gridding blocks, region grid, half spectra, grid after
 * the inverse FFT, element means of a near field or of integrated-window
 * gridding) is carved out of one static device array of
 * SLP_STATIC_WORKSPACE_BYTES per device instead of the context's own buffers.
 * The call allocates nothing (no hipMalloc/hipFree); the first call on a
 * device looks up the array's address there. Evaluations whose work buffers
 * exceed the workspace fail with SLP_ENOMEM and a message giving the bytes
 * needed (cube64 with the Gaussian m = 8 in FP64 needs ~40 MiB; the 1024 x
 * 1024 x 64 film needs several hundred). Every call on a device shares that
 * device's array and leaves its contents behind (nothing in it has to start
 * at zero): calls whose work overlaps on one device, on any streams, race and
 * must be ordered by the caller. Direct kernel launches only (graph replay of
 * slp_set_graph does not apply). phi as for slp_eval_single_layer. */
#define SLP_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int slp_eval_single_layer_static(slp_geom *g, double *phi, void *stream);

/* Batched evaluation: item b uses geometry geoms[b], density dens[b] (device
 * float64 [3 * n_tris(geoms[b])]) and writes phi[b] (device float64
 * [n_targets(geoms[b])]). Repeating one geometry evaluates several densities on
 * one mesh. The work is ordered on `stream` (the call returns once it is
 * enqueued); the result equals calling set_density + eval for each item, up to
 * the rounding order of the gridding's block accumulation. geoms/dens/phi are
 * host arrays of length batch >= 1. Same as slp_eval_batched_mode with
 * SLP_BATCH_AUTO. */
int slp_eval_batched(slp_geom *const *geoms, const double *const *dens, double *const *phi,
                     int32_t batch, void *stream);

/* How slp_eval_batched_mode runs a batch (the steps of Sec. 3 per item either
 * way):
 *  SLP_BATCH_LANES  consecutive items on one geometry share every launch (the
 *                   density index is a launch dimension); the launch sequences
 *                   of different geometries overlap on four library streams
 *                   forked from and joined back into `stream`;
 *  SLP_BATCH_FUSED  one launch per stage for up to 64 items on any geometries
 *                   (gridding, block sum, each FFT pass once per line length,
 *                   interpolation), the workgroups taken from work lists in
 *                   device memory (the gridding's units longest first over all
 *                   items); the tables are built on the first call for a batch
 *                   composition (synchronous upload) and cached (8 per
 *                   process; eviction synchronises the device). Needs one
 *                   precision, cut-off m and window (kind and shape b) on every
 *                   item and the point-source gridding (SLP_EINVAL
 *                   otherwise); a near field is applied
 *                   per geometry after the interpolation. Stage timing
 *                   (slp_set_timing) and graph replay (slp_set_graph) do not
 *                   apply; a geometry occurring k times grows its per-item
 *                   buffers to k items;
 *  SLP_BATCH_AUTO   FUSED when the batch holds more than one geometry and
 *                   FUSED applies, else LANES.
 * Errors: SLP_EINVAL for NULL arrays or items, batch < 1 or an unknown mode;
 * SLP_ENOMEM when buffers or tables cannot be allocated. */
#define SLP_BATCH_AUTO 0
#define SLP_BATCH_LANES 1
#define SLP_BATCH_FUSED 2
int slp_eval_batched_mode(slp_geom *const *geoms, const double *const *dens, double *const *phi,
                          int32_t batch, int32_t mode, void *stream);

int slp_geom_get_info(const slp_geom *g, slp_geom_info *info);

/* Replay evaluations through HIP graphs (enable != 0) or launch every kernel
 * directly (0, the default). With graphs, the kernel sequence of one
 * evaluation with a given number of batch items is captured once (on first
 * use, on a stream of the context) and each later evaluation only updates the
 * density and result pointers of the gridding and interpolation launches and
 * launches the graph on the caller's stream: one submission instead of one per
 * kernel. The results are those of direct launches. Stage timing
 * (slp_set_timing) records only direct launches. Growing the batch capacity or
 * switching graphs off drops the captured graphs (synchronising the device). */
int slp_set_graph(slp_geom *g, int32_t enable);

/* Per-stage device timing. With every = k >= 1, every k-th evaluation (one
 * single eval, or one launch group of slp_eval_batched) records HIP events
 * around each stage on its stream: 0 gridding into per-segment blocks (charges
 * included), 1 sum of the blocks into the grid, 2 FFT x fwd, 3 FFT y fwd,
 * 4 FFT z (fwd, multiply, inv), 5 FFT y inv, 6 FFT x inv, 7 interpolation,
 * 8 near-field correction (zero time without one). Sampling keeps the cost of
 * the event packets off the other evaluations; every = 0 switches timing off.
 * slp_stage_times synchronises the recorded evaluations and accumulates into
 * ms[9] (summed since the last reset) and *count (recorded evaluations). */
int slp_set_timing(slp_geom *g, int32_t every);
int slp_stage_times(slp_geom *g, double *ms, int64_t *count, int32_t reset);

/* Copy an intermediate array of the last evaluation to a device buffer, for
 * stage-by-stage comparison (which: 0 = spread grid, region [P_z][P_y][P_x] with
 * P = 8*tiles; 1 = grid after the inverse FFT, [extent_z][extent_y][extent_x];
 * 2 = the float64 [3 n_tris] density formed by slp_set_density_from_m).
 * Values of 0 and 1 are in the context's precision; dst must hold the array. */
int slp_debug_copy(const slp_geom *g, int32_t which, void *dst, size_t dst_bytes, void *stream);

/* Cheapest window and cut-off m (alpha = 2) whose predicted relative error
 * against the definition is at most tol. Predicted error: the window's bound
 * divided by 5 (Kaiser-Bessel: eq. error_bound_nufft; Gaussian: 4 exp(-2 pi m/3)),
 * the factor measured on the sphere and cube workloads to stay 2-6x on the safe
 * side; FP32 adds a rounding floor of 2e-6.
 *   window_in : -1 any window, or SLP_WINDOW_GAUSS / SLP_WINDOW_KB to fix it
 *   window, m : receive the choice (the smaller m; Gaussian on a tie)
 * EINVAL if no m <= 8 reaches tol (or tol <= 0). Host only. */
int slp_choose_cutoff(double tol, int32_t precision, int32_t window_in, int32_t *window,
                      int32_t *m);

/* Exponential sum by the trapezoidal rule on 1/r = 2/sqrt(pi) int exp(-r^2 e^{2u} + u) du
 * (Sec. 3.3 uses a tabulated sum of this family): nodes u_t = u_lo + t h up to
 * u_hi = ln(7/r_lo), u_lo = ln(tol sqrt(pi) / (2 r_hi)); omega_t = 2 h e^{u_t}/sqrt(pi),
 * gamma_t = e^{2 u_t}. Host arrays of capacity cap; *count receives the number of
 * terms (EINVAL if cap is too small, with *count set to the required size). */
int slp_expsum_sinc(double h, double r_lo, double r_hi, double tol, double *omega,
                    double *gamma, int32_t cap, int32_t *count);

/* ---- Near-field correction (Sec. 3.4) -----------------------------------------
 * The kernel is split as 1/r = (1/r - N_s) + N_s (eq. splitting1) with N_s the
 * kept exponential-sum terms. The smooth part above carries N_s through its
 * Fourier series; the near field adds, for every target x_i and every triangle
 * S_j at distance d(x_i, S_j) <= eps (index set of eq. nf_index),
 *   phi_i += 1/(4 pi) gbar_j C_ij,                                  (eq. nfcorr)
 *   C_ij  = int_{S_j} dsigma(y) / |x_i - y| - |S_j|/3 sum_s N_s(|x_i - y_{j,s}|),
 * gbar_j the mean of the triangle's three density values (g_j itself for the
 * element-constant densities of the P1 ansatz). The first term is the exact
 * integral (closed form for flat triangles, so the weakly singular case needs
 * no special quadrature); the second removes the smooth kernel with the same
 * three-point rule the gridding uses, so that near pairs end up with the exact
 * integral of 1/r. With eps at least the radius from which N_s matches 1/r
 * (slp_near_radius), phi becomes the complete single-layer potential up to the
 * Fourier error of N_s and the three-point rule on the far pairs. */

/* Build the near field of a context: the index sets on the host (uniform cell
 * grid over triangle centroids, up to 16 threads), the matrix C on the device
 * (one FP64 value per pair; FP32 for an FP32 context), held as CSR over the
 * targets: int64 row offsets; rows padded to groups of 4 entries, or, when
 * rows average 2048 pairs or more, to chunks of 256 stored lane-interleaved
 * with their triangle indices packed as one int32 base per chunk plus a 16-bit
 * offset per entry (int32 indices if a chunk spans 65535 triangles or more).
 * Every later evaluation
 * of this context (single, batched, graph replay) adds phi_NF after the
 * interpolation. Geometries of a request server get theirs from
 * slp_server_add_geometry_near.
 * eps <= 0 removes the near field. The smooth kernel's share of a pair is
 * taken with the gridding's quadrature: the three-point rule, or the
 * collapsed rule of slp_setup_integrated_gridding when that is set.
 * Synchronises `stream` and the device; drops captured graphs.
 *   eps : physical distance, the paper's eps of Alg. 1 (Require line)
 * Errors: EINVAL for non-finite eps; ENOMEM when the pattern does not fit in
 * host or device memory (the context is left without a near field). */
int slp_setup_near_field(slp_geom *g, double eps, void *stream);

/* As slp_setup_near_field, with the values C_ij stored in `storage`
 * (SLP_FP64 or SLP_FP32) whatever the context's precision (slp_setup_near_field
 * stores them in the context's). They are computed in FP64 either way and
 * rounded once when stored; the product accumulates in FP64. The product is
 * bound by HBM, so FP32 storage in an FP64 context moves 4 + 2 instead of
 * 8 + 2 bytes per packed entry, at a relative rounding of the stored
 * correction of 2^-24 per entry. The choice persists when the near field is
 * rebuilt by slp_setup_integrated_gridding. EINVAL for another storage. */
int slp_setup_near_field_stored(slp_geom *g, double eps, int32_t storage, void *stream);

/* Smallest eps on the scan r_k = r_max * 0.999^k (k = 0, 1, ...), r_max the
 * bounding-box diagonal of nodes and targets, from which up to r_max the kept
 * exponential sum matches 1/r to |N_s(r) r - 1| <= tol at every scan point
 * (Sec. 3.3: the truncated sum is accurate on [eps, 1/2] only). EINVAL if
 * tol <= 0 or if r_max itself misses tol. Host only. */
int slp_near_radius(const slp_geom *g, double tol, double *eps);

/* Device bytes slp_setup_near_field(eps) would add for this mesh and these
 * targets (NULL: the nodes) with values stored in this precision, computed on the host (index
 * sets and storage layout included, so it costs what the setup's host part
 * costs). 0 for eps <= 0 or an empty near field. Used for admission by memory. */
int slp_near_field_device_bytes(const double *nodes, int64_t n_nodes, const int32_t *tris,
                                int64_t n_tris, const double *targets, int64_t n_targets,
                                double eps, int32_t precision, int64_t *bytes);

/* eps, pairs (nnz), r_max, stored entries (pairs plus row padding) and whether
 * the columns are packed, of a context (any pointer may be NULL). */
int slp_near_field_info(const slp_geom *g, double *eps, int64_t *nnz, double *r_max,
                        int64_t *stored, int32_t *packed);

/* Integrated-window gridding (Sec. 3.1, eq. gridding2 and the matrix A of
 * eq. A): the paper's own gridding, in which the window is integrated over
 * each triangle in the setup phase instead of being sampled at the three
 * quadrature points, A_rj = int_{S_j} Psi(r - t(y)) dsigma(y) over the index
 * box of S_j (eq. indexset2: floor(t_min) - m + 1 .. floor(t_max) + m per
 * axis). The integrals are taken on the device with the collapsed Gauss rule
 * (xi_1 = u (1 - v), xi_2 = u v, `order` Gauss-Legendre points in u and in v)
 * and stored by grid cell; every evaluation then grids a_r = sum_j A_rj g_j,
 * g_j the mean of the density's three values on S_j (the element density
 * of the paper's P1 ansatz), instead of gridding the point sources. The rest
 * of the evaluation is unchanged.
 *   order : 1..16 Gauss points per direction (8 resolves the window to
 *           rounding on meshes whose triangles are about a grid cell); 0
 *           returns to the point gridding
 * A near field of the context (slp_setup_near_field, before or after) then
 * subtracts the smooth kernel integrated over S_j with the same rule, so that
 * near pairs still carry the exact integral of 1/r; switching the gridding
 * rebuilds it. Synchronises `stream` and the device. Errors: EINVAL for an
 * order out of range, a triangle whose index box leaves the grid region (the
 * nodes must be among the evaluation points), or a context with captured
 * evaluations (they do not combine with it); ENOMEM. After a failed call the
 * context grids the point sources; an evaluation with a near field built for
 * the other gridding fails with EINVAL until the near field is set up again. */
int slp_setup_integrated_gridding(slp_geom *g, int32_t order, void *stream);
/* order (0 = off), stored window integrals (nnz), entries including the row
 * padding and whether the columns are packed (any pointer may be NULL). */
int slp_integrated_gridding_info(const slp_geom *g, int32_t *order, int64_t *nnz, int64_t *stored,
                                 int32_t *packed);

/* Copy the near-field matrix to host memory (synchronises the device):
 * rowptr int64 [n_targets + 1], cols int32 [nnz] (may be NULL), vals float64
 * [nnz] (may be NULL; FP32 values converted). cap = room in cols / vals;
 * EINVAL if it is below nnz. */
int slp_debug_copy_near(const slp_geom *g, int64_t *rowptr, int32_t *cols, double *vals,
                        int64_t cap);

/* Host-only versions of the near-field building blocks (no device needed).
 * slp_near_pattern_host: the index sets as CSR; pass cols = NULL to learn nnz
 * (EINVAL if cols_cap < nnz), rowptr int64 [n_targets + 1] may be NULL.
 * slp_triangle_potential_host: out[i] = int over the flat triangle
 * (a_i, b_i, c_i) of 1/|x_i - y|, all arrays [count][3] float64.
 * slp_near_radius_host: the radius of slp_near_radius for given terms and r_max. */
int slp_near_pattern_host(const double *nodes, int64_t n_nodes, const int32_t *tris,
                          int64_t n_tris, const double *targets, int64_t n_targets, double eps,
                          int64_t *rowptr, int32_t *cols, int64_t cols_cap, int64_t *nnz);
int slp_triangle_potential_host(const double *x, const double *a, const double *b,
                                const double *c, int64_t count, double *out);
int slp_near_radius_host(const double *es_w, const double *es_gamma, int32_t terms, double r_max,
                         double tol, double *eps);

/* ---- Dirichlet problem for phi_1 and the complete scalar potential ------------
 * Sec. 2 splits phi = phi_1 + phi_2: -Laplace phi_1 = -div m in the body with
 * phi_1 = 0 on its boundary (eq. GR1), solved by P1 finite elements on a
 * tetrahedral mesh (Sec. 2.1: weak form eq. varu1, free-node system eq.
 * poisson), and phi_2 the single-layer potential of g = m.n - d phi_1/dn
 * (eq. slayer). Alg. 1's computation phase is slp_scalar_potential. */
typedef struct slp_fem slp_fem;   /* opaque; owns the mesh tables and the solver buffers */

/* Setup for a tetrahedral mesh: gradients of the barycentric coordinates and
 * volumes, the boundary triangles (faces of exactly one tetrahedron, oriented
 * outward, ordered by their sorted vertex triple), the free (interior) nodes,
 * and the stiffness matrix on the free nodes S_km = sum_T int grad eta_m .
 * grad eta_k as CSR (FP64), all held on the device.
 *   nodes : host float64 [n_nodes][3];  tets : host int32 [n_tets][4], 0-based
 * Errors: EINVAL for indices out of range, non-finite coordinates, degenerate
 * tetrahedra, faces shared by more than two tetrahedra or a mesh without
 * boundary; ENOMEM; EDEVICE. */
int slp_fem_setup(slp_fem **out, const double *nodes, int64_t n_nodes, const int32_t *tets,
                  int64_t n_tets, void *stream);
/* Free nodes, boundary triangles, stored entries of S_ff (entries whose
 * element contributions cancel to within rounding are not stored) and device
 * bytes (any pointer may be NULL). */
int slp_fem_info(const slp_fem *f, int64_t *n_free, int64_t *n_boundary_tris, int64_t *nnz,
                 int64_t *device_bytes);
/* The boundary triangles, host int32 [n_boundary_tris][3] (cap = room, in
 * triangles): the surface mesh to hand to slp_setup_geometry together with all
 * nodes (so that the targets are every node), in the order of dphi1_dn. */
int slp_fem_boundary(const slp_fem *f, int32_t *tris, int64_t cap);
/* Preconditioner of the conjugate gradients on the free-node system (Sec. 2.1
 * names algebraic-multigrid preconditioned CG among the solvers of eq.
 * poisson). SLP_PRECOND_JACOBI (the default): z = D^-1 r. SLP_PRECOND_AMG:
 * one V(1,1) cycle of smoothed-aggregation multigrid (aggregates of strongly
 * connected nodes, |a_ij| >= theta sqrt(a_ii a_jj) with theta = 0.08 halved
 * per level; prolongation = one damped-Jacobi step applied to the piecewise
 * constants; Galerkin coarse operators P^T A P; damped-Jacobi pre- and
 * post-smoothing; every Jacobi step with the l1 weights (4/3) / sum_j |a_ij|;
 * the coarsest operator, at most 512 unknowns, inverted densely), a symmetric
 * positive definite preconditioner. Selecting it the first time builds the
 * hierarchy on the host and copies it to the device (synchronising `stream`).
 * Errors: EINVAL for an unknown kind or a hierarchy that cannot be built
 * (stalled aggregation, coarsest operator not positive definite); ENOMEM. */
#define SLP_PRECOND_JACOBI 0
#define SLP_PRECOND_AMG 1
int slp_fem_set_preconditioner(slp_fem *f, int32_t kind, void *stream);
/* Sizes and stored entries of the operators of the hierarchy, finest first
 * (the last is the dense coarsest inverse): rows, nnz host int64 [cap] (either
 * may be NULL). EINVAL before SLP_PRECOND_AMG was selected or if cap is too
 * small for *n_levels. */
int slp_fem_amg_info(const slp_fem *f, int32_t *n_levels, int64_t *rows, int64_t *nnz,
                     int32_t cap);
/* Host only (no device work): the mesh analysis and stiffness assembly of
 * slp_fem_setup (eq. varu1 / poisson: S_ij = sum_T |T| grad eta_i . grad eta_j
 * over the free, i.e. non-boundary, nodes; entries whose element contributions
 * cancel to within their rounding are not stored). *n_free and *nnz receive
 * the sizes; the arrays (host, may be NULL to learn the sizes first): rowptr
 * int64 [n_free + 1], cols int32 [nnz] (free-node numbers, ascending per row),
 * vals float64 [nnz], free_nodes int32 [n_free] (the mesh node of each free
 * node). Errors as slp_fem_setup. */
int slp_fem_assemble_host(const double *nodes, int64_t n_nodes, const int32_t *tets,
                          int64_t n_tets, int64_t *n_free, int64_t *nnz, int64_t *rowptr,
                          int32_t *cols, double *vals, int32_t *free_nodes);
/* Host-only: builds the hierarchy of SLP_PRECOND_AMG for the symmetric
 * positive definite CSR matrix (rowptr int64 [n + 1], cols int32, vals float64,
 * host memory) and applies one cycle on the host, z = B r (host float64 [n]),
 * with the steps of the device cycle; n_levels receives the operator count
 * (may be NULL). For testing the hierarchy without a device. EINVAL for a
 * malformed matrix or a hierarchy that cannot be built; ENOMEM. */
int slp_amg_apply_host(int64_t n, const int64_t *rowptr, const int32_t *cols, const double *vals,
                       const double *r, double *z, int32_t *n_levels);
/* phi_1 at every node (0 on the boundary): load vector b_k = sum_T |T| mbar_T .
 * grad eta_k (m the nodal P1 field, mbar_T its vertex mean), then
 * preconditioned conjugate gradients on the free nodes until |r| <= tol |b|
 * or max_iter iterations. The residual is checked every 16 iterations with
 * Jacobi; with the multigrid cycle after 4 and 8 iterations, then where the
 * rate between the last two checks predicts tol (1 to 8 iterations later).
 *   m_nodes : device float64 [n_nodes][3];  phi1 : device float64 [n_nodes]
 *   warm_start != 0: start from the free-node values phi1 holds
 *   iters, rel_res : receive the iterations done and |r|/|b| (may be NULL)
 * Synchronises `stream` at every check. EINVAL if tol is not met (phi1 then
 * holds the last iterate). */
int slp_fem_solve_phi1(slp_fem *f, const double *m_nodes, double *phi1, double tol,
                       int32_t max_iter, int32_t warm_start, int32_t *iters, double *rel_res,
                       void *stream);
/* d phi_1/dn on every boundary triangle: the gradient of the P1 function phi_1
 * in the tetrahedron owning the face, dotted with its unit outward normal.
 *   phi1 : device float64 [n_nodes];  dphi1_dn : device float64 [n_boundary_tris] */
int slp_fem_dphi1_dn(slp_fem *f, const double *phi1, double *dphi1_dn, void *stream);
/* Computation phase of Alg. 1: phi_1 (as slp_fem_solve_phi1, into a buffer of
 * the context; warm_start reuses the previous call's phi_1), d phi_1/dn, the
 * element density g = mean(m.n) - d phi_1/dn (slp_set_density_from_m), phi_2 at
 * every node (slp_eval_single_layer: smooth part, plus the near-field
 * correction if g has one), and phi = phi_1 + phi_2.
 *   g   : a context set up with all of the mesh's nodes as nodes (hence as
 *         targets) and the triangles of slp_fem_boundary
 *   phi : device float64 [n_nodes]
 * EINVAL if g does not match the mesh or the solve misses tol. */
int slp_scalar_potential(slp_fem *f, slp_geom *g, const double *m_nodes, double *phi, double tol,
                         int32_t max_iter, int32_t warm_start, int32_t *iters, void *stream);
/* Stray-field energy E = -(1/2) int m . H = (1/2) int m . grad phi (units of
 * mu_0 Ms^2 times length^3; the quantity of Tables 3-4): with m the nodal P1
 * field and phi a P1 potential (e.g. from slp_scalar_potential), each
 * tetrahedron contributes |T| mbar_T . grad phi_T exactly. The paper forms the
 * field by mass lumping, which gives the same value for uniform m.
 *   m_nodes : device float64 [n_nodes][3];  phi : device float64 [n_nodes]
 * Synchronises `stream`; the sum over tetrahedra is taken in a fixed order. */
int slp_fem_energy(slp_fem *f, const double *m_nodes, const double *phi, double *energy,
                   void *stream);
int slp_fem_destroy(slp_fem *f);

int slp_geom_destroy(slp_geom *g);
const char *slp_last_error(void);

/* ---- Queued / served evaluation ----------------------------------------------
 * A server owns a worker thread, n_slots HIP streams and a device-memory budget.
 * Registered geometries are built on the device when first needed (setup phase
 * of Alg. 1) and stay resident; when admitting one would exceed the budget, idle
 * geometries are evicted, least recently used first, and rebuilt on their next
 * request. Requests are admitted in arrival order as slots and memory free up,
 * except that a request whose geometry is already running never blocks later
 * requests for other geometries. The pending requests of one geometry are
 * coalesced into one batched evaluation (as slp_eval_batched; up to 8 per
 * launch, as many as the geometry's work buffers were sized for at setup, which
 * counts towards the budget), launched on a free stream or chained behind the
 * geometry's running work (continuous batching, up to 4 launches in flight per
 * stream). Once an older request waits for a stream or for memory, nothing more
 * is chained onto busy streams, so waiting is bounded under any load. A device
 * error fails the requests of its launch only. A geometry larger than the whole
 * budget fails its requests with SLP_ENOMEM. The server calls are thread-safe;
 * submissions never wait for setups, evictions or launches (a worker thread
 * does those). Latency is measured from the moment slp_server_submit is
 * entered. Statistics reset (slp_server_get_stats with reset != 0) clears the
 * latencies and every counter. */
typedef struct slp_server slp_server;

typedef struct {
  double p50_s, p99_s, mean_s;  /* latency of completed requests, submit -> result ready */
  double pts_per_s;             /* sum of (M_q + N) over completed requests / (last completion -
                                   first submission) */
  int64_t completed, failed, queued, in_flight;
  int64_t resident_bytes, setups, evictions;
  int64_t launches;             /* batched launches that served the completed requests */
} slp_server_stats;

/* n_slots in [1, 64] streams; device_budget_bytes > 0 bounds the device memory
 * held by resident geometries. Uses the calling thread's current device. */
int slp_server_create(slp_server **out, size_t device_budget_bytes, int32_t n_slots);
/* Register a geometry (host arrays copied; same meaning as slp_setup_geometry,
 * p->es_w / p->es_gamma copied as well). *geom_id receives its id (>= 0). */
int slp_server_add_geometry(slp_server *s, const double *nodes, int64_t n_nodes,
                            const int32_t *tris, int64_t n_tris, const slp_params *p,
                            int64_t *geom_id);
/* As slp_server_add_geometry, with the near-field correction within eps
 * (physical units, eps <= 0: none) built whenever the geometry is set up; its
 * memory (slp_near_field_device_bytes) counts towards the budget. */
int slp_server_add_geometry_near(slp_server *s, const double *nodes, int64_t n_nodes,
                                 const int32_t *tris, int64_t n_tris, const slp_params *p,
                                 double eps, int64_t *geom_id);
/* Queue one solve: dens device float64 [3 * n_tris], phi device float64 [n_nodes]
 * (caller owned; both must stay valid until the request is done).
 * *ticket identifies the request. */
int slp_server_submit(slp_server *s, int64_t geom_id, const double *dens, double *phi,
                      uint64_t *ticket);
/* *done = 1 once phi is written (status SLP_OK) or the request failed (its negative
 * status is returned); 0 while queued or running. */
int slp_server_poll(slp_server *s, uint64_t ticket, int32_t *done);
/* Block until the request is done (SLP_OK), failed (its status) or timeout_s passed
 * (SLP_ENOTREADY); timeout_s <= 0 waits without limit. */
int slp_server_wait(slp_server *s, uint64_t ticket, double timeout_s);
int slp_server_get_stats(slp_server *s, slp_server_stats *st, int32_t reset);
/* Finishes every admitted request, then frees streams and resident geometries. */
int slp_server_destroy(slp_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SLP_H */
