// Internal declarations shared by the host API (slp_api.cpp) and the device
// code (slp_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slp {

constexpr int kTile = 8;      // edge of the grid tiles that sort sources and targets
constexpr int kMaxM = 8;      // largest supported window cut-off

// Gridding (type-1 spread). Sources are sorted by (tile, cell in tile). The
// sources of one tile form a segment (tiles with far more sources than the
// average share of a workgroup slot are cut into several); every segment owns a
// padded accumulation block of (8 + 2m - 1)^3 cells in `scratch` (slot =
// segment index, the segments of a tile consecutive; blocked layout, see
// pad_block_index). A work unit (one workgroup) takes a list of segments; the
// setup gives every unit one segment, longest first. A segment is cut into
// chunks of at most spread_chunk(fp64, m) sources; a run is a sequence of
// sources of one chunk that share one grid cell. FP64 with m = 4 stages fewer
// sources per chunk so that its larger factor batches (ten sources per run)
// still leave two gridding workgroups per CU.
constexpr int spread_chunk(bool fp64, int m) { return fp64 && m == 4 ? 448 : 512; }
// Units are sized for this many compute units (MI355X).
constexpr int kComputeUnits = 256;
// Densities evaluated on one geometry by one launch of every stage.
constexpr int kMaxBatch = 64;

// Static device workspace of the evaluation that allocates nothing
// (slp_eval_single_layer_static): one array of this many bytes per device,
// held from the moment the library is loaded on that device until the process
// ends. static_workspace() returns its device address on the current device.
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_workspace(void **ptr);

// Kaiser-Bessel window factors in the gridding and interpolation kernels: on
// each unit interval of the stencil the window is a polynomial in
// u = 2 (t - floor(t)) - 1, fitted on the host at setup by interpolation at the
// Chebyshev points of that degree (max error over the interval, relative to
// the window's peak: below 1e-14 in FP64 at degree 16 for m <= 2 and at
// degree 14 for m >= 3, below FP32 rounding at degree 8, for every
// m <= kMaxM). Coefficients of stencil point j at [j * (deg + 1) + d],
// d = 0 .. deg (monomial, ascending).
constexpr int kKbDeg64 = 16;
constexpr int kKbDeg32 = 8;
constexpr int kKbCoef = 2 * kMaxM * (kKbDeg64 + 1);
constexpr int kb_degree(bool fp64, int m) { return fp64 ? (m <= 2 ? kKbDeg64 : 14) : kKbDeg32; }
template <typename T, int M>
constexpr int kb_degree() { return kb_degree(sizeof(T) == 8, M); }

// Per-item caller pointers of a batched launch (passed by value).
struct BatchPtrs {
  const double *dens[kMaxBatch];
  double *phi[kMaxBatch];
};
template <typename T>
struct SpreadBinsArgs {
  const T *frac;         // [3][ns] t - floor(t), sorted order
  const double *w;       // [ns] quadrature weights, sorted order
  const int32_t *perm;   // [ns] sorted -> caller (long) index of the density
  const int4 *units;         // [n_units][2] {slot (segment), first chunk, end chunk, reach box
                             // of the tile}, the first chunk's record
  const int4 *chunks;        // {first source, source count, first run, run count}
  const int32_t *runs;       // cell x | y << 3 | z << 6 | offset in chunk << 9 | count << 19
  T *scratch;            // [n_slots][PD^3], blocked layout
  int64_t ns;
  int64_t scratch_bstride;   // per batch item (blockIdx.y)
  T inv_b;               // 1 / b of the Gaussian exp(-tau^2 / b)
  T step_ratio;          // exp(-2 / b): ratio of consecutive weight ratios
  int32_t window;        // 0 Gaussian (recurrence), 1 Kaiser-Bessel
  T kb_c[kKbCoef];       // Kaiser-Bessel window polynomials (see kKbDeg64)
};

// Sum of the padded blocks of the segments in the neighbouring tiles into the
// region grid.
template <typename T>
struct SpreadReduceArgs {
  const T *scratch;
  const int4 *tile_slots;        // [tiles] {first slot, slot count, reach box, 0}: the pad
                                 // cells the tile's sources reach, lo x | y << 5 | z << 10,
                                 // hi << 15 | << 20 | << 25 (inclusive)
  T *grid;                       // [P_z][P_y][P_x]
  int32_t tiles[3];
  int64_t scratch_bstride, grid_bstride;
};

// Interpolation (type-2 gather) at the tile-sorted targets.
template <typename T>
struct InterpArgs {
  const int32_t *cell;   // [3][nt] local cell, sorted by tile
  const T *frac;         // [3][nt]
  const int32_t *perm;   // [nt] sorted -> caller index
  const int4 *rec;       // [n_active] tiles holding targets, most targets first: {tile, first
                         // target, end target, cell box of its targets: lo x|y<<3|z<<6,
                         // hi <<9|<<12|<<15}
  const T *g;            // [R_z][R_y][R_x] grid after the inverse FFT
  int64_t g_bstride;
  int32_t R[3];
  int32_t tiles[3];
  int64_t nt;
  T inv_b;
  int32_t window;
  const T *kb_tab;           // [2m (deg + 1)] Kaiser-Bessel window polynomials (see kKbDeg64)
};

// One batched 1-D FFT pass over "lines" of a 3-D array. Element e of line L is
// read at in + (L % l1) * in_s1 + (L / l1) * in_s2 + e * in_es and placed at
// LDS position (e + in_shift) mod N; after the transform, position
// (e + out_shift) mod N is written to the analogous output address.
template <typename T>
struct FftPass {
  const void *in;
  void *out;
  const void *tw;        // [N] e^{-2 pi i k / N}
  const T *mu;           // fused multiplier (mode kMulInv), same addressing as `in`
  int64_t n_lines;
  int64_t l1;
  int64_t in_s1, in_s2, in_es;
  int64_t out_s1, out_s2, out_es;
  int32_t in_cnt, in_shift;
  int32_t out_cnt, out_shift;
  int32_t mu_cnt, mu_shift;
  // fused multiplier: mu = h(l) F(kx, |ky|, |kz|), F folded over the signs of
  // ky and kz ([n_z/2 + 1][n_y/2 + 1][n_x/2 + 1]); line (kx, ky index) of the z
  // pass, element kz index = (pos - mu_shift) mod N
  int32_t mu_n[3];       // n_x, n_y, n_z
  int32_t sign;          // -1 forward, +1 inverse
  int32_t in_real;       // input is real (T) instead of complex
  int32_t in_hermitian;  // also place conj(v_e) at N - e (e >= 1)
  int32_t out_real;      // store the real part only
  int32_t mul_inv;       // forward, multiply by mu (zero elsewhere), inverse
  int64_t in_bstride, out_bstride;   // per batch item (blockIdx.y)
};

// Region tiles (times batch items) from which the block sum takes two cells
// per thread in workgroups of 256 when left automatic (below: one cell per
// thread in workgroups of 512). Both forms add a cell's terms in one order.
constexpr int64_t kReduceTwoCells = 2048;

// Every launch covers nb batch items (gridDim.y = nb, 1 <= nb <= kMaxBatch).
// The gridding forms the charges q = w g itself from the density pointers.
// cells: block-sum cells per thread, 1 or 2, 0 = automatic (kReduceTwoCells).
template <typename T>
hipError_t launch_spread(const SpreadBinsArgs<T> &a, const SpreadReduceArgs<T> &r,
                         const BatchPtrs &p, int n_units, int m, int nb, int cells, hipStream_t s,
                         hipEvent_t between);   // recorded between the two kernels if set
// Work units per compute unit for the gridding kernel of cut-off m (how many
// of its workgroups fit in one CU's LDS, at most 2). Host-only.
int spread_units_per_cu(int m, bool fp64);
template <typename T>
hipError_t launch_interp(const InterpArgs<T> &a, const BatchPtrs &p, int n_active, int m, int nb,
                         hipStream_t s);
// Cells of the padded accumulation block of one segment: (8 + 2m - 1)^3.
int64_t pad_cells(int m);
template <typename T>
hipError_t launch_fft(const FftPass<T> &p, int N, int nb, hipStream_t s);

// Fused launches over several geometries (a batch of different meshes): one
// launch per stage for all items, an item being one density on one geometry.
// The arguments of every item sit in a device table, the pointers of its work
// buffers already offset to that item (the batch-stride fields are unused);
// a work list in device memory maps workgroup i to {item, unit} (gridding:
// work unit; block sum: region tile; interpolation: position in `rec`).
// The density and potential of item i are p.dens[i] and p.phi[i] (at most
// kMaxBatch items per launch). The gridding's window (window, inv_b,
// step_ratio, kb_c of `win`; its other fields unused) is one for all items.
template <typename T>
struct MultiItem {
  SpreadBinsArgs<T> sp;
  SpreadReduceArgs<T> rd;
  InterpArgs<T> ip;
};
template <typename T>
hipError_t launch_spread_multi(const MultiItem<T> *items, const int2 *bins_work, int64_t n_bins,
                               const int2 *red_work, int64_t n_red, int m, const BatchPtrs &p,
                               const SpreadBinsArgs<T> &win, hipStream_t s);
template <typename T>
hipError_t launch_interp_multi(const MultiItem<T> *items, const int2 *work, int64_t n, int m,
                               const BatchPtrs &p, hipStream_t s);
// The kernel that launch_fft uses for pass p of length N (an id >= 0 shared
// by passes that can go into one fused launch), with the workgroups one item
// of it takes in *blocks; -1 if launch_fft rejects the pass. Host-only.
template <typename T>
int fft_variant(const FftPass<T> &p, int N, int64_t *blocks);
// One launch of that kernel over several passes: workgroup i (after the
// same XCD-aware renumbering as launch_fft) takes block work[i].y of pass
// work[i].x of the device table `passes`.
template <typename T>
hipError_t launch_fft_multi(int variant, int N, const FftPass<T> *passes, const int2 *work,
                            int64_t n, hipStream_t s);

// Host handles of the two kernels that take the per-item pointers (their
// launches are updated in place when a captured evaluation is replayed).
template <typename T>
const void *spread_bins_kernel(int m);
template <typename T>
const void *interp_kernel(int m);

// Near-field correction (Sec. 3.4, eq. nfcorr). CSR over the targets: row i
// lists the triangles j within eps of target i (eq. nf_index) with
//   C_ij = int_{S_j} dsigma / |x_i - y| - |S_j| / 3 sum_s N_s(|x_i - y_{j,s}|),
// N_s the kept exponential sum (physical units), y_{j,s} the three quadrature
// points of triangle j.
// Rows are stored in groups of four entries: every row starts at a multiple of
// four and is padded to one with entries of column -1 and value 0, so that a
// lane reads four entries with one 16-byte column load. When rows are long,
// they are padded to chunks of 4 x 64 entries instead, and within a chunk the
// group of lane l holds entries l, l + 64, l + 128, l + 192: the four density
// gathers of a wave then read consecutive triangles of the sorted row.
constexpr int kNearGroup = 4;
constexpr int kNearChunk = 4 * 64;
// Chunked rows may also store their columns packed: one int32 base per chunk
// and a 16-bit offset per entry (padding: offset 0, value 0), used when every
// chunk spans fewer than 65535 triangles.
template <typename T>
struct NearArgs {
  const int64_t *rowptr;   // [rows + 1], multiples of kNearGroup (kNearChunk if chunked)
  const int32_t *cols;     // triangle of each entry, -1 = padding (values kernel; the
                           // product too unless packed)
  const int32_t *bases;    // packed: [stored / kNearChunk] smallest triangle of each chunk
  const uint16_t *offs;    // packed: [stored] triangle - base
  T *vals;                 // C_ij (0 on padding)
  double *gbar;            // [items][M] element means of the densities of one launch
  int64_t rows;            // targets
  int64_t M;               // triangles; density value s of triangle j at j + s M
};
// Fills a.vals from the pattern. targets [rows][3], nodes [n][3], tris [M][3]
// (device, FP64 physical coordinates); es_w / es_g [terms] the kept terms;
// rule [npts][3] the collapsed rule of integrated-window gridding, or null for
// the three-point rule.
template <typename T>
hipError_t launch_near_values(const NearArgs<T> &a, const double *targets, const double *nodes,
                              const int32_t *tris, const double *es_w, const double *es_g,
                              int32_t terms, const double *rule, int32_t npts, hipStream_t s);
// phi_i += 1/(4 pi) sum_j C_ij gbar_j for every batch item, gbar_j =
// (g_j + g_{j+M} + g_{j+2M}) / 3 formed first into a.gbar (density and
// potential from the per-item pointers). Up to eight items share one pass over
// the matrix.
template <typename T>
hipError_t launch_near_apply(const NearArgs<T> &a, const BatchPtrs &p, int nb, bool packed,
                             hipStream_t s);
// Integrated-window gridding (Sec. 3.1, eq. gridding2, the matrix A): the
// window integrated over each triangle, stored by cell of the region in the
// near-field layout (rows = region cells x + R_x (y + R_y z), columns =
// triangles), evaluated as a = A gbar into the region grid.
struct IwGeom {
  const double *tv;      // [M][3][3] vertex coordinates in grid units
  const double *area;    // [M] physical areas
  const double *rule;    // [npts][3] collapsed Gauss rule on the unit triangle: xi_1, xi_2, weight
  int32_t npts;
  int32_t lo[3], R[3];   // region origin (grid index) and extent
  int32_t m, window;     // cut-off; 0 Gaussian exp(-tau^2 / b), 1 Kaiser-Bessel
  double inv_b, b, kb_inv_norm;
};
template <typename T>
struct IwOut {
  T *grid;               // region grid of item 0, [P_z][P_y][P_x]
  int64_t bstride;       // elements between items
  int32_t R[3], P[3];
};
template <typename T>
hipError_t launch_iw_values(const NearArgs<T> &a, const IwGeom &g, hipStream_t s);
// Element means of the densities (into a.gbar), then the product; short_rows
// (unpacked rows of fewer than 512 stored entries on average) puts four cells
// on a wave instead of one.
template <typename T>
hipError_t launch_iw_apply(const NearArgs<T> &a, const IwOut<T> &o, const BatchPtrs &p, int nb,
                           bool packed, bool short_rows, hipStream_t s);
// Host handles of the two kernels of launch_near_apply (the element means, the
// product), whose per-item pointers are updated when a captured evaluation is
// replayed.
const void *near_gbar_kernel();
template <typename T>
const void *near_apply_kernel(int nb, bool packed);

}  // namespace slp

struct slp_geom;

namespace slp {

// For the request server (host only): bytes of one item's work buffers; grow a
// context's work buffers to nb items (synchronises `s`, and the device only if
// captured graphs of the context may still run); destroy a context whose
// launches have all completed (no device-wide synchronisation).
int64_t item_device_bytes(const slp_geom *g);
int reserve_items(slp_geom *g, int nb, hipStream_t s);
void destroy_idle(slp_geom *g);

// Message returned by slp_last_error() on the calling thread.
void set_error_message(const char *msg);

// g_j = (m_a + m_b + m_c) . n_j / 3 - dphi1_dn[j] for every triangle j, written to
// dens[j], dens[j + M], dens[j + 2M] (one value per quadrature source).
hipError_t launch_density_from_m(const int32_t *tri_v, const double *tri_n, const double *m_nodes,
                                 const double *dphi1_dn, int64_t n_tris, double *dens,
                                 hipStream_t s);

// FP64 setup kernels.
hipError_t launch_chat(double *C, const double *gamma_scaled, int32_t S, int32_t L,
                       const double *gl_x, const double *gl_w, int32_t order, int32_t panels,
                       hipStream_t s);
// F(kx, |ky|, |kz|) = c_l dec_x[kx] dec_y[|ky|] dec_z[|kz|] / (4 pi), with dec_q
// the per-axis deconvolution factors 1 / u^(l_q / N_q)^2 of the window (FP64
// tables of n_q/2 + 1 entries each); the z pass multiplies by mu_l = h(l) F.
template <typename T>
hipError_t launch_mu(T *mu, const double *C0, const double *C1, const double *C2,
                     const double *omega, int32_t S, const int32_t n[3], const double *dec0,
                     const double *dec1, const double *dec2, hipStream_t s);

}  // namespace slp
