// rp_internal.h -- private interface between the HIP kernels (rp_kernels.hip)
// and the C-ABI drivers (rp_api.hip) of librp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpk {

constexpr int BS = 256;      // threads per block of every row kernel
constexpr int PAD = 64;      // reduced rows of an instance are padded to a multiple of this

// Per-instance iteration status kept on the device.
enum : int32_t {
  ST_RUN = 0,
  ST_CONVERGED = 1,
  ST_MAXITER = 2,
  ST_BREAKDOWN = 3,
  ST_NONFINITE = 4,
  ST_SKIP = 5,     // not part of this solve (empty instance or already finished)
  ST_STALLED = 6,  // paper's rule: the stopping measure stopped falling above the tolerance
};

// Work decomposition of the padded reduced rows: one block per chunk; a
// chunk never straddles two instances, so every block's partial reduction
// belongs to exactly one instance (chunk c's partial lives at slot c).
struct Chunks {
  const int32_t* row0;     // [nchunk] first reduced row of the chunk
  const int32_t* nrows;    // [nchunk] rows in the chunk (multiple of PAD)
  const int32_t* inst;     // [nchunk] owning instance
  const int32_t* inst_c0;  // [K+1]   chunks of instance k: [inst_c0[k], inst_c0[k+1])
  int32_t nchunk;
  int32_t K;
};

// Tiles for the LDS-staged kernels: a tile is a row range of one instance
// with an x window [w0, w0 + nw) copied into LDS.  The window kind is the same
// for every tile of an instance:
//   WIN_WHOLE  the instance's whole padded row block: every read is in LDS;
//   WIN_BAND   a band around the tile's rows; reads outside go to global memory;
//   WIN_NONE   no window (nw = 0): every read goes to global memory.
enum : int32_t { WIN_WHOLE = 0, WIN_BAND = 1, WIN_NONE = 2 };
struct Tiles {
  const int32_t* row0;     // [ntile]
  const int32_t* nrows;    // [ntile]
  const int32_t* inst;     // [ntile]
  const int32_t* inst_t0;  // [K+1] tiles of instance k: [inst_t0[k], inst_t0[k+1])
  const int32_t* w0;       // [ntile]
  const int32_t* nw;       // [ntile]
  const int32_t* kind;     // [ntile] WIN_*
  int32_t ntile;
  int32_t K;
  int32_t maxw;            // largest window (rows)
  const int32_t* order;    // [ntile] tile taken by block b of a launch of ntile blocks (null: the
                           //         contiguous per-XCD ranges of xcd_tile)
  const int64_t* sbase;    // replayed graphs: sweep numbers passed to the Jacobi sweep and check
                           //         kernels count from *sbase (null: they are absolute)
};
constexpr size_t TILE_LDS_BYTES = 163840 - 512;  // dynamic LDS available to a tile block

// Sparse matrix M = diag(d) - A_off over the padded reduced rows.
template <typename T>
struct MatView {
  const int32_t* rp;   // [npad+1]
  const int32_t* col;  // [z]
  const T* val;        // [z] off-diagonal entries of A (probabilities, positive)
  const T* d;          // [npad] diagonal of I - A (1 on padding rows)
  const uint16_t* c16; // [z] col minus the first row of the row's instance block (blocks of at
                       //     most 65,536 rows; read by tiles whose window is the whole block)
};

// Sliced rows of one tile set and one matrix: the rows of each tile sorted
// by decreasing entry count (ties in row order) and cut into slices of SLICE
// rows, one row per lane.  Entry j of lane l of slice s is at off[s] + SLICE*j
// + l; rows shorter than the slice's width are padded with value 0 and
// column 0.  Columns are relative to the tile's window start w0 (16-bit on
// tiles whose window is the whole instance block, 32-bit on the others).
constexpr int SLICE = 64;
template <typename T>
struct Sliced {
  const int32_t* t_s0;   // [ntile+1] slices of tile t: [t_s0[t], t_s0[t+1])
  const int32_t* off;    // [nslice]  first slot of the slice
  const int32_t* width;  // [nslice]  entries per lane (longest row of the slice)
  const int32_t* row;    // [nslice*SLICE] row of each lane, -1 past the tile's last row
  const T* d;            // [nslice*SLICE] diagonal of that row (1 where no row)
  const T* val;          // [nslot]
  const uint16_t* c16;   // [nslot] column - w0 (tiles with whole-block windows)
  const int32_t* c32;    // [nslot] column - w0 (other tiles)
  int32_t stream;        // 1: read val/columns with nontemporal loads (slices larger than the
                         //    last-level cache, so keeping them there only evicts the vectors)
  // Column panels.  A tile of an instance whose block is too large for one
  // LDS window and whose columns have no band (uniformly spread targets) can
  // be "paneled": the instance block's columns are cut into panels of pw
  // rows, staged into LDS one after the other, and every lane keeps the sums
  // of its rows in registers across the panels.  Per slice, the entries are
  // stored panel after panel, and within a panel lane after lane (each
  // lane's entries of that panel contiguous, in column order); cnt holds,
  // per slice, panel and lane, how many entries the lane has in the panel,
  // so a lane finds its entries from a prefix sum over the lanes.  Columns
  // are relative to the panel start (16-bit, c16).  A row's entries keep
  // their column order, so row sums are bit-identical to the slices'.
  const int32_t* npan;   // [ntile] panels of the tile's instance block (0: not paneled)
  const int32_t* hoff;   // [ntile] first count byte of the tile: slice s, panel p, lane l at
                         //         hoff[t] + ((s - t_s0[t]) * npan[t] + p) * SLICE + l
  const uint8_t* cnt;    // count bytes of all paneled tiles
  const int32_t* pent;   // [nslice] first entry of a paneled slice in val / c16
  const int32_t* pend;   // [ntile] end (exclusive) of the instance block of a paneled tile
  int32_t pw;            // panel width (rows, a multiple of PAD)
  int32_t paneled;       // 1 when some tile is paneled
};
// Most slices a wavefront of a paneled tile keeps sums for (rows of a paneled
// tile <= PanelShape<T>::MAXS * 1024): a quarter of the 128 registers a lane
// has at 16 wavefronts per CU for FP64 sums, and as many slices in FP32,
// whose per-slice entry offsets (scalar registers) are the limit there.
// Spare entries after the last one of a sliced set with panels (value 0,
// column 0): the paneled sweep loads entry pos + j of every lane for
// j below the wavefront's largest count (at most 255), whether or not the
// lane has that many.
constexpr int PANEL_SLACK = 256;
template <typename T>
struct PanelShape {
  static constexpr int MAXS = 16;
};

// Stopping measure of the inner iterations.
enum : int32_t {
  MEAS_DELTA = 0,     // Jacobi: max |x' - x|
  MEAS_WDELTA = 1,    // Jacobi: max d_i |x'_i - x_i|  (= residual of x)
  MEAS_S = 2,         // BiCGStab: max |s_i|
  MEAS_R = 3,         // BiCGStab: max |r_i| (recurrence residual)
};

// Per-instance device state of the tiled BiCGStab launches.
struct BicgState {
  int32_t* status;
  int64_t* iters;
  double* meas;
  const double* thr;
  double* rho;     // [2][K] by step parity
  double* alpha;   // [K]
  double* omega;   // [K]
  int32_t* ndone;
  int measmode;
  int64_t max_iter;
};

// ---- precomputation ----------------------------------------------------------
// matrix = 0: a Markov chain (entries in [0,1], rows sum to 1 within tol);
// matrix = 1: a general matrix (finite entries, nonzero diagonal stored)
hipError_t launch_validate(hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp,
                           const int32_t* col, const double* val, const int64_t* inst_off,
                           int32_t K, double tol, int matrix, unsigned long long* bad_key);
hipError_t launch_identity_minus(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                                 double* out);
hipError_t launch_inv_gap(hipStream_t st, int64_t npad, const int32_t* row_state, const int32_t* arp,
                          const double* aval, const double* d, double* out);
hipError_t launch_seed_goal(hipStream_t st, int64_t n, const uint8_t* goal, uint32_t* mark);
hipError_t launch_seed_complement(hipStream_t st, int64_t n, const uint32_t* src, uint32_t* mark);
// one pull step, numbered `step` from 1 within a search; *changed (zero
// before the first step) receives the number of the last step that marked
hipError_t launch_reach_step(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                             const double* val, const uint8_t* blocked, uint32_t* mark,
                             int32_t* changed, int32_t step);
hipError_t launch_classes(hipStream_t st, int64_t n, const uint32_t* reach_goal,
                          const uint32_t* reach_s0, const uint8_t* goal, int prob0_only,
                          uint8_t* cls, uint8_t* class_out, int32_t* flags_sq);
// whole search in one workgroup for chains of at most REACH_RESIDENT_MAX states
hipError_t launch_reach_resident(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                                 const double* val, const uint8_t* blocked, uint32_t* mark);
constexpr int64_t REACH_RESIDENT_MAX = 32768;
// deep searches: merge states of equal reachability (parent, cmark: n each;
// mark: the marks so far), then pull steps on the classes, then expand
hipError_t launch_reach_contract(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                                 const uint8_t* blocked, const uint32_t* mark, int32_t* parent, uint32_t* cmark);
hipError_t launch_reach_step_classes(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                                     const double* val, const uint8_t* blocked, const int32_t* root, uint32_t* cmark,
                                     int32_t* changed, int32_t step);
hipError_t launch_classes_expand(hipStream_t st, int64_t n, const uint8_t* blocked, const int32_t* root,
                                 const uint32_t* cmark, uint32_t* mark);
size_t scan_scratch_elems(int64_t n);
hipError_t launch_scan(hipStream_t st, const int32_t* in, int32_t* out, int64_t n,
                       int32_t* scratch);
hipError_t launch_inst_counts(hipStream_t st, int32_t K, const int64_t* inst_off,
                              const int32_t* rank, int32_t* counts);
hipError_t launch_map(hipStream_t st, int64_t n, const uint8_t* cls, const int32_t* rank,
                      const int64_t* inst_off, int32_t K, const int64_t* roff, int32_t* map,
                      int32_t* row_state, int32_t* row_inst_unused);
hipError_t launch_row_count(hipStream_t st, int64_t npad, const int32_t* row_state,
                            const int32_t* rp, const int32_t* col, const double* val,
                            const uint8_t* cls, int32_t* cnt, double* d64, float* d32,
                            double* b64, int any_sign);
hipError_t launch_fill_rows(hipStream_t st, int64_t npad, const int32_t* row_state,
                            const int32_t* rp, const int32_t* col, const double* val,
                            const uint8_t* cls, const int32_t* map, const int32_t* arp,
                            int32_t* acol, double* av64, float* av32, int any_sign);
// (any_sign: keep every nonzero off-diagonal entry, not only P > 0: the
// general systems of rp_matrix_system)
// Transpose of the reduced matrix (npad rows, z entries): trp (npad + 1),
// tcol / tv64 / tv32 (z).  Work arrays erow, idx, key_out, perm (z each) and
// temp (transpose_temp_bytes) belong to the caller.
hipError_t transpose_temp_bytes(int64_t npad, int64_t z, size_t* bytes);
hipError_t launch_transpose(hipStream_t st, int64_t npad, int64_t z, const int32_t* arp, const int32_t* acol,
                            const double* av64, int32_t* trp, int32_t* tcol, double* tv64, float* tv32,
                            int32_t* erow, int32_t* idx, int32_t* key_out, int32_t* perm, void* temp,
                            size_t temp_bytes);

// ---- solver kernels ----------------------------------------------------------
template <typename T>
hipError_t launch_jacobi(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, T* xn,
                         Chunks ch, const int32_t* status, double* partial, int weighted);
template <typename T>
hipError_t launch_jacobi_inplace(hipStream_t st, int L, MatView<T> m, const T* rhs, T* x, Chunks ch,
                                 const int32_t* status, double* partial, int weighted);
hipError_t launch_fill_erow(hipStream_t st, int64_t n, const int32_t* rp, int32_t* erow);
template <typename T>
hipError_t launch_jacobi_segscan(hipStream_t st, MatView<T> m, const int32_t* erow, const T* rhs, const T* x, T* xn,
                                 Chunks ch, const int32_t* status, double* partial, int weighted);
hipError_t launch_fin_jacobi(hipStream_t st, Chunks ch, const double* partial, int32_t* status,
                             int64_t* iters, double* meas, const double* thr, int strict,
                             int64_t max_iter, int32_t* ndone);
template <typename T>
hipError_t launch_jacobi_tile(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, T* xn,
                              Tiles tl, int64_t s, const double* pprev, double* pcur,
                              int32_t* status, int64_t* iters, double* meas, const double* thr,
                              int strict, int64_t max_iter, int32_t* ndone, int weighted);
template <typename T>
hipError_t launch_jacobi_resident(hipStream_t st, int L, MatView<T> m, const T* rhs, T* xa, T* xb, Tiles tl,
                                  int64_t s0, int nsweeps, int32_t* status, int64_t* iters, double* meas,
                                  const double* thr, int strict, int64_t max_iter, int32_t* ndone, int weighted);
// resident sweeps on the sliced rows of whole-window tiles: tile c of tl is an
// instance block whose slices are [s_lo[c], s_hi[c]) of sl
template <typename T>
hipError_t launch_jacobi_resident_sliced(hipStream_t st, Sliced<T> sl, const T* rhs, T* xa, T* xb, Tiles tl,
                                         const int32_t* s_lo, const int32_t* s_hi, int64_t s0, int nsweeps,
                                         int32_t* status, int64_t* iters, double* meas, const double* thr,
                                         int strict, int64_t max_iter, int32_t* ndone, int weighted);
// The resident BiCGStab keeps up to BICG_RESIDENT_SLOTS rows per lane group
// (of L lanes, 1024 threads per block) in registers.
constexpr int BICG_RESIDENT_SLOTS = 2;
inline int64_t bicg_resident_rows(int L) { return (int64_t)BICG_RESIDENT_SLOTS * (1024 / L); }
template <typename T>
hipError_t launch_bicg_resident(hipStream_t st, int L, MatView<T> m, const T* rhs, T* x, T* r, T* q, T* p, T* v,
                                Tiles tl, int64_t s0, int nsteps, int x_is_zero, double* pc, double* ps,
                                BicgState b);
hipError_t launch_jacobi_check(hipStream_t st, Tiles tl, int64_t s, const double* pprev,
                               int32_t* status, int64_t* iters, double* meas, const double* thr,
                               int strict, int64_t max_iter, int32_t* ndone);

template <typename T>
hipError_t launch_bicg_init(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x,
                            int x_is_zero, T* r, T* q, T* p, T* v, Chunks ch,
                            const int32_t* status, double* partial2);
hipError_t launch_fin_bicg_init(hipStream_t st, Chunks ch, const double* partial2,
                                int32_t* status, double* rho, double* alpha, double* omega,
                                double* beta, double* meas, const double* thr, int measmode,
                                int32_t* ndone);
template <typename T>
hipError_t launch_bicg_p(hipStream_t st, const T* r, T* p, const T* v, const double* beta,
                         const double* omega, Chunks ch, const int32_t* status);
template <typename T>
hipError_t launch_spmv_dot(hipStream_t st, int L, int mode, MatView<T> m, const T* u, T* y,
                           const T* q, Chunks ch, const int32_t* status, double* partial);
hipError_t launch_fin_alpha(hipStream_t st, Chunks ch, const double* partial, int32_t* status,
                            const double* rho, double* alpha, int32_t* ndone);
template <typename T>
hipError_t launch_bicg_s(hipStream_t st, const T* r, const T* v, T* s, const double* alpha,
                         Chunks ch, const int32_t* status, double* partial);
hipError_t launch_fin_omega(hipStream_t st, Chunks ch, const double* partial2,
                            int32_t* status, double* omega, int32_t* ndone);
template <typename T>
hipError_t launch_bicg_xr(hipStream_t st, T* x, const T* p, const T* s, T* r, const T* t,
                          const T* q, const double* alpha, const double* omega, Chunks ch,
                          const int32_t* status, double* partial2);
hipError_t launch_fin_rho(hipStream_t st, Chunks ch, const double* partial_xr,
                          const double* partial_s, int32_t* status, double* rho,
                          const double* alpha, const double* omega, double* beta,
                          int64_t* iters, double* meas, const double* thr, int measmode,
                          int64_t max_iter, int32_t* ndone);

template <typename T>
hipError_t launch_bicg_tile_init(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, int x_is_zero,
                                 T* r, T* q, T* p, T* v, Tiles tl, const int32_t* status, double* pc);
template <typename T>
hipError_t launch_spmv_tile(hipStream_t st, int L, int mode, MatView<T> m, const T* u, T* y, const T* q,
                            Tiles tl, const int32_t* status, double* part);
template <typename T>
hipError_t launch_bicg_p_tile(hipStream_t st, const T* r, T* p, const T* v, Tiles tl, int64_t j,
                              const double* pc, const double* ps, BicgState b);
template <typename T>
hipError_t launch_bicg_s_tile(hipStream_t st, const T* r, const T* v, T* s, Tiles tl, int64_t j,
                              const double* pa, double* ps, BicgState b);
template <typename T>
hipError_t launch_bicg_xr_tile(hipStream_t st, T* x, const T* p, const T* s, T* r, const T* t, const T* q,
                               Tiles tl, int64_t j, const double* pb, double* pc, BicgState b);
hipError_t launch_bicg_check(hipStream_t st, Tiles tl, int64_t j, const double* pc, const double* ps,
                             BicgState b);
// sliced rows: build (order + widths per tile, then the slices) and sweeps
hipError_t launch_slice_order(hipStream_t st, const int32_t* rp, Tiles tl, const int32_t* t_s0, int32_t window,
                              int32_t* row, int32_t* width);
template <typename T>
hipError_t launch_slice_fill(hipStream_t st, MatView<T> m, Tiles tl, const int32_t* stile, int32_t nslice,
                             const int32_t* off, const int32_t* width, const int32_t* row, T* d, T* val,
                             uint16_t* c16, int32_t* c32);
// column panels: per paneled slice (pslice: slice index, ptile: its tile)
// the count bytes (sl.cnt) and its number of entries; then the entries
template <typename T>
hipError_t launch_panel_count(hipStream_t st, MatView<T> m, Tiles tl, Sliced<T> sl, const int32_t* pslice,
                              const int32_t* ptile, int32_t npslice, uint8_t* cnt, int32_t* entries);
template <typename T>
hipError_t launch_panel_fill(hipStream_t st, MatView<T> m, Tiles tl, Sliced<T> sl, const int32_t* pslice,
                             const int32_t* ptile, int32_t npslice, T* val, uint16_t* c16);
template <typename T>
hipError_t launch_jacobi_sliced(hipStream_t st, Sliced<T> sl, const T* rhs, const T* x, T* xn, Tiles tl, int64_t s,
                                const double* pprev, double* pcur, int32_t* status, int64_t* iters, double* meas,
                                const double* thr, int strict, int64_t max_iter, int32_t* ndone, int weighted);
// mode 0: y = M u, partial q.y (qv = q); mode 1: partials (y.u, y.y); mode 2:
// y = qv - M u (the FP64 refinement residual, qv = b), partial max |y|
template <typename T>
hipError_t launch_spmv_sliced(hipStream_t st, int mode, Sliced<T> sl, const T* u, T* y, const T* qv, Tiles tl,
                              const int32_t* status, double* part);
hipError_t launch_residual_tile(hipStream_t st, int L, MatView<double> m, const double* b, const double* x,
                                double* r, Tiles tl, const int32_t* status, double* part);

// ---- refinement and bookkeeping ------------------------------------------------
hipError_t launch_residual64(hipStream_t st, int L, MatView<double> m, const double* b,
                             const double* x, double* r, Chunks ch, const int32_t* status,
                             double* partial);
hipError_t launch_fin_outer(hipStream_t st, Chunks ch, const double* partial, int32_t* status,
                            int64_t* outer_it, double* rn, double* scale, const double* tb,
                            double tol, int certified, int32_t max_refine, double* thr_in,
                            double inner_tol, double floor_rel, double margin, double* rbest, int32_t* stall,
                            const int64_t* tot_it, int64_t max_iter, int32_t* ndone);
// graph replays: publish *src with the next sequence number kept on the
// device (*seq incremented), and advance the sweep base by n
hipError_t launch_publish_next(hipStream_t st, const int32_t* src, int32_t* dst, int32_t* seq);
hipError_t launch_advance(hipStream_t st, int64_t* base, int64_t n);
hipError_t launch_set_i64(hipStream_t st, int64_t* p, int64_t v);
hipError_t launch_set_i32(hipStream_t st, int32_t* p, int32_t v);
hipError_t launch_stall(hipStream_t st, int32_t K, int64_t launched, int32_t* status, int64_t* iters,
                        const double* meas, double* best, int64_t* best_it, int64_t min_window, int32_t* ndone);
hipError_t launch_accum_inner(hipStream_t st, int32_t K, const int32_t* status_out, const int64_t* iters_in,
                              const double* meas_in, int64_t* tot_it, double* last_meas);
template <typename T>
hipError_t launch_scale_rhs(hipStream_t st, const double* r64, const double* scale, T* rhs,
                            Chunks ch, const int32_t* status);
template <typename T>
hipError_t launch_correct(hipStream_t st, double* x64, const T* xa, const T* xb,
                          const int64_t* parity_iters, int prev, const int32_t* status_in,
                          const double* scale, Chunks ch, const int32_t* status_out);
hipError_t launch_inner_init(hipStream_t st, int32_t K, const int32_t* status_out,
                             const int64_t* nq, int32_t* status_in, int64_t* iters_in,
                             int32_t* ndone);
template <typename T>
hipError_t launch_gather_full(hipStream_t st, int64_t npad, const int32_t* row_state,
                              const double* full, T* out);
hipError_t launch_scatter_full(hipStream_t st, int64_t n, const uint8_t* cls, const int32_t* map,
                               const int64_t* inst_off, int32_t K, const double* xa,
                               const double* xb, const int64_t* parity_iters, double s1_value,
                               double* out);
hipError_t launch_copy_sel(hipStream_t st, Chunks ch, const double* xa, const double* xb,
                           const int64_t* parity_iters, double* out);
hipError_t launch_absmax(hipStream_t st, const double* x, Chunks ch, double* partial);
hipError_t launch_fin_absmax(hipStream_t st, Chunks ch, const double* partial, double* out);
hipError_t launch_gradient(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                           const uint8_t* cls, const int32_t* map, const double* lam,
                           const double* xfull, double* g);
hipError_t launch_fill_f64(hipStream_t st, double* p, int64_t n, double v);
hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_publish(hipStream_t st, const int32_t* src, int32_t* dst, int32_t seq);
hipError_t launch_col16(hipStream_t st, Chunks ch, const int64_t* roff, const int32_t* rp, const int32_t* col,
                        uint16_t* c16);
hipError_t launch_band_hist(hipStream_t st, Chunks ch, const int32_t* arp, const int32_t* acol, int32_t* hist);
hipError_t launch_gather_at(hipStream_t st, const int32_t* src, const int64_t* idx, int32_t count, int32_t* out);

// strongly connected components of S_? and their level-by-level solve
hipError_t launch_scc_trim(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                           int32_t* comp, int dir, int32_t* changed);
hipError_t launch_scc_color_init(hipStream_t st, int64_t n, const int32_t* comp, int32_t* color, int32_t* mark);
hipError_t launch_scc_color(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                            const int32_t* comp, int32_t* color, int dir, int32_t* changed);
hipError_t launch_scc_root(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* color, int32_t* mark);
hipError_t launch_scc_mark(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                           const int32_t* comp, const int32_t* color, int32_t* mark, int dir, int32_t* changed);
hipError_t launch_scc_assign(hipStream_t st, int64_t n, int32_t* comp, const int32_t* color, const int32_t* mark,
                             int32_t* left);
hipError_t launch_scc_stats(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* row_state,
                            int32_t* minrow, int32_t* size, int32_t* cnt);
hipError_t launch_scc_level(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                            const int32_t* comp, int32_t* lvl, int dir, int32_t* changed);
hipError_t launch_scc_rowlevel(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* lvl,
                               const int32_t* size, int32_t* key, int32_t* rowid, int32_t* maxlvl,
                               int32_t* cyclic_rows);
hipError_t launch_scc_levelcount(hipStream_t st, int64_t n, const int32_t* key, int32_t* count);
hipError_t launch_scc_out(hipStream_t st, int64_t nfull, const int32_t* map, const int32_t* comp,
                          const int32_t* minrow, const int32_t* lvl, const int32_t* row_state, int32_t* label,
                          int32_t* level);
hipError_t launch_scc_rows(hipStream_t st, const int32_t* rows, int32_t nr, MatView<double> m, const double* b,
                           double* x, unsigned long long* dmax);
hipError_t launch_sort_by_key(hipStream_t st, int32_t* key, int32_t* val, int32_t* key_tmp, int32_t* val_tmp,
                              int64_t n, int end_bit, void* temp, size_t* temp_bytes);

}  // namespace rpk
