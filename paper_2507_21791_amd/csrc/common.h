// Internal declarations shared by the gfx950 kernels and the host driver.
//
// Data layout in HBM
//   X, Q      column-major, block column k = columns [k*s, (k+1)*s).
//   Q slot k  also holds the intermediate blocks of block column k before Q_k
//             exists (U_k, V_k, W_k of section 2): every kernel that turns one
//             into the next reads a row and writes the same row, so the
//             update happens in place and no m-row scratch is needed.
//   workspace small s x s / (n x s) coefficient matrices, the per-workgroup
//             partial Gram matrices of the current reduction, and the TSQR
//             tree (leaf R factors, node Q factors, downward coefficients).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "bcgs.h"

namespace bcgs {

constexpr int kMaxS = 64;          // largest block width
constexpr int kThreads = 256;      // threads per workgroup of every kernel
constexpr int kWaves = kThreads / 64;

// Global-memory access through an explicit global-address-space pointer.
// Kernels see their pointer arguments as global already; a device function
// that receives its pointers from memory (a step record of the persistent
// batch) would otherwise use flat instructions, which the hardware counts
// together with LDS operations, so every LDS wait would also wait for the
// global loads in flight.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline int64_t round_up64(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- pass ---
// One streaming pass over the rows of the tall matrices: the only kind of
// kernel that touches m-row data besides TSQR.  A workgroup owns a
// contiguous range of rows and walks it in tiles of TR rows.  For each tile
// it stages a window of columns in LDS (Q columns [0, nq), then an optional
// block F, then an optional block E), optionally rewrites two blocks in
// place through the block update of Alg. 1 / Alg. 2,
//     B <- (B - Q_{1:j} C) T^{-1}      (T upper triangular, optional),
// writes them back, and accumulates A^T B Gram products of LDS columns in
// registers; at the end each workgroup writes its partial Gram matrix.
template <typename T>
struct PassArgs {
  int64_t m;
  int s;          // block width
  int sp;         // s rounded up to 16 (MFMA tile width)
  int tr;         // rows per tile: 16, 32 or 64
  int64_t rows_per_wg;
  int ncols;      // staged columns = nq + fcols + ecols
  int ncols_p;    // ncols rounded up to 16 (extra columns are zero)
  // sources of the staged columns
  const T* q; int64_t ldq; int nq;
  const T* f; int64_t ldf; int fcols;
  const T* e; int64_t lde; int ecols;
  // update 1: columns [u1_c0, u1_c0 + s) <- cols[0, u1_c0 + s) F1
  int upd1; int u1_c0;
  const double* c1; T* dst1; int64_t ldd1;
  // update 2: columns [u2_c0, u2_c0 + s) <- cols[0, u2_c0 + s) F2
  int upd2; int u2_c0;
  const double* c2; T* dst2; int64_t ldd2;
  // Gram: A = cols [0, ga), B = cols [gb0, gb0 + gbn)
  int gram; int ga_p; int gb0; int gbn_p;
  int a_blocks_per_group;  // 16-column A blocks handled by one y-group
  int skip_a0;             // skip tiles with a >= skip_a0 and b < skip_b1
  int skip_b1;
  int groups;              // H: workgroups per row range (Gram split)
  double* partial;         // [G][gbn_p][ga_p]
};

// Block updates as one product.  The update B <- (B - Q_{1:j} C) T^{-1} of
// Alg. 1 / Alg. 2 is evaluated as [Q_{1:j} B] F with the (K + s) x s
// coefficient matrix F = [-C T^{-1}; T^{-1}] (F = [-C; I] for the updates
// without a triangular factor), built once per block column by the
// epilogue.  Coefficient and triangular matrices are stored row-major with
// row stride `sp` and zero padding: C (K x s) at C[k * sp + j].

// ---------------------------------------------------------------- TSQR ---
struct TsqrPlan {
  int s;
  bool wave;       // one wave per chunk (s <= 16) instead of one workgroup
  int cr;          // rows per leaf chunk
  int fan;         // children per tree node (fan * s <= cr)
  int64_t nchunks;
  int levels;      // upward tree levels (>= 1)
  int64_t nodes[24];         // nodes[0] = nchunks, nodes[levels] = 1
  int64_t r_off[24];         // offset (doubles) of level-l R factors
  int64_t q_off[24];         // offset of level-l node Q factors (l >= 1)
  int64_t c_off[24];         // offset of level-l downward coefficients
  int64_t cnt_off;           // offset of the node arrival counters (ints,
                             // one per node of levels 1..levels)
  int64_t cnt_doubles;       // their size in doubles
  int64_t total;             // doubles
};

TsqrPlan make_tsqr_plan(int64_t m, int s);

// ------------------------------------------------------- workspace plan ---
// Launch choices that the autotuner may set per problem class.  They change
// the row split (and so the order of the cross-workgroup sums) and the tile
// shape, never the method: results stay within the stated tolerances and
// are bitwise repeatable for a fixed choice.
struct Tuning {
  int max_wg = 512;   // upper bound on the workgroups of a streaming pass
  int shape = -1;     // pass16 tile shape index, -1 = automatic
};

struct Plan {
  int64_t m, n;
  int s, sp, q;
  int variant, precision;
  int G;                  // workgroups (row ranges) of the streaming passes
  int64_t rows_per_wg;
  int tr_max;             // largest tile the widest pass can afford
  Tuning tune;
  TsqrPlan tsqr;
  // workspace offsets in bytes
  size_t off_c1, off_c2, off_t1, off_t2, off_f1, off_f2, off_gram,
      off_partial, off_tsqr;
  size_t off_fsplit;      // s = 32, 64: two (n + s) x 16 column blocks of a
                          // coefficient matrix (block updates on the s <= 16
                          // pass)
  size_t off_scratch_info;
  size_t bytes;
  int64_t gram_ld;        // leading dimension of the reduced Gram matrix
  int64_t partial_elems;  // per workgroup
};

bool make_plan(int64_t m, int64_t n, int64_t s, int variant, int precision,
               Plan* p, const Tuning* t = nullptr);

// Process-wide table of tuned choices, keyed by problem class (see tune.hip);
// every entry point consults it, so a problem run alone, batched or served
// takes the same choices and gives the same bits.
bool tuned_choice(int64_t m, int64_t n, int s, int variant, int precision,
                  Tuning* out);

// Argument checks shared by every entry point (BCGS_ERR_ARG before anything
// is enqueued); fills the plan with the tuned choices of the problem class.
bcgs_status check_problem(const void* X, int64_t ldx, int64_t m, int64_t n,
                          int64_t s, int variant, int precision,
                          const void* Q, int64_t ldq, const double* R,
                          int64_t ldr, const bcgs_info* d_info, Plan* p);
// Frees the batch arenas, cached graphs and library streams (batch.hip).
void batch_release();
// The batch as one persistent launch (batch_persist.hip); *used = false
// when some problem needs a kernel the persistent launch does not run.
bcgs_status persist_run(const std::vector<Plan>& plans,
                        const bcgs_problem* probs,
                        const std::vector<size_t>& offs, void* arena,
                        const std::vector<char>& key, hipStream_t stream,
                        bool* used);
void persist_release();

// Enqueue the whole factorization on `st` (workspace of p.bytes bytes).
bcgs_status run_problem(const Plan& p, const void* X, int64_t ldx, void* Q,
                        int64_t ldq, double* R, int64_t ldr, void* ws,
                        bcgs_info* info, hipStream_t st);

// Launchers (return hipError_t of the launch).
// *tag receives the kernel instantiation (see bcgs_launch_record).
template <typename T>
hipError_t launch_pass(const PassArgs<T>& a, int G, hipStream_t st, int* tag);
// syncs: device counter of completed synchronization points (the info
// record's field), incremented once by each reduction; may be null
hipError_t launch_gram_reduce(const double* partial, int G, int64_t elems,
                              double* out, int32_t* syncs, hipStream_t st);
// Fast path for s <= 16 (pass16.hip); hipErrorNotSupported when it does not
// apply (nothing launched).
hipError_t launch_pass16(const PassArgs<double>& a, int64_t m,
                         const Tuning& tune, hipStream_t st, int* tag,
                         int* G_out);
int pass16_shape_count();
// shape `shape` has four waves per workgroup (the batched persistent
// kernel runs those); problems of at most pass16_small_rows() rows choose
// only such shapes
bool pass16_shape_four_waves(int shape);
int64_t pass16_small_rows();
// The same pass on binary32 storage (FP32-bulk form).
hipError_t launch_pass16_f32(const PassArgs<float>& a, int64_t m,
                             const Tuning& tune, hipStream_t st, int* tag,
                             int* G_out);
size_t pass16_lds_bytes(int ncols_p, int tr, int nw);

struct EpiArgs;
hipError_t launch_epilogue(const EpiArgs& a, hipStream_t st);

// TSQR of the m x s block v (leading dimension ldv) into dst (may equal v);
// the s x s factor R (positive diagonal) goes to r_out(i, j) =
// r_out[i * r_rs + j * r_cs] (full square, zeros below the diagonal).
// The root of the reduction tree increments *syncs once (may be null).
template <typename T>
hipError_t launch_tsqr(const TsqrPlan& tp, const T* v, int64_t ldv, T* dst,
                       int64_t ldd, int64_t m, double* ws, double* r_out,
                       int64_t r_rs, int64_t r_cs, int32_t* syncs,
                       hipStream_t st);

hipError_t launch_fill(double* p, int64_t rows, int64_t cols, int64_t ld,
                       double value, hipStream_t st);
// Columns [c0, c0 + 16) and [c0 + 16, c0 + 32) of the K x sp row-major
// matrix F (c0 + 32 <= sp) as two K x 16 row-major matrices fa and fb.
hipError_t launch_split_coef(const double* F, int64_t K, int sp, int c0,
                             double* fa, double* fb, hipStream_t st);

// --------------------------------------------------------- epilogues ---
enum EpiMode : int {
  EPI_S_ONLY = 0,     // C2 <- gram(0:js, 0:s)                      (S)
  EPI_Y_ONLY = 1,     // C1 <- gram(0:js, 0:s)                      (Y)
  EPI_S_CHOL = 2,     // [S; T] of block j: C2 <- S, T2 <- chol(T - S^T S)
  EPI_ONE_SYNC = 3,   // after [Q U]^T [U E]: Y_kk, R block column, eq. (1)
  EPI_R_ASSEMBLE = 4, // BCGSI+: R block column from C2, C1, T2, T1
};

// coefficient matrices the epilogue leaves for the next streaming pass
enum CoefMode : int {
  COEF_NONE = 0,
  COEF_SCALED = 1,     // F = [-C T^{-1}; T^{-1}]
  COEF_UNSCALED = 2,   // F = [-C; I]
};

struct EpiArgs {
  int mode;
  int s, sp;
  int j;              // block column index being completed (0-based)
  int has_e;          // the Gram included E = X_{j+1}
  int chol_s;         // form T2 <- chol(T - S^T S) (P-1S) after eq. (1)
  const double* gram; int64_t gld;
  double* c1; double* c2; double* t1; double* t2;
  double* f1; double* f2;
  int f1_mode, f1_rows;   // F1 from (C1, T1), C1 having f1_rows rows
  int f2_mode, f2_rows;   // F2 from (C2, T2)
  int fold12;             // the next pass runs both updates on the staged
                          // columns: fold F1 into F2's rows [0, f1_rows + s)
  int unit_s;             // BCGSI+1s: S_{j+1,j+1} = I (T2 <- I)
  double* r; int64_t ldr;
  bcgs_info* info;
};

// Recording of a schedule for the batched persistent kernel
// (batch_persist.hip): while the calling thread records, every launcher
// describes its launch as a step of work items instead of launching it
// (and returns hipSuccess); a launch the persistent kernel cannot run marks
// the recording unsupported.
bool rec_active();
void rec_unsupported();
void rec_reduce(const double* partial, int G, int64_t elems, double* out,
                int32_t* syncs, int64_t blocks);
void rec_fill(double* p, int64_t rows, int64_t cols, int64_t ld, double v,
              int64_t blocks);
void rec_init(bcgs_info* info);
void rec_epi(const EpiArgs& a);
void rec_tsqr_leaf(int S, const double* v, int64_t ldv, int64_t m,
                   int64_t nchunks, double* rleaf, int64_t blocks);
void rec_tsqr_node(int S, const double* rprev, int64_t nprev, int fan,
                   int64_t nnodes, double* rcur, double* qcur, int is_root,
                   double* r_out, int64_t r_rs, int64_t r_cs, int32_t* syncs,
                   int64_t blocks);
void rec_tsqr_down(const double* qpar, const double* cpar, int64_t nchild,
                   int fan, int s, double* cchild, int parent_is_root);
void rec_tsqr_apply(int S, const double* v, int64_t ldv, int64_t m,
                    int64_t nchunks, const double* cleaf, double* dst,
                    int64_t ldd, int64_t blocks);

// launch profiling (profile.hip); no-ops unless bcgs_profile_start ran on
// the stream being attached
void prof_attach(hipStream_t st);
void prof_detach();
void prof_begin(int kind, int tag, double bytes, double flops);
void prof_end();
// replaces the byte and flop model of the launch being recorded
void prof_model(double bytes, double flops);
// Names the launch being recorded (printf-style; a no-op unless profiling
// is active) in the short form profiler summaries print: the kernel's name
// and template arguments, without namespaces or parameter list.
void prof_name(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
template <typename T>
constexpr const char* type_name() { return sizeof(T) == 8 ? "double" : "float"; }
constexpr const char* bool_name(bool b) { return b ? "true" : "false"; }

}  // namespace bcgs
