// Internal declarations of the MI355X H-matrix library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hh.h"

#define HH_WAVE 64

// ------------------------------------------------------------------ errors

struct hh_error {
  hh_status st;
  std::string msg;
};

#define HIP_OK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw hh_error{HH_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HH_REQUIRE(cond, status, text)                 \
  do {                                                 \
    if (!(cond)) throw hh_error{status, std::string(text)}; \
  } while (0)

// ------------------------------------------------------------- device memory

// A stream-ordered device buffer (hipMallocAsync / hipFreeAsync on the
// context stream). Freed on the stream in the destructor.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();
  void alloc(hipStream_t stream, size_t nbytes);
  // keeps the buffer when it already holds nbytes (no allocation, so a
  // repeated call can be captured in a graph)
  void ensure(hipStream_t stream, size_t nbytes) {
    if (!p || bytes < nbytes) alloc(stream, nbytes);
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct PhaseRec {
  int phase;
  hipEvent_t a, b;
};

struct hh_ctx_s {
  int device = 0;
  int n_cu = 1;                // compute units of the device
  hipStream_t stream = nullptr;
  // second stream (default priority) on which the workgroup-team ACA kernel
  // runs beside the single-wave kernel, forked from and joined to `stream`
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::string last_error;
  DevBuf scratch_flag;   // small device scratch for readbacks (64 x int64)
  int64_t* pinned = nullptr;  // host pinned mirror for readbacks (64 x int64)
  bool profiling = false;
  std::vector<PhaseRec> pending;
  std::vector<hipEvent_t> event_pool;
  size_t budget_bytes = 0;     // device memory the ACA may use for factors
  int team_cls = 12;           // blocks with c + q >= 2^team_cls go to whole workgroups
  double phase_ms[HH_NPHASE] = {0};
  int64_t phase_cnt[HH_NPHASE] = {0};
  // this device's copy of the static scratch of hh_matvec_noalloc
  // (HH_NOALLOC_SCRATCH_BYTES), located when the context was created
  void* noalloc_scratch = nullptr;
};

// Records HIP events around a phase when profiling is on (RAII).
struct PhaseTimer {
  hh_ctx ctx;
  int phase;
  hipEvent_t a = nullptr;
  // on = false: records nothing (the allocation-free product)
  PhaseTimer(hh_ctx c, int ph, bool on = true);
  ~PhaseTimer();
};

// --------------------------------------------------------------- the kernel

// KIND_RPY6: the 6N Rotne-Prager mobility with rotations, on a tree whose
// rows are the 2n generalized rows (2i: translation / force of particle i,
// 2i + 1: rotation / torque)
enum { KIND_RPY = 0, KIND_MLP = 1, KIND_RPY6 = 2 };

struct hh_kernel_s {
  hh_ctx ctx = nullptr;
  int kind = KIND_RPY;
  int input_mode = HH_MLP_INPUT_DIRECTION;
  double a = 1.0, mu = 1.0;
  double alpha1 = 0.0;
  double alpha2 = 0.0;              // self mobility of odd rows (= alpha1 but for KIND_RPY6)
  std::vector<double> host_params;  // MLP, packed (HH_MLP_NPARAM)
  DevBuf p64;                       // MLP params FP64, packed
  DevBuf p32;                       // MLP params FP32, packed
  DevBuf pbf;                       // MLP params for the BF16 MFMA path
  DevBuf pf32;                      // MLP params for the FP32 MFMA path (fragment table)
  DevBuf pf32t;                     // transposed weights for the FP32 MFMA backward
};

// Offsets of the packed MLP parameter vector.
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * 3)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H * MLP_H)
#define OFF_W4 (OFF_B3 + MLP_H)
#define OFF_B4 (OFF_W4 + 9 * MLP_H)
#define MLP_NP (OFF_B4 + 9)
static_assert(MLP_NP == HH_MLP_NPARAM, "packed MLP layout");

// ----------------------------------------------------------------- the tree

struct hh_tree_s {
  hh_ctx ctx = nullptr;
  int64_t n = 0;
  int32_t c_leaf = 0;            // largest leaf size over the systems
  DevBuf cl;                     // int32 [n_sys] leaf size of every system
  int64_t n_nodes = 0, n_leaves = 0;
  DevBuf perm;      // int32 [n]   input index at sorted position
  DevBuf keys;      // uint64 [n]  sorted Morton keys
  DevBuf xs;        // double [n][3] sorted positions
  DevBuf nodes;     // int4 [n_nodes] (begin, end, left, right)
  DevBuf parent;    // int32 [n_nodes]
  DevBuf bbox;      // double [n_nodes][6]
  DevBuf leaf_id;   // int32 [n_nodes] rank among leaves, -1 for internal
  DevBuf leaves;    // int32 [n_leaves] node id of each leaf, in order
  DevBuf leaf_of;   // int32 [n] leaf node of sorted position s
  DevBuf units;     // int2 [n_units] (leaf rank, chunk of 32 targets), built with the tree
  int64_t n_units = 0;
  int n_sys = 1;                    // independent systems (batched build)
  std::vector<int64_t> offs_host;   // particle offsets of the systems [n_sys+1]
  DevBuf offs;                      // same, on the device
  DevBuf roots;                     // int32 [n_sys] root node of each system
  // the rows are the 2 n_particles generalized rows of the 6N mobility
  // (n = 2 n_particles; sorted row 2p + s is row s of sorted particle p)
  bool six = false;
};

// A tree of generalized rows goes with the 6N kernel and only with it.
inline void check_kernel_tree(hh_tree t, hh_kernel k) {
  HH_REQUIRE(t->six == (k->kind == KIND_RPY6), HH_ERR_INVALID_ARG,
             "the 6N kernel needs a tree from hh_build_tree6, and such a tree the 6N kernel");
}

// ------------------------------------------------------------ the partition

struct hh_part_s {
  hh_ctx ctx = nullptr;
  hh_tree tree = nullptr;
  int64_t nG = 0, nH = 0;
  DevBuf G;        // int2 [nG] (tau, sigma) sorted
  DevBuf H;        // int2 [nH] (tau, sigma) sorted
  DevBuf near_ptr; // int32 [n_leaves+1] CSR of H by target leaf rank
  DevBuf far_ptr;  // int32 [n_nodes+1]  CSR of G by target node
  int64_t near_pairs = 0;   // sum over H of |tau||sigma|
  int64_t far_entries = 0;  // sum over G of |tau||sigma|
};

// ----------------------------------------------------- low-rank factors

#define LMAX_CAP 64

// Huge blocks of one size class in a launch (streamed mode): their count,
// the factor elements the largest of them may need, and their rows c + q.
struct HugeTier {
  int64_t nblk, need, rows;
};

// Work counters per launch range (int64 words): single waves, workgroups and
// up to ACA_MAX_TIERS huge tiers (ints), then the pool top (int64).
#define ACA_MAX_TIERS 20
#define ACA_COUNTERS 16

struct hh_lowrank_s {
  hh_ctx ctx = nullptr;
  hh_part part = nullptr;
  int prec = HH_FP64;
  int64_t nG = 0;
  int32_t l_max = 0;
  double eps = 0.0;
  DevBuf rank;      // int32 [nG]
  DevBuf flag;      // int32 [nG] 1 = dense fallback
  DevBuf piv;       // int32 [nG][2][LMAX_CAP] (i_k then j_k), local indices
  DevBuf fptr;      // int64 [nG][LMAX_CAP] element offset of factor k in pool
  DevBuf pool;      // factor storage (double or float), 9 (c + q + 1) per step: c_k, q_k, P_k
  int64_t pool_elems = 0;
  int64_t rank_sum = 0, n_fallback = 0, samples = 0, used_elems = 0;
  DevBuf toff;      // int64 [nG] offset of the block's t vectors (rank*3)
  DevBuf tbuf;      // t_k = Q_k F  storage (double), [rank_sum][3]
  // streamed mode: factors live only inside a batch of blocks
  bool streamed = false;
  bool stats_dirty = true;
  hh_kernel kern = nullptr;
  int64_t est_elems = 0;
  std::vector<int64_t> bounds;   // launch ranges of the work order
  int64_t ub_elems = 0;          // largest launch sum of c
  DevBuf uoff;                   // int64 [nG+1] prefix sums of c over the work order
  DevBuf lid, pos;               // int32 [nG] launch and work-order position of block b
  DevBuf arena;                  // per-wave factor arenas (streamed mode)
  int64_t arena_elems = 0, arena_workers = 0;
  DevBuf huge;                   // arenas of the workgroups taking huge blocks
  int64_t huge_elems = 0;        // elements allocated in `huge`
  DevBuf ublk;                   // double [ub_elems][3]
  DevBuf order;                  // int32 [nG] ACA work order (largest blocks first)
  std::vector<int64_t> nbig;     // per launch range: blocks for whole workgroups
  std::vector<int64_t> nhuge;    // per launch range: huge blocks (streamed mode)
  // per launch range: the huge blocks by size class, largest first (one tier
  // per class), and the rows c + q of the whole range
  std::vector<std::vector<HugeTier>> tiers;
  std::vector<int64_t> launch_rows, team_rows;   // rows c + q: all blocks, team blocks
  // product workspaces, kept between products (sorted F, near rows, far rows,
  // work counters)
  DevBuf ws_f, ws_near, ws_far, ws_cnt;
  // Gram history of the block being approximated, one slot per ACA worker
  DevBuf gram;
  int64_t gram_workers = 0, gram_stride = 0;
};

// ------------------------------------------------------------- helpers

size_t elem_size(int prec);
inline bool is_bf16(int prec) { return prec == HH_BF16 || prec == HH_BF16_SPLIT; }
void ctx_sync(hh_ctx ctx);
// Zeroes n 64-bit words on the stream with a kernel (no memset node, so it
// can sit in a captured graph).
void zero_words(hh_ctx ctx, void* p, int64_t n);
int64_t read_i64(hh_ctx ctx, const void* dev_ptr);
void read_bytes(hh_ctx ctx, void* host, const void* dev, size_t bytes);

// Scan / sort primitives (sort.hip).
// Exclusive prefix sum of n int64 values (in place allowed: in == out).
void scan_exclusive_i64(hh_ctx ctx, const int64_t* in, int64_t* out, int64_t n);
// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of key.
void radix_sort_u64(hh_ctx ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits);

// Near-field, ACA, far-field and combine launches (near.hip, aca.hip, apply.hip).
void launch_near(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec, const void* F,
                 void* Unear);
void launch_near_bf16(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const void* Fs, void* Un,
                      bool split);
// sgn = -1: the transposed product sum_j K(x_j - x_i) v_j
void launch_near_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const void* Fs, void* Un,
                     float sgn = 1.0f);
// FP32 MFMA back-propagation of near pairs and of the ACA samples
// (backward_mfma.hip); slots: vjp_f32_waves(ctx) x MLP_NP doubles each.
int64_t vjp_f32_waves(hh_ctx ctx);
void launch_near_vjp_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const float* Fs,
                         const float* ws, double* dXs, double* slots);
void launch_far_vjp_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k,
                        int64_t b0, int64_t b1, const int64_t* goff, const float* gpool,
                        double* dXs, double* slots);
void ensure_units(hh_ctx ctx, hh_tree t);
void launch_near_neg(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec, const void* Vs,
                     void* out);
void launch_aca(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr, double eps,
                int32_t l_max, int64_t* pool_top_dev);
