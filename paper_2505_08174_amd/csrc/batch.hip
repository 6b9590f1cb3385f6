// The batched form as one handle: many independent systems in one tree, one
// partition and one set of ACA launches (every system keeps its own root box,
// tree, leaf size and blocks), with the product U = M F recorded once in a HIP
// graph and replayed by a single graph launch per call.
//
// The graph holds every launch of hh_matvec on this handle: the gather of F,
// the near field, the far field (in streamed mode the ACA itself with the
// fused apply, including the workgroup-team kernel forked onto the context's
// second stream and joined back), the combine and the unpermute. It is
// recorded on a private capture stream after one eager product has sized
// every workspace, so the recorded launches allocate nothing and no memset
// node is recorded (workspaces are cleared by kernels). The graph is bound to
// the F and U pointers it was recorded with; a call with other pointers
// records a new one.
#include "api_guard.h"
#include "internal.h"

struct hh_batch_s {
  hh_ctx ctx = nullptr;
  hh_kernel kern = nullptr;
  hh_precision prec = HH_FP64;
  hh_tree tree = nullptr;
  hh_part part = nullptr;
  hh_lowrank lr = nullptr;
  int32_t n_sys = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* F = nullptr;
  void* U = nullptr;
  size_t graph_nodes = 0;
  int64_t launches = 0;
  ~hh_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) {
      (void)hipStreamSynchronize(cap);
      (void)hipStreamDestroy(cap);
    }
    hh_lowrank_free(lr);
    hh_part_free(part);
    hh_tree_free(tree);
  }
};

// A status of a nested entry point becomes an exception of this one.
static void nested(hh_ctx ctx, hh_status st) {
  if (st != HH_OK) throw hh_error{st, ctx->last_error};
}

extern "C" {

hh_status hh_batch_create(hh_ctx ctx, const double* X, const hh_batch_params* prm,
                          hh_kernel kern, hh_batch* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && X && prm && kern, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(prm->n_sys >= 1 && prm->offsets, HH_ERR_INVALID_ARG, "n_sys >= 1 and offsets needed");
  HH_REQUIRE(kern->kind != KIND_RPY6, HH_ERR_INVALID_ARG, "batched products take the 3N kernels");
  HH_REQUIRE(prm->prec == HH_FP64 || prm->prec == HH_FP32 || is_bf16(prm->prec),
             HH_ERR_INVALID_ARG, "unknown precision");
  hh_batch_s* b = new hh_batch_s();
  try {
    b->ctx = ctx;
    b->kern = kern;
    b->prec = prm->prec;
    b->n_sys = prm->n_sys;
    std::vector<int32_t> cls(prm->n_sys, prm->c_leaf);
    if (prm->c_leafs)
      for (int s = 0; s < prm->n_sys; ++s) cls[s] = prm->c_leafs[s];
    nested(ctx, hh_build_tree_batch_leaf(ctx, X, prm->offsets, prm->n_sys, cls.data(), &b->tree));
    nested(ctx, hh_partition(ctx, b->tree, prm->eta, 0, &b->part));
    nested(ctx, hh_aca_build(ctx, b->tree, b->part, kern, prm->prec, prm->eps, prm->l_max,
                             nullptr, &b->lr));
    HIP_OK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  } catch (...) {
    delete b;
    throw;
  }
  *out = b;
  HH_API_END(ctx)
}

hh_status hh_batch_matvec(hh_ctx ctx, hh_batch b, const void* F, void* U) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(b && F && U, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(b->ctx == ctx, HH_ERR_INVALID_ARG, "batch belongs to another context");
  if (!b->exec || b->F != F || b->U != U) {
    if (b->exec) {
      HIP_OK(hipGraphExecDestroy(b->exec));
      b->exec = nullptr;
    }
    if (b->graph) {
      HIP_OK(hipGraphDestroy(b->graph));
      b->graph = nullptr;
    }
    // eager product: computes U and sizes every workspace
    nested(ctx, hh_matvec(ctx, b->tree, b->part, b->lr, b->kern, b->prec, F, U));
    // the capture stream starts after everything queued so far
    hipStream_t home = ctx->stream;
    HIP_OK(hipStreamSynchronize(home));
    ctx->stream = b->cap;
    hipGraph_t g = nullptr;
    hh_status st = HH_OK;
    std::string msg;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      st = hh_matvec(ctx, b->tree, b->part, b->lr, b->kern, b->prec, F, U);
      msg = ctx->last_error;
      e = hipStreamEndCapture(b->cap, &g);
    }
    ctx->stream = home;
    if (st != HH_OK) {
      if (g) (void)hipGraphDestroy(g);
      throw hh_error{st, "while recording the product: " + msg};
    }
    HIP_OK(e);
    b->graph = g;
    HIP_OK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    HIP_OK(hipGraphGetNodes(g, nullptr, &b->graph_nodes));
    b->F = F;
    b->U = U;
  } else {
    HIP_OK(hipGraphLaunch(b->exec, ctx->stream));
    b->launches += 1;
  }
  HH_API_END(ctx)
}

hh_status hh_batch_info(hh_batch b, int64_t* n, int32_t* n_sys, int64_t* graph_nodes,
                        int64_t* graph_launches, hh_tree* tree, hh_part* part,
                        hh_lowrank* lr) {
  if (!b) return HH_ERR_INVALID_ARG;
  if (n) *n = b->tree->n;
  if (n_sys) *n_sys = b->n_sys;
  if (graph_nodes) *graph_nodes = (int64_t)b->graph_nodes;
  if (graph_launches) *graph_launches = b->launches;
  if (tree) *tree = b->tree;
  if (part) *part = b->part;
  if (lr) *lr = b->lr;
  return HH_OK;
}

void hh_batch_free(hh_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  delete b;
}

}  // extern "C"
