// Batches of independent all-at-once problems (declared in include/aao_heat.h).
//
// Each problem of a batch is an ordinary handle with its own slice of the
// batch workspace.  A batch call hands the problems, largest first, to a
// small pool of host threads, each driving its own HIP stream: the solves of
// different problems then overlap on the device, which matters most for the
// sequential S-tilde sweeps (small, latency-bound kernels).  Before the first
// solve the preconditioner graphs of all problems are captured one after the
// other, so that worker threads only replay graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "aao_internal.h"

struct aao_batch {
  std::vector<aao_problem*> probs;
  std::vector<int64_t> off_u, off_n, off_f;  // prefix sums: unknowns, nodes, forcing values
  std::vector<size_t> ws_off;                // byte offset of each problem's workspace
  size_t ws_need = 0;
  char* ws = nullptr;
  int device = 0;
  int nstreams = 4;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;            // one per stream, plus the caller's
  hipStream_t caller = nullptr;
  bool graphs_ready[2] = {false, false};
  std::vector<int> order;                    // problems by decreasing size
  std::string err;
};

namespace {

std::string g_batch_create_error;

int bfail(aao_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  else g_batch_create_error = msg;
  return code;
}

int bhip(aao_batch* b, hipError_t e, const char* what) {
  if (e == hipSuccess) return AAO_OK;
  return bfail(b, AAO_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

// Run job(i, stream) for every problem i on the worker streams.  The workers
// start after the work already queued on the caller's stream, and the
// caller's stream waits for all of them.  Returns the first failing status.
template <class Job>
int run_pool(aao_batch* b, Job job) {
  const int count = (int)b->probs.size();
  const int W = std::min(b->nstreams, count);
  hipEvent_t start = b->events[b->nstreams];
  int rc = bhip(b, hipEventRecord(start, b->caller), "batch start event");
  for (int w = 0; rc == AAO_OK && w < W; ++w) rc = bhip(b, hipStreamWaitEvent(b->streams[w], start, 0), "stream wait");
  if (rc != AAO_OK) return rc;
  std::atomic<int> next{0};
  std::vector<int> status(count, AAO_OK);
  auto worker = [&](int w) {
    if (hipSetDevice(b->device) != hipSuccess) {
      status[0] = AAO_HIP_ERROR;
      return;
    }
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= count) break;
      const int i = b->order[k];
      status[i] = job(i, b->streams[w]);
    }
  };
  std::vector<std::thread> threads;
  threads.reserve(W);
  for (int w = 0; w < W; ++w) threads.emplace_back(worker, w);
  for (auto& t : threads) t.join();
  for (int w = 0; w < W; ++w) {
    hipError_t e = hipEventRecord(b->events[w], b->streams[w]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->caller, b->events[w], 0);
    if (e != hipSuccess && rc == AAO_OK) rc = bhip(b, e, "batch end event");
  }
  int worst = AAO_OK;
  for (int i = 0; i < count; ++i) {
    if (status[i] == AAO_OK) continue;
    if (worst == AAO_OK || (worst == AAO_NOT_CONVERGED && status[i] < 0)) {
      worst = status[i];
      b->err = "problem " + std::to_string(i) + ": " + (b->probs[i]->err.empty() ? "failed" : b->probs[i]->err);
    }
  }
  return rc != AAO_OK ? rc : worst;
}

int check_ready(aao_batch* b) {
  if (!b) return AAO_INVALID_ARG;
  if (!b->ws) return bfail(b, AAO_NO_WORKSPACE, "aao_batch_set_workspace first");
  return AAO_OK;
}

// Capture the preconditioner graphs of every problem, one after the other.
int ensure_graphs(aao_batch* b, bool transpose) {
  if (b->graphs_ready[transpose]) return AAO_OK;
  for (size_t i = 0; i < b->probs.size(); ++i) {
    aao_problem* h = b->probs[i];
    const hipError_t e = aao::prepare_graph(h, transpose);
    if (e != hipSuccess) return bhip(b, e, "graph capture");
  }
  b->graphs_ready[transpose] = true;
  return AAO_OK;
}

}  // namespace

extern "C" {

int aao_create_batch(const aao_desc* descs, int count, const aao_opts* opts, int streams, aao_batch** out) {
  if (!descs || !out || count < 1) return bfail(nullptr, AAO_INVALID_ARG, "descs, out and count >= 1 required");
  if (streams < 1 || streams > AAO_BATCH_MAX_STREAMS)
    return bfail(nullptr, AAO_INVALID_ARG, "streams must be in [1, 4]");
  *out = nullptr;
  aao_batch* b = new (std::nothrow) aao_batch();
  if (!b) return bfail(nullptr, AAO_INVALID_ARG, "out of host memory");
  b->nstreams = streams;
  b->off_u.assign(1, 0);
  b->off_n.assign(1, 0);
  b->off_f.assign(1, 0);
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    aao_problem* h = nullptr;
    const int rc = aao_create_problem(&descs[i], opts, &h);
    if (rc != AAO_OK) {
      const std::string why = aao_last_error(nullptr);
      aao_batch_destroy(b);
      return bfail(nullptr, rc, "problem " + std::to_string(i) + ": " + why);
    }
    b->probs.push_back(h);
    b->off_u.push_back(b->off_u.back() + h->U);
    b->off_n.push_back(b->off_n.back() + h->N);
    b->off_f.push_back(b->off_f.back() + h->UV);
    size_t need = 0;
    aao_workspace_size(h, &need);
    b->ws_off.push_back(off);
    off += (need + 255) & ~size_t(255);
  }
  b->ws_need = off;
  b->order.resize(count);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [b](int x, int y) { return b->probs[x]->U * b->probs[x]->s > b->probs[y]->U * b->probs[y]->s; });
  *out = b;
  return AAO_OK;
}

int aao_batch_count(const aao_batch* b) { return b ? (int)b->probs.size() : 0; }

int aao_batch_offsets(const aao_batch* b, int64_t* unknowns, int64_t* nodes, int64_t* forcing) {
  if (!b) return AAO_INVALID_ARG;
  const size_t c = b->probs.size() + 1;
  if (unknowns) std::copy(b->off_u.begin(), b->off_u.begin() + c, unknowns);
  if (nodes) std::copy(b->off_n.begin(), b->off_n.begin() + c, nodes);
  if (forcing) std::copy(b->off_f.begin(), b->off_f.begin() + c, forcing);
  return AAO_OK;
}

int aao_batch_workspace_size(const aao_batch* b, size_t* bytes) {
  if (!b || !bytes) return AAO_INVALID_ARG;
  *bytes = b->ws_need;
  return AAO_OK;
}

int aao_batch_set_workspace(aao_batch* b, void* dev_ptr, size_t bytes) {
  if (!b) return AAO_INVALID_ARG;
  if (!dev_ptr) return bfail(b, AAO_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return bfail(b, AAO_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < b->ws_need) return bfail(b, AAO_WORKSPACE_TOO_SMALL, "workspace too small");
  int rc = bhip(b, hipGetDevice(&b->device), "hipGetDevice");
  if (rc != AAO_OK) return rc;
  if (b->streams.empty()) {
    b->streams.assign(b->nstreams, nullptr);
    b->events.assign(b->nstreams + 1, nullptr);
    for (int w = 0; w < b->nstreams && rc == AAO_OK; ++w)
      rc = bhip(b, hipStreamCreateWithFlags(&b->streams[w], hipStreamNonBlocking), "stream create");
    for (int w = 0; w <= b->nstreams && rc == AAO_OK; ++w)
      rc = bhip(b, hipEventCreateWithFlags(&b->events[w], hipEventDisableTiming), "event create");
    if (rc != AAO_OK) return rc;
  }
  char* base = static_cast<char*>(dev_ptr);
  for (size_t i = 0; i < b->probs.size(); ++i) {
    aao_problem* h = b->probs[i];
    aao_set_stream(h, b->streams[i % b->nstreams]);
    const int r = aao_set_workspace(h, base + b->ws_off[i], h->ws_need);
    if (r != AAO_OK) return bfail(b, r, "problem " + std::to_string(i) + ": " + h->err);
  }
  b->ws = base;
  b->graphs_ready[0] = b->graphs_ready[1] = false;
  return AAO_OK;
}

int aao_batch_set_stream(aao_batch* b, void* stream) {
  if (!b) return AAO_INVALID_ARG;
  b->caller = static_cast<hipStream_t>(stream);
  return AAO_OK;
}

int aao_batch_problem(aao_batch* b, int i, aao_problem** h) {
  if (!b || !h || i < 0 || i >= (int)b->probs.size()) return AAO_INVALID_ARG;
  *h = b->probs[i];
  return AAO_OK;
}

int aao_batch_assemble_rhs(aao_batch* b, const double* f, const double* u0, double* rhs) {
  int rc = check_ready(b);
  if (rc != AAO_OK) return rc;
  if (!f || !u0 || !rhs) return bfail(b, AAO_INVALID_ARG, "null pointer");
  return run_pool(b, [&](int i, hipStream_t st) {
    aao_problem* h = b->probs[i];
    aao_set_stream(h, st);
    return aao_assemble_rhs(h, f + b->off_f[i], u0 + b->off_n[i], rhs + b->off_u[i]);
  });
}

static int batch_solve(aao_batch* b, const double* rhs, double* x, aao_stats* stats, bool transpose) {
  int rc = check_ready(b);
  if (rc != AAO_OK) return rc;
  if (!rhs || !x || rhs == x) return bfail(b, AAO_INVALID_ARG, "right-hand side and solution must be distinct");
  // the graphs are captured with the device idle of this batch's work
  rc = bhip(b, hipStreamSynchronize(b->caller), "caller stream");
  if (rc == AAO_OK) rc = ensure_graphs(b, transpose);
  if (rc != AAO_OK) return rc;
  return run_pool(b, [&](int i, hipStream_t st) {
    aao_problem* h = b->probs[i];
    aao_set_stream(h, st);
    aao_stats* si = stats ? &stats[i] : nullptr;
    return transpose ? aao_solve_adjoint(h, rhs + b->off_u[i], x + b->off_u[i], si)
                     : aao_solve(h, rhs + b->off_u[i], x + b->off_u[i], si);
  });
}

int aao_batch_solve(aao_batch* b, const double* rhs, double* x, aao_stats* stats) {
  return batch_solve(b, rhs, x, stats, false);
}

int aao_batch_solve_adjoint(aao_batch* b, const double* g, double* lam, aao_stats* stats) {
  return batch_solve(b, g, lam, stats, true);
}

int aao_batch_grad_logkappa(aao_batch* b, const double* x, const double* lam, double* grad) {
  int rc = check_ready(b);
  if (rc != AAO_OK) return rc;
  if (!x || !lam || !grad) return bfail(b, AAO_INVALID_ARG, "null pointer");
  return run_pool(b, [&](int i, hipStream_t st) {
    aao_problem* h = b->probs[i];
    aao_set_stream(h, st);
    return aao_grad_logkappa(h, x + b->off_u[i], lam + b->off_u[i], grad + b->off_n[i]);
  });
}

const char* aao_batch_last_error(const aao_batch* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int aao_batch_destroy(aao_batch* b) {
  if (!b) return AAO_INVALID_ARG;
  for (aao_problem* h : b->probs) aao_destroy(h);
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->events)
    if (e) (void)hipEventDestroy(e);
  delete b;
  return AAO_OK;
}

}  // extern "C"
