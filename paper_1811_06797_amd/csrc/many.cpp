// Batching form for whole solves: many independent block-AMEn solves (Section 5), each a
// sequence of small, latency-bound launches, run concurrently on one GPU. Host worker
// threads take problems from a shared counter; each worker owns a context (stream, caching
// allocator, scratch) on the caller's device, so the solves' kernels overlap on the chip
// while every solve runs exactly the kernels, in exactly the order, of a lone
// iga_amen_solve. Solutions are copied into the caller's context before the workers end.
#include <atomic>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

namespace iga {

int amen_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, double tol, const iga_amen_opts* opts,
              const iga_btt* x0, iga_btt** sol, iga_amen_stats* stats);
void release_scratch(iga_ctx* ctx);
void release_raw_cache(iga_ctx* ctx);
void release_batch_cache(iga_ctx* ctx);

namespace {

struct Worker {
  std::unique_ptr<iga_ctx> ctx;
  hipStream_t stream = nullptr;
};

// A copy of x whose buffers belong to ctx (enqueued on ctx's stream).
std::unique_ptr<iga_btt> copy_btt(iga_ctx* ctx, const iga_btt* x) {
  std::unique_ptr<iga_btt> y(new iga_btt());
  y->ctx = ctx;
  y->ell = x->ell;
  y->nblk = x->nblk;
  for (int d = 0; d < 3; ++d) y->n[d] = x->n[d];
  for (int d = 0; d < 4; ++d) y->r[d] = x->r[d];
  for (int d = 0; d < 3; ++d) {
    const size_t sz = (size_t)(d == x->ell ? x->nblk : 1) * x->r[d] * x->n[d] * x->r[d + 1];
    y->core[d].reset(ctx, sz);
    IGA_HIP(hipMemcpyAsync(y->core[d].get(), x->core[d].get(), sz * sizeof(double), hipMemcpyDeviceToDevice,
                           ctx->stream));
  }
  return y;
}

}  // namespace

int amen_many_impl(iga_ctx* ctx, int nprob, const iga_kkt* const* kkts, const iga_tt* const* yhats,
                   const double* tols, const iga_amen_opts* opts, int nworkers, iga_btt** sols,
                   iga_amen_stats* stats, int* status) {
  for (int i = 0; i < nprob; ++i) sols[i] = nullptr;
  if (nprob == 0) return IGA_OK;
  const int nw = std::max(1, std::min(nworkers, nprob));
  std::vector<Worker> workers(nw);
  for (auto& w : workers) {
    IGA_HIP(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
    w.ctx.reset(new iga_ctx());
    w.ctx->device = ctx->device;
    w.ctx->stream = w.stream;
    w.ctx->pool.reset(new Pool(ctx->device));
  }
  std::vector<iga_btt*> raw(nprob, nullptr);
  std::vector<std::string> msg(nprob);
  std::atomic<int> next{0};
  auto run = [&](Worker& w) {
    (void)hipSetDevice(ctx->device);
    for (int i = next++; i < nprob; i = next++) {
      iga_btt* sol = nullptr;
      int rc;
      try {
        rc = amen_impl(w.ctx.get(), kkts[i], yhats[i], tols[i], opts, nullptr, &sol, stats ? &stats[i] : nullptr);
      } catch (const Error& e) {
        rc = e.code;
        msg[i] = e.what();
      } catch (const std::bad_alloc&) {
        rc = IGA_ENOMEM;
        msg[i] = "host allocation failed";
      } catch (const std::exception& e) {
        rc = IGA_EINVAL;
        msg[i] = e.what();
      }
      status[i] = rc;
      raw[i] = sol;
    }
  };
  {
    std::vector<std::thread> threads;
    threads.reserve(nw);
    for (auto& w : workers) threads.emplace_back(run, std::ref(w));
    for (auto& t : threads) t.join();
  }
  // every worker stream is idle (each solve synchronises its stream before returning)
  int first_error = IGA_OK;
  std::string first_msg;
  for (int i = 0; i < nprob; ++i) {
    if (raw[i]) {
      sols[i] = copy_btt(ctx, raw[i]).release();
    } else if (first_error == IGA_OK) {
      first_error = status[i];
      first_msg = "amen_solve_many: problem " + std::to_string(i) + ": " + msg[i];
    }
  }
  IGA_HIP(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < nprob; ++i) delete raw[i];
  for (auto& w : workers) {
    IGA_HIP(hipStreamSynchronize(w.stream));
    release_scratch(w.ctx.get());
    release_raw_cache(w.ctx.get());
    release_batch_cache(w.ctx.get());
    w.ctx.reset();
    IGA_HIP(hipStreamDestroy(w.stream));
  }
  if (first_error != IGA_OK) fail(first_error, first_msg);
  return IGA_OK;
}

}  // namespace iga
