// Shared internals of the IgA-TT library: error handling, a caching device
// allocator, device buffers and the opaque handle types of iga.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/iga.h"

namespace iga {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& msg);
inline void require(bool ok, int code, const std::string& msg) {
  if (!ok) fail(code, msg);
}
void set_last_error(const std::string& msg);
// Name of the driver phase in progress (reported with allocation failures).
extern thread_local const char* g_phase;

#define IGA_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      ::iga::fail(IGA_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_));     \
  } while (0)

// Caching device allocator: freed blocks are kept per exact size and reused,
// so that the solver's inner loops never call hipMalloc after warm-up.
class Pool {
 public:
  explicit Pool(int device) : device_(device) {}
  ~Pool();
  void* alloc(size_t bytes);
  void release(void* p);
  size_t bytes_in_use() const { return in_use_; }

 private:
  int device_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t in_use_ = 0;
};

}  // namespace iga

struct iga_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<iga::Pool> pool;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // optional event timing of the banded stage of the local matvec (iga_profile_*)
  struct ProfRec {
    hipEvent_t a, b;
    int op;  // 0: M, 1: K (FP64); 2, 3: FP32; 4, 5: BF16 products
    int launches;
    double flops;
    int stage = 2;  // 1: left interface, 2: banded operator core, 3: right interface
  };
  bool prof_on = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> prof_events;  // created events, reused
  size_t prof_next = 0;                 // next unused entry of prof_events
};

namespace iga {

// Owning device buffer from the context pool.
template <class T>
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(iga_ctx* ctx, size_t count) { reset(ctx, count); }
  ~DevBuf() { free(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ctx_(o.ctx_), p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      free();
      ctx_ = o.ctx_; p_ = o.p_; n_ = o.n_;
      o.p_ = nullptr; o.n_ = 0;
      ++gen_;
    }
    return *this;
  }
  void reset(iga_ctx* ctx, size_t count) {
    free();
    ctx_ = ctx;
    n_ = count;
    p_ = count ? static_cast<T*>(ctx->pool->alloc(count * sizeof(T))) : nullptr;
    ++gen_;
  }
  // grow-only reuse for scratch buffers
  void ensure(iga_ctx* ctx, size_t count) {
    if (count > n_ || ctx != ctx_) reset(ctx, count);
  }
  void free() {
    if (p_ && ctx_) ctx_->pool->release(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  // changes whenever the buffer is (re)allocated, so owners can cache facts about its contents
  unsigned gen() const { return gen_; }

 private:
  iga_ctx* ctx_ = nullptr;
  T* p_ = nullptr;
  size_t n_ = 0;
  unsigned gen_ = 0;
};
using DBuf = DevBuf<double>;
using FBuf = DevBuf<float>;
using IBuf = DevBuf<int>;

// A block of a TT-matrix core that is nonzero: left ranks [a0, a0+na), right ranks [b0, b0+nb).
struct RankBlock {
  int a0, na, b0, nb;
};

// Banded TT-matrix core [R0][n][2p+1][R1] plus the list of its nonzero rank blocks
// (one block for dense cores, nine for the block-diagonal middle core of K).
struct OpCore {
  int R0 = 0, R1 = 0, n = 0;
  std::vector<RankBlock> blocks;
  DBuf data;
};

}  // namespace iga

struct iga_tt {
  iga_ctx* ctx = nullptr;
  int n[3] = {0, 0, 0};
  int r[4] = {1, 0, 0, 1};
  double* core[3] = {nullptr, nullptr, nullptr};
  iga::DBuf own[3];
};

struct iga_btt {
  iga_ctx* ctx = nullptr;
  int n[3] = {0, 0, 0};
  int r[4] = {1, 0, 0, 1};
  int ell = 0;
  int nblk = 3;  // components carried by core ell: [nblk][r_ell][n_ell][r_ell+1]
  iga::DBuf core[3];
};

struct iga_ttop {
  iga_ctx* ctx = nullptr;
  int p = 0;
  int n[3] = {0, 0, 0};
  int R[4] = {1, 0, 0, 1};
  iga::OpCore core[3];
  // Reference operators for the local preconditioner (set by the assembly):
  // univariate banded [n][2p+1] mass and stiffness factors with the dominant
  // separable part of omega, and scales of the stiffness per direction.
  bool has_ref = false;
  iga::DBuf refM[3], refK[3];
  double ref_c[3] = {1, 1, 1};
};

struct iga_kkt {
  iga_ctx* ctx = nullptr;
  const iga_ttop* M = nullptr;
  const iga_ttop* K = nullptr;
  double beta = 0;
  // Block structure: block o of A f is sum_l cM[o][l] M f_l + cK[o][l] K f_l and block o of
  // the right-hand side is cb[o] M yhat. Stationary: 3 blocks (y, u, lambda). Time-dependent
  // (nt > 0 implicit Euler steps of length tau): 3 nt blocks y_1..y_nt, u_1..u_nt,
  // lambda_1..lambda_nt.
  int nblk = 3;
  int nt = 0;
  double tau = 0;
  std::vector<double> cM, cK, cb;  // [nblk][nblk], [nblk][nblk], [nblk]
  // Laplace-form reference TT-matrix (ranks 1,2,2,1) for the local preconditioner
  iga_ttop* Kref = nullptr;
  // univariate generalised eigen-decompositions of (c_d Kbar_d, Mbar_d): V_d [n][n], lambda_d [n]
  iga::DBuf Vn[3], lamn[3];
  ~iga_kkt();
};

namespace iga {
// Upload/attach helpers shared by the API and the solver.
void opcore_setup_blocks(iga_ctx* ctx, OpCore& c, const std::vector<RankBlock>& blocks);
int ceil_div(long a, long b);
}  // namespace iga
