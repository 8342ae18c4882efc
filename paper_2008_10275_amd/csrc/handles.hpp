// The C ABI's opaque handles and the error guard every entry point runs its
// body in (shared by the translation units that implement include/lrcheb.h).
#pragma once
#include <memory>
#include <new>
#include <stdexcept>

#include "mlp.hpp"
#include "solver.hpp"

struct lrc_ctx_s {
  lrc::Ctx c;
};
struct lrc_ops_s {
  lrc::Ops o;
};
struct lrc_prob_s {
  lrc::Prob p;
  std::unique_ptr<lrc_ops_s> owned_ops;
};
struct lrc_mlp_s {
  lrc_ctx ctx;
  lrc::Mlp m;
};

namespace lrc {

// Runs f(), turning exceptions into status codes and the context's message.
template <class F>
lrc_status guarded(Ctx* ctx, F&& f) {
  try {
    if (ctx) ctx->err.clear();
    return f();
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return LRC_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return LRC_EINVAL;
  }
}

// Per-device set-up of the fixed scratch array of the allocation-free entry
// points (noalloc.hip); called by lrc_create with the device current.
void noalloc_init_device(int device);

}  // namespace lrc
