// C ABI (include/lrcheb.h): argument checking, ownership, error capture.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "handles.hpp"
#include "prof.hpp"

using namespace lrc;

namespace {

using clk = std::chrono::steady_clock;

void validate_csr(int64_t n, const int64_t* rp, const int32_t* col, const double* val, int i) {
  const std::string op = "operator " + std::to_string(i) + ": ";
  LRC_CHECK(rp && (rp[n] == 0 || (col && val)), ST_EINVAL, op + "null CSR array");
  LRC_CHECK(rp[0] == 0, ST_EINVAL, op + "rowptr[0] must be 0");
  LRC_CHECK(rp[n] >= 0 && rp[n] < (int64_t(1) << 31), ST_EINVAL, op + "nnz out of range");
  for (int64_t r = 0; r < n; ++r) {
    LRC_CHECK(rp[r + 1] >= rp[r], ST_EINVAL, op + "rowptr not non-decreasing");
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
      LRC_CHECK(col[e] >= 0 && col[e] < n, ST_EINVAL, op + "column index out of range");
      LRC_CHECK(e == rp[r] || col[e] > col[e - 1], ST_EINVAL,
                op + "column indices must be strictly ascending within a row");
      LRC_CHECK(std::isfinite(val[e]), ST_EINVAL, op + "non-finite value");
    }
  }
}

// P = sum_i w_i K_i on the union pattern (host CSR)
CsrHost combine(const Ops& o, const std::vector<double>& w) {
  CsrHost P;
  P.n = o.n;
  P.rowptr.assign(o.n + 1, 0);
  std::vector<int32_t> cols;
  std::vector<double> vals;
  std::vector<double> acc(o.n, 0.0);
  std::vector<char> seen(o.n, 0);
  for (int64_t r = 0; r < o.n; ++r) {
    cols.clear();
    for (int i = 0; i < o.q; ++i) {
      const auto& K = o.host[i];
      for (int64_t e = K.rowptr[r]; e < K.rowptr[r + 1]; ++e) {
        const int32_t c = K.col[e];
        if (!seen[c]) { seen[c] = 1; cols.push_back(c); acc[c] = 0.0; }
        acc[c] += w[i] * K.val[e];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t c : cols) {
      P.col.push_back(c);
      P.val.push_back(acc[c]);
      seen[c] = 0;
    }
    P.rowptr[r + 1] = int64_t(P.col.size());
  }
  return P;
}

void build_levels(Prec& pr, hipStream_t s) {
  const SupernodalFactor& F = pr.F;
  const int TR = 16;   // output rows per product workgroup
  std::vector<std::vector<int2>> ft(F.nlev_fwd), bt(F.nlev_bwd), fr(F.nlev_fwd), br(F.nlev_bwd);
  std::vector<int64_t> soff_f(F.nsn, 0), soff_b(F.nsn, 0), lf(F.nlev_fwd, 0), lb(F.nlev_bwd, 0);
  std::vector<double> blk_f(F.nlev_fwd, 0.0), blk_b(F.nlev_bwd, 0.0);
  std::vector<int64_t> ns_f(F.nlev_fwd, 0), ns_b(F.nlev_bwd, 0);
  std::vector<int> nin_f(F.nlev_fwd, 0), nin_b(F.nlev_bwd, 0);
  std::vector<int> contrib_f(F.nlev_fwd, 0);
  std::vector<int64_t> out_b(F.nlev_bwd, 0);
  std::vector<std::vector<GatherRow>> gf(F.nlev_fwd), gb(F.nlev_bwd);
  for (int sn = 0; sn < F.nsn; ++sn) {
    const int f = F.ns[sn] + F.nb[sn];
    const int hf = F.height[sn], db = F.depth[sn];
    // nonzero entries of the dense blocks: a triangle of ns (ns + 1) / 2 and
    // the ns x nb rectangle (the products skip the triangle's zeros)
    const double nz = 0.5 * double(F.ns[sn]) * (F.ns[sn] + 1) + double(F.nb[sn]) * F.ns[sn];
    blk_f[hf] += nz;
    blk_b[db] += nz;
    ns_f[hf] += F.ns[sn];
    ns_b[db] += F.ns[sn];
    // x rows only for supernodes with children (they are boundaries of deeper fronts)
    out_b[db] += int64_t(F.height[sn] > 0 ? 2 : 1) * F.ns[sn];
    nin_f[hf] = std::max(nin_f[hf], F.ns[sn]);
    nin_b[db] = std::max(nin_b[db], f);
    for (int r0 = 0; r0 < f; r0 += TR) ft[hf].push_back(make_int2(sn, r0));
    for (int r0 = 0; r0 < F.ns[sn]; r0 += TR) bt[db].push_back(make_int2(sn, r0));
    soff_f[sn] = lf[hf];
    soff_b[sn] = lb[db];
    for (int p = 0; p < f; ++p) {
      fr[hf].push_back(make_int2(sn, p));
      br[db].push_back(make_int2(sn, p));
      const int64_t q = F.front_off[sn] + p;
      LRC_CHECK(F.asm_ptr[q + 1] - F.asm_ptr[q] < (int64_t(1) << 30), ST_EINVAL,
                "preconditioner: too many contributions to one front row");
      gf[hf].push_back(GatherRow{p < F.ns[sn] ? F.perm[F.j0[sn] + p] : -1,
                                 int(F.asm_ptr[q + 1] - F.asm_ptr[q]), F.asm_ptr[q]});
      if (F.asm_ptr[q + 1] > F.asm_ptr[q]) contrib_f[hf] = 1;
      gb[db].push_back(GatherRow{p < F.ns[sn] ? F.j0[sn] + p : -F.bnd[F.bnd_off[sn] + p - F.ns[sn]] - 1,
                                 0, 0});
    }
    lf[hf] += f;
    lb[db] += f;
  }
  pr.stage_rows = std::max(*std::max_element(lf.begin(), lf.end()),
                           *std::max_element(lb.begin(), lb.end()));
  std::vector<int2> all;
  std::vector<size_t> fto, bto, fro, bro;
  for (auto& L : ft) { fto.push_back(all.size()); all.insert(all.end(), L.begin(), L.end()); }
  for (auto& L : bt) { bto.push_back(all.size()); all.insert(all.end(), L.begin(), L.end()); }
  for (auto& L : fr) { fro.push_back(all.size()); all.insert(all.end(), L.begin(), L.end()); }
  for (auto& L : br) { bro.push_back(all.size()); all.insert(all.end(), L.begin(), L.end()); }
  pr.fwd_tasks = upload(all, s);
  pr.soff_fwd = upload(soff_f, s);
  pr.soff_bwd = upload(soff_b, s);
  std::vector<GatherRow> gall;
  std::vector<size_t> gfo, gbo;
  for (auto& L : gf) { gfo.push_back(gall.size()); gall.insert(gall.end(), L.begin(), L.end()); }
  for (auto& L : gb) { gbo.push_back(gall.size()); gall.insert(gall.end(), L.begin(), L.end()); }
  pr.grows = upload(gall, s);
  const int2* base = pr.fwd_tasks.as<int2>();
  const GatherRow* gbase = pr.grows.as<GatherRow>();
  pr.fwd.clear();
  pr.bwd.clear();
  // forward products read the ns own rows of each front and write all f rows;
  // backward products read all f rows and write the ns own rows twice (x, Z),
  // once (Z) for leaves
  for (size_t l = 0; l < ft.size(); ++l)
    pr.fwd.push_back({base + fto[l], int(ft[l].size()), base + fro[l], int(fr[l].size()),
                      gbase + gfo[l], nin_f[l], contrib_f[l] ? 0 : 1, blk_f[l], ns_f[l], lf[l]});
  for (size_t l = 0; l < bt.size(); ++l) {
    pr.bwd.push_back({base + bto[l], int(bt[l].size()), base + bro[l], int(br[l].size()),
                      gbase + gbo[l], nin_b[l], 1, blk_b[l], lb[l], out_b[l]});
    pr.bwd.back().z_rows = ns_b[l];
  }
  LRC_HIP(hipStreamSynchronize(s));
}

void upload_prec(Prec& pr, hipStream_t s) {
  auto t0 = clk::now();
  SupernodalFactor& F = pr.F;
  pr.perm = upload(F.perm, s);
  pr.j0 = upload(F.j0, s);
  pr.ns = upload(F.ns, s);
  pr.nb = upload(F.nb, s);
  pr.fw_off = upload(F.fw_off, s);
  pr.bw_off = upload(F.bw_off, s);
  pr.front_off = upload(F.front_off, s);
  pr.cb_off = upload(F.cb_off, s);
  pr.asm_ptr = upload(F.asm_ptr, s);
  pr.asm_src = upload(F.asm_src, s);
  pr.bnd_off = upload(F.bnd_off, s);
  pr.bnd = upload(F.bnd, s);
  {
    std::vector<int> leaf(size_t(F.nsn));
    for (int sn = 0; sn < F.nsn; ++sn) leaf[sn] = F.height[sn] == 0 ? 1 : 0;
    pr.leaf = upload(leaf, s);
    LRC_HIP(hipStreamSynchronize(s));   // leaf is a temporary
  }
  pr.fw64 = upload(F.fw, s);
  pr.bw64 = upload(F.bw, s);
  {
    std::vector<float> f32(F.fw.begin(), F.fw.end());
    pr.fw32 = upload(f32, s);
    LRC_HIP(hipStreamSynchronize(s));
    std::vector<float> b32(F.bw.begin(), F.bw.end());
    pr.bw32 = upload(b32, s);
    LRC_HIP(hipStreamSynchronize(s));
  }
  pr.cb_rows = F.cb_off[F.nsn];
  auto fill = [&](auto& P, const void* fw, const void* bw) {
    P.kind = 0;
    P.n = F.n;
    P.perm = pr.perm.as<int>();
    P.j0 = pr.j0.as<int>();
    P.ns = pr.ns.as<int>();
    P.nb = pr.nb.as<int>();
    P.fw_off = pr.fw_off.as<int64_t>();
    P.bw_off = pr.bw_off.as<int64_t>();
    P.front_off = pr.front_off.as<int64_t>();
    P.cb_off = pr.cb_off.as<int64_t>();
    P.asm_ptr = pr.asm_ptr.as<int64_t>();
    P.asm_src = pr.asm_src.as<int64_t>();
    P.bnd_off = pr.bnd_off.as<int64_t>();
    P.bnd = pr.bnd.as<int>();
    using TT = std::remove_const_t<std::remove_pointer_t<decltype(P.fw)>>;
    P.fw = static_cast<const TT*>(fw);
    P.bw = static_cast<const TT*>(bw);
    P.soff_fwd = pr.soff_fwd.as<int64_t>();
    P.soff_bwd = pr.soff_bwd.as<int64_t>();
    P.leaf = pr.leaf.as<int>();
  };
  build_levels(pr, s);
  fill(pr.p64, pr.fw64.p, pr.bw64.p);
  fill(pr.p32, pr.fw32.p, pr.bw32.p);
  LRC_HIP(hipStreamSynchronize(s));
  // the dense blocks live on the device now
  std::vector<double>().swap(F.fw);
  std::vector<double>().swap(F.bw);
  pr.seconds_upload = std::chrono::duration<double>(clk::now() - t0).count();
}

}  // namespace

extern "C" {

lrc_status lrc_mlp_create(lrc_ctx ctx, const int sizes[4], const float* params, lrc_mlp* out) {
  if (!ctx || !out) return LRC_EINVAL;
  *out = nullptr;
  return guarded(&ctx->c, [&]() -> lrc_status {
    LRC_CHECK(sizes && params, ST_EINVAL, "mlp: sizes and params are required");
    auto h = std::make_unique<lrc_mlp_s>();
    h->ctx = ctx;
    h->m.init(sizes, params, ctx->c.stream);
    *out = h.release();
    return LRC_OK;
  });
}

void lrc_mlp_destroy(lrc_mlp mlp) {
  if (!mlp) return;
  (void)hipStreamSynchronize(mlp->ctx->c.stream);
  delete mlp;
}

static void mlp_check_batch(int B) {
  LRC_CHECK(B >= 1 && B <= 4096, ST_EINVAL, "mlp: batch size must be in [1, 4096]");
}

lrc_status lrc_mlp_fit_scaling(lrc_mlp mlp, int B, const double* X, const double* T) {
  if (!mlp) return LRC_EINVAL;
  return guarded(&mlp->ctx->c, [&]() -> lrc_status {
    mlp_check_batch(B);
    LRC_CHECK(X && T, ST_EINVAL, "mlp: null data");
    mlp->m.fit(B, X, T, mlp->ctx->c.stream);
    return LRC_OK;
  });
}

lrc_status lrc_mlp_grad(lrc_mlp mlp, int B, const double* X, const double* T, float* loss,
                        float* grads) {
  if (!mlp) return LRC_EINVAL;
  return guarded(&mlp->ctx->c, [&]() -> lrc_status {
    mlp_check_batch(B);
    LRC_CHECK(X && T, ST_EINVAL, "mlp: null data");
    hipStream_t s = mlp->ctx->c.stream;
    mlp->m.targets(B, T, s);
    mlp->m.forward(B, X, s);
    mlp->m.backward(B, s);
    if (loss) LRC_HIP(hipMemcpyAsync(loss, mlp->m.lossd.p, 4, hipMemcpyDeviceToHost, s));
    if (grads)
      LRC_HIP(hipMemcpyAsync(grads, mlp->m.Gr.p, size_t(mlp->m.np) * 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    return LRC_OK;
  });
}

lrc_status lrc_mlp_train(lrc_mlp mlp, int B, const double* X, const double* T, int steps,
                         float lr, float beta1, float beta2, float eps, float* loss_hist) {
  if (!mlp) return LRC_EINVAL;
  return guarded(&mlp->ctx->c, [&]() -> lrc_status {
    mlp_check_batch(B);
    LRC_CHECK(X && T && steps >= 0, ST_EINVAL, "mlp: null data or negative step count");
    hipStream_t s = mlp->ctx->c.stream;
    DevBuf hist(size_t(std::max(steps, 1)) * 4);
    mlp->m.targets(B, T, s);
    for (int it = 0; it < steps; ++it) {
      mlp->m.forward(B, X, s);
      mlp->m.backward(B, s);
      LRC_HIP(hipMemcpyAsync(hist.as<float>() + it, mlp->m.lossd.p, 4, hipMemcpyDeviceToDevice, s));
      mlp->m.adam(lr, beta1, beta2, eps, s);
    }
    if (loss_hist && steps > 0)
      LRC_HIP(hipMemcpyAsync(loss_hist, hist.p, size_t(steps) * 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    return LRC_OK;
  });
}

lrc_status lrc_mlp_predict(lrc_mlp mlp, int B, const double* X, double* Y) {
  if (!mlp) return LRC_EINVAL;
  return guarded(&mlp->ctx->c, [&]() -> lrc_status {
    mlp_check_batch(B);
    LRC_CHECK(X && Y, ST_EINVAL, "mlp: null data");
    hipStream_t s = mlp->ctx->c.stream;
    mlp->m.forward(B, X, s);
    mlp->m.outputs(B, Y, s);
    return LRC_OK;
  });
}

lrc_status lrc_mlp_get_params(lrc_mlp mlp, float* params) {
  if (!mlp || !params) return LRC_EINVAL;
  return guarded(&mlp->ctx->c, [&]() -> lrc_status {
    hipStream_t s = mlp->ctx->c.stream;
    LRC_HIP(hipMemcpyAsync(params, mlp->m.P.p, size_t(mlp->m.np) * 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    return LRC_OK;
  });
}

lrc_status lrc_profile_enable(int mode) {
  if (mode < 0 || mode > 2) return LRC_EINVAL;
  Profiler& p = profiler();
  if (mode) p.clear();
  p.mode = mode;
  return LRC_OK;
}

int lrc_profile_read(int ncls, double* ms, int* count, double* work, int* unit) {
  double t[K_COUNT], w[K_COUNT];
  int c[K_COUNT], u[K_COUNT];
  profiler().read(t, c, w, u);
  for (int k = 0; k < K_COUNT && k < ncls; ++k) {
    if (ms) ms[k] = t[k];
    if (count) count[k] = c[k];
    if (work) work[k] = w[k];
    if (unit) unit[k] = u[k];
  }
  return K_COUNT;
}

const char* lrc_profile_class_name(int c) { return kclass_name(c); }

void lrc_opts_default(lrc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rank_cap = 20;
  o->trunc_tol = 1e-8;
  o->res_tol = 1e-8;
  o->max_iter = 200;
  o->restart = 6;
  o->cheb_c = 0.0;
  o->cheb_d = 0.0;
  o->precision = LRC_FP64;
  o->refine_max = 8;
  o->inner_tol = 1e-4;
  o->init = LRC_INIT_MEDIAN;
  o->median_tol = 1e-6;   // the Newton accuracy of the median problem in Sec. 5
  o->verify_fp64 = 1;
}

lrc_status lrc_create(lrc_ctx* out, int device, void* stream) {
  if (!out) return LRC_EINVAL;
  *out = nullptr;
  auto* c = new (std::nothrow) lrc_ctx_s();
  if (!c) return LRC_ENOMEM;
  lrc_status st = guarded(&c->c, [&]() -> lrc_status {
    int count = 0;
    LRC_HIP(hipGetDeviceCount(&count));
    LRC_CHECK(device >= 0 && device < count, ST_EINVAL, "lrc_create: no such device");
    LRC_HIP(hipSetDevice(device));
    c->c.device = device;
    c->c.handle = c;
    c->c.stream = static_cast<hipStream_t>(stream);
    noalloc_init_device(device);
    LRC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->c.pinned), 64 * sizeof(double)));
    LRC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->c.pinned_i), 64 * sizeof(int)));
    return LRC_OK;
  });
  if (st != LRC_OK) {
    static thread_local std::string last;
    last = c->c.err;
    delete c;
    return st;
  }
  *out = c;
  return LRC_OK;
}

void lrc_destroy(lrc_ctx ctx) {
  if (!ctx) return;
  if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
  if (ctx->c.pinned_i) (void)hipHostFree(ctx->c.pinned_i);
  delete ctx;
}

const char* lrc_last_error(lrc_ctx ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

lrc_status lrc_set_stream(lrc_ctx ctx, void* stream) {
  if (!ctx) return LRC_EINVAL;
  ctx->c.stream = static_cast<hipStream_t>(stream);
  return LRC_OK;
}

lrc_status lrc_ops_create(lrc_ctx ctx, int64_t n, int q, const int64_t* const* rowptr,
                          const int32_t* const* col, const double* const* val, lrc_ops* out) {
  if (!ctx || !out) return LRC_EINVAL;
  *out = nullptr;
  return guarded(&ctx->c, [&]() -> lrc_status {
    LRC_CHECK(n >= 1 && n < (int64_t(1) << 31), ST_EINVAL, "lrc_ops_create: n out of range");
    LRC_CHECK(q >= 1 && q <= kMaxOps, ST_EINVAL, "lrc_ops_create: q must be in [1, 8]");
    LRC_CHECK(rowptr && col && val, ST_EINVAL, "lrc_ops_create: null array list");
    for (int i = 0; i < q; ++i) validate_csr(n, rowptr[i], col[i], val[i], i);
    auto o = std::make_unique<lrc_ops_s>();
    Ops& O = o->o;
    O.ctx = &ctx->c;
    O.n = n;
    O.q = q;
    hipStream_t s = ctx->c.stream;
    LRC_HIP(hipSetDevice(ctx->c.device));
    for (int i = 0; i < q; ++i) {
      CsrHost h;
      h.n = n;
      const int64_t nnz = rowptr[i][n];
      h.rowptr.assign(rowptr[i], rowptr[i] + n + 1);
      h.col.assign(col[i], col[i] + nnz);
      h.val.assign(val[i], val[i] + nnz);
      std::vector<int> rp32(h.rowptr.begin(), h.rowptr.end());
      O.rowptr.push_back(upload(rp32, s));
      O.col.push_back(upload(h.col, s));
      O.val64.push_back(DevBuf(std::max<size_t>(nnz, 1) * 8));
      O.val32.push_back(DevBuf(std::max<size_t>(nnz, 1) * 4));
      LRC_HIP(hipStreamSynchronize(s));
      O.host.push_back(std::move(h));
      O.upload_values(i);
    }
    for (int i = 0; i < q; ++i) {
      const auto& rp = O.host[i].rowptr;
      const int64_t nnz = rp[n];
      int64_t maxrow = 0;
      for (int64_t r = 0; r < n; ++r) maxrow = std::max<int64_t>(maxrow, rp[r + 1] - rp[r]);
      const int mr = int(std::min<int64_t>(maxrow, 1 << 30));
      // the rows that hold entries (a list only when some rows are empty)
      std::vector<int> nz;
      for (int64_t r = 0; r < n; ++r)
        if (rp[r + 1] > rp[r]) nz.push_back(int(r));
      const bool list = int64_t(nz.size()) < n;
      O.rowlist.push_back(list ? upload(nz, s) : DevBuf());
      LRC_HIP(hipStreamSynchronize(s));   // nz is a temporary
      const int* rl = list ? O.rowlist.back().as<int>() : nullptr;
      const int64_t nr = list ? int64_t(nz.size()) : n;
      // padded copy for the solver's SpMM when the rows are about equally long
      // (stencils: a row then costs one round of index loads before its
      // factor rows, without the row-pointer round)
      const int ew = (mr >= 1 && mr <= 27 && double(mr) * double(nr) <= 1.5 * double(nnz) + 64.0 &&
                      double(mr) * double(nr) < double(int64_t(1) << 31))
                         ? mr
                         : 0;
      std::vector<int64_t> mp;
      if (ew) {
        mp.assign(size_t(ew) * nr, -1);
        std::vector<int> ec(size_t(ew) * nr, 0);
        for (int64_t x = 0; x < nr; ++x) {
          const int64_t r = list ? nz[size_t(x)] : x;
          const int64_t b = rp[r], e = rp[r + 1];
          for (int u = 0; u < ew; ++u) {
            const size_t slot = size_t(u) * nr + x;
            if (b + u < e) {
              mp[slot] = b + u;
              ec[slot] = O.host[i].col[size_t(b + u)];
            } else {
              ec[slot] = e > b ? O.host[i].col[size_t(b)] : int(r);
            }
          }
        }
        O.ecol.push_back(upload(ec, s));
        LRC_HIP(hipStreamSynchronize(s));   // ec is a temporary
        O.eval64.push_back(DevBuf(mp.size() * 8));
        O.eval32.push_back(DevBuf(mp.size() * 4));
      } else {
        O.ecol.push_back(DevBuf());
        O.eval64.push_back(DevBuf());
        O.eval32.push_back(DevBuf());
      }
      O.emap.push_back(std::move(mp));
      O.upload_values(i);
      O.d64.push_back({O.rowptr[i].as<int>(), O.col[i].as<int>(), O.val64[i].as<double>(), n, nnz,
                       mr, rl, nr, ew ? O.ecol[i].as<int>() : nullptr,
                       ew ? O.eval64[i].as<double>() : nullptr, ew});
      O.d32.push_back({O.rowptr[i].as<int>(), O.col[i].as<int>(), O.val32[i].as<float>(), n, nnz,
                       mr, rl, nr, ew ? O.ecol[i].as<int>() : nullptr,
                       ew ? O.eval32[i].as<float>() : nullptr, ew});
    }
    *out = o.release();
    return LRC_OK;
  });
}

lrc_status lrc_ops_update_values(lrc_ops ops, int i, const double* val) {
  if (!ops) return LRC_EINVAL;
  return guarded(ops->o.ctx, [&]() -> lrc_status {
    LRC_CHECK(i >= 0 && i < ops->o.q && val, ST_EINVAL, "lrc_ops_update_values: bad arguments");
    auto& h = ops->o.host[i];
    for (size_t e = 0; e < h.val.size(); ++e)
      LRC_CHECK(std::isfinite(val[e]), ST_EINVAL, "lrc_ops_update_values: non-finite value");
    std::copy(val, val + h.val.size(), h.val.begin());
    ops->o.upload_values(i);
    return LRC_OK;
  });
}

void lrc_ops_destroy(lrc_ops ops) { delete ops; }

lrc_status lrc_ops_spmm_dev(lrc_ops ops, int dtype, int r, const void* U, int ldu, void* W,
                            int ldw) {
  if (!ops) return LRC_EINVAL;
  return guarded(ops->o.ctx, [&]() -> lrc_status {
    const Ops& o = ops->o;
    const bool skip = (dtype & LRC_SPMM_SKIP_EMPTY) != 0;
    dtype &= ~LRC_SPMM_SKIP_EMPTY;
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "spmm: dtype must be 0 (fp64) or 1 (fp32)");
    LRC_CHECK(r >= 1 && r <= (dtype == 0 ? 128 : 256), ST_EINVAL, "spmm: r out of range");
    LRC_CHECK(U && W, ST_EINVAL, "spmm: null pointer");
    if (dtype == 0) {
      double* Wp[kMaxOps];
      for (int i = 0; i < o.q; ++i) Wp[i] = static_cast<double*>(W) + size_t(i) * o.n * ldw;
      auto l = make_spmm<double>(o.d64.data(), o.q, static_cast<const double*>(U), ldu, nullptr,
                                 r, r, Wp, ldw, spmm_config<double>(o, r), skip);
      l.a.wpad = 0;   // the caller's W: columns past r are left untouched
      enqueue_spmm(l, Batched<SpmmArgs<double>>(), o.ctx->stream);
    } else {
      float* Wp[kMaxOps];
      for (int i = 0; i < o.q; ++i) Wp[i] = static_cast<float*>(W) + size_t(i) * o.n * ldw;
      auto l = make_spmm<float>(o.d32.data(), o.q, static_cast<const float*>(U), ldu, nullptr, r,
                                r, Wp, ldw, spmm_config<float>(o, r), skip);
      l.a.wpad = 0;
      enqueue_spmm(l, Batched<SpmmArgs<float>>(), o.ctx->stream);
    }
    return LRC_OK;
  });
}

lrc_status lrc_ops_spmm_shape_dev(lrc_ops ops, int dtype, int r, const void* U, int ldu, void* W,
                                  int ldw, const int cfg[3]) {
  if (!ops || !cfg) return LRC_EINVAL;
  return guarded(ops->o.ctx, [&]() -> lrc_status {
    const Ops& o = ops->o;
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "spmm: dtype must be 0 (fp64) or 1 (fp32)");
    LRC_CHECK(r >= 1 && r <= (dtype == 0 ? 128 : 256), ST_EINVAL, "spmm: r out of range");
    LRC_CHECK(U && W, ST_EINVAL, "spmm: null pointer");
    const SpmmCfg c{cfg[0], cfg[1], cfg[2]};
    if (dtype == 0) {
      double* Wp[kMaxOps];
      for (int i = 0; i < o.q; ++i) Wp[i] = static_cast<double*>(W) + size_t(i) * o.n * ldw;
      auto l = make_spmm<double>(o.d64.data(), o.q, static_cast<const double*>(U), ldu, nullptr,
                                 r, r, Wp, ldw, c);
      l.a.wpad = 0;
      enqueue_spmm(l, Batched<SpmmArgs<double>>(), o.ctx->stream);
    } else {
      float* Wp[kMaxOps];
      for (int i = 0; i < o.q; ++i) Wp[i] = static_cast<float*>(W) + size_t(i) * o.n * ldw;
      auto l = make_spmm<float>(o.d32.data(), o.q, static_cast<const float*>(U), ldu, nullptr, r,
                                r, Wp, ldw, c);
      l.a.wpad = 0;
      enqueue_spmm(l, Batched<SpmmArgs<float>>(), o.ctx->stream);
    }
    return LRC_OK;
  });
}

lrc_status lrc_ops_spmm_tune(lrc_ops ops, int dtype, int r, int cfg[3], double times_us[2]) {
  if (!ops) return LRC_EINVAL;
  return guarded(ops->o.ctx, [&]() -> lrc_status {
    const Ops& o = ops->o;
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "spmm tune: dtype must be 0 (fp64) or 1 (fp32)");
    LRC_CHECK(r >= 1 && r <= (dtype == 0 ? 128 : 256), ST_EINVAL, "spmm tune: r out of range");
    const SpmmTuneResult res = dtype == 0 ? tune_spmm<double>(o, r) : tune_spmm<float>(o, r);
    if (cfg) {
      cfg[0] = res.best.cpl;
      cfg[1] = res.best.waves;
      cfg[2] = res.best.max_blocks;
    }
    if (times_us) {
      times_us[0] = res.best_us;
      times_us[1] = res.default_us;
    }
    return LRC_OK;
  });
}

lrc_status lrc_prob_create(lrc_ops ops, int64_t m, const double* d, int rF, const double* FU,
                           const double* Fs, const double* FV, lrc_prob* out) {
  if (!ops || !out) return LRC_EINVAL;
  *out = nullptr;
  return guarded(ops->o.ctx, [&]() -> lrc_status {
    Ops& o = ops->o;
    LRC_CHECK(m >= 1, ST_EINVAL, "lrc_prob_create: m must be positive");
    LRC_CHECK(d && FU && FV, ST_EINVAL, "lrc_prob_create: null input");
    LRC_CHECK(rF >= 1 && rF <= 64, ST_EINVAL, "lrc_prob_create: rank of F must be in [1, 64]");
    for (int64_t e = 0; e < int64_t(o.q) * m; ++e)
      LRC_CHECK(std::isfinite(d[e]), ST_EINVAL, "lrc_prob_create: non-finite parameter");
    for (int64_t e = 0; e < o.n * rF; ++e)
      LRC_CHECK(std::isfinite(FU[e]), ST_EINVAL, "lrc_prob_create: non-finite entry in FU");
    for (int64_t e = 0; e < m * rF; ++e)
      LRC_CHECK(std::isfinite(FV[e]), ST_EINVAL, "lrc_prob_create: non-finite entry in FV");
    auto pr = std::make_unique<lrc_prob_s>();
    Prob& P = pr->p;
    P.ops = &o;
    P.ctx = o.ctx;
    P.m = m;
    P.d.assign(d, d + size_t(o.q) * m);
    P.rF = rF;
    P.FU.assign(FU, FU + size_t(o.n) * rF);
    P.FV.assign(FV, FV + size_t(m) * rF);
    P.Fs.assign(rF, 1.0);
    if (Fs) P.Fs.assign(Fs, Fs + rF);
    std::vector<double> rows(size_t(o.q) * m);
    for (int i = 0; i < o.q; ++i)
      for (int64_t j = 0; j < m; ++j) rows[size_t(i) * m + j] = d[size_t(j) * o.q + i];
    hipStream_t s = o.ctx->stream;
    P.d_rows = upload(rows, s);
    P.F64.alloc(o.n, m, rF, s);
    // host column-major -> device row-major
    {
      std::vector<double> u(size_t(o.n) * P.F64.ld, 0.0), v(size_t(m) * P.F64.ld, 0.0);
      for (int a = 0; a < rF; ++a) {
        for (int64_t i = 0; i < o.n; ++i) u[size_t(i) * P.F64.ld + a] = FU[size_t(a) * o.n + i];
        for (int64_t j = 0; j < m; ++j) v[size_t(j) * P.F64.ld + a] = FV[size_t(a) * m + j];
      }
      LRC_HIP(hipMemcpyAsync(P.F64.U.p, u.data(), u.size() * 8, hipMemcpyHostToDevice, s));
      LRC_HIP(hipMemcpyAsync(P.F64.V.p, v.data(), v.size() * 8, hipMemcpyHostToDevice, s));
      LRC_HIP(hipMemcpyAsync(P.F64.s.p, P.Fs.data(), rF * 8, hipMemcpyHostToDevice, s));
      LRC_HIP(hipMemcpyAsync(P.F64.rank.p, &rF, 4, hipMemcpyHostToDevice, s));
      LRC_HIP(hipStreamSynchronize(s));
    }
    // ||F||_F^2 = sum_ab Fs_a Fs_b (FU^T FU)_ab (FV^T FV)_ab
    double f2 = 0.0;
    for (int a = 0; a < rF; ++a)
      for (int b = 0; b < rF; ++b) {
        double gu = 0.0, gv = 0.0;
        for (int64_t i = 0; i < o.n; ++i) gu += FU[size_t(a) * o.n + i] * FU[size_t(b) * o.n + i];
        for (int64_t j = 0; j < m; ++j) gv += FV[size_t(a) * m + j] * FV[size_t(b) * m + j];
        f2 += P.Fs[a] * P.Fs[b] * gu * gv;
      }
    P.fnorm = std::sqrt(std::max(f2, 0.0));
    LRC_CHECK(P.fnorm > 0.0, ST_EINVAL, "lrc_prob_create: F is zero");
    P.dbar.assign(o.q, 0.0);
    for (int i = 0; i < o.q; ++i) {
      double acc = 0.0;
      for (int64_t j = 0; j < m; ++j) acc += d[size_t(j) * o.q + i];
      P.dbar[i] = acc / double(m);
    }
    *out = pr.release();
    return LRC_OK;
  });
}

void lrc_prob_destroy(lrc_prob prob) { delete prob; }

// ILU(0) of P on the device: L\U values in fp64 and fp32 on P's pattern, the
// level row lists, one level entry per forward / backward level
static void upload_ilu(Prec& pr, hipStream_t s) {
  auto t0 = clk::now();
  const Ilu0& I = pr.ilu;
  LRC_CHECK(I.rowptr.back() < (int64_t(1) << 31) && I.n < (int64_t(1) << 31), ST_EINVAL,
            "ILU(0): the level kernels index rows and entries with 32-bit integers");
  std::vector<int> rp(I.rowptr.begin(), I.rowptr.end());
  pr.irp = upload(rp, s);
  pr.icol = upload(I.col, s);
  pr.idiag = upload(I.diag, s);
  pr.irows_f = upload(I.rows_f, s);
  pr.irows_b = upload(I.rows_b, s);
  pr.ilu64 = upload(I.lu, s);
  std::vector<float> f32(I.lu.begin(), I.lu.end());
  pr.ilu32 = upload(f32, s);
  LRC_HIP(hipStreamSynchronize(s));   // rp and f32 are temporaries
  auto levels = [&](const std::vector<int32_t>& rows, const std::vector<int32_t>& off, bool fw,
                    std::vector<LevelTasks>& out) {
    out.clear();
    for (size_t l = 0; l + 1 < off.size(); ++l) {
      LevelTasks L{};
      L.count = off[l + 1] - off[l];
      L.ilu_off = off[l];
      int64_t nnz = 0;
      for (int32_t x = off[l]; x < off[l + 1]; ++x) {
        const int32_t r = rows[x];
        nnz += fw ? I.diag[r] - I.rowptr[r] : I.rowptr[r + 1] - I.diag[r];
      }
      L.ilu_nnz = nnz;
      out.push_back(L);
    }
  };
  levels(I.rows_f, I.off_f, true, pr.fwd);
  levels(I.rows_b, I.off_b, false, pr.bwd);
  pr.stage_rows = 0;
  pr.cb_rows = 0;
  auto fill = [&](auto& P, const void* lu) {
    P = {};
    P.kind = 1;
    P.n = I.n;
    P.irp = pr.irp.as<int>();
    P.icol = pr.icol.as<int>();
    P.idiag = pr.idiag.as<int>();
    P.irows_f = pr.irows_f.as<int>();
    P.irows_b = pr.irows_b.as<int>();
    using TT = std::remove_const_t<std::remove_pointer_t<decltype(P.fw)>>;
    P.fw = static_cast<const TT*>(lu);
    P.bw = static_cast<const TT*>(lu);
  };
  fill(pr.p64, pr.ilu64.p);
  fill(pr.p32, pr.ilu32.p);
  pr.seconds_upload = std::chrono::duration<double>(clk::now() - t0).count();
}

lrc_status lrc_prob_precondition(lrc_prob prob, const double* dbar, int leaf_size, int kind) {
  if (!prob) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    auto t0 = clk::now();
    const Ops& o = *P.ops;
    LRC_CHECK(kind == LRC_PREC_LU || kind == LRC_PREC_ILU0, ST_EINVAL,
              "lrc_prob_precondition: kind must be LRC_PREC_LU or LRC_PREC_ILU0");
    if (dbar) {
      for (int i = 0; i < o.q; ++i)
        LRC_CHECK(std::isfinite(dbar[i]), ST_EINVAL, "lrc_prob_precondition: non-finite dbar");
      P.dbar.assign(dbar, dbar + o.q);
    }
    CsrHost Pm = combine(o, P.dbar);
    if (kind == LRC_PREC_ILU0) {
      auto pr = std::make_unique<Prec>();
      pr->kind = 1;
      std::string err;
      const int rc = ilu0_factor(Pm, &pr->ilu, &err);
      if (rc == -4) throw Error(ST_ESINGULAR, err);
      if (rc != 0) throw Error(ST_EINVAL, err);
      upload_ilu(*pr, P.ctx->stream);
      P.prec = std::move(pr);
      P.seconds_setup = std::chrono::duration<double>(clk::now() - t0).count();
      return LRC_OK;
    }
    auto pr = std::make_unique<Prec>();
    std::string err;
    // 64-node leaves: two tree levels (six launches per apply) fewer than 16-node
    // leaves for a denser leaf level; fastest of 16..256 on the 513 x 513 grid
    const int rc = nd_factor(Pm, leaf_size > 0 ? leaf_size : 64, 0, &pr->F, &err);
    if (rc == -4) throw Error(ST_ESINGULAR, err);
    if (rc != 0) throw Error(ST_EINVAL, err);
    upload_prec(*pr, P.ctx->stream);
    P.prec = std::move(pr);
    P.seconds_setup = std::chrono::duration<double>(clk::now() - t0).count();
    return LRC_OK;
  });
}

lrc_status lrc_prob_spectrum(lrc_prob prob, double* c, double* d) {
  if (!prob || !c || !d) return LRC_EINVAL;
  const Prob& P = prob->p;
  double lo = 1.0, hi = 1.0;
  for (int64_t j = 0; j < P.m; ++j)
    for (int i = 0; i < P.ops->q; ++i) {
      const double r = P.d[size_t(j) * P.ops->q + i] / P.dbar[i];
      lo = std::min(lo, r);
      hi = std::max(hi, r);
    }
  *c = 0.5 * (hi - lo);
  *d = 0.5 * (hi + lo);
  return LRC_OK;
}

lrc_status lrc_prob_precond_stats(lrc_prob prob, double out[8]) {
  if (!prob || !out) return LRC_EINVAL;
  const Prob& P = prob->p;
  if (!P.prec) {
    P.ctx->err = "lrc_prob_precond_stats: no preconditioner";
    return LRC_EINVAL;
  }
  const auto& F = P.prec->F;
  if (P.prec->kind == 1) {
    // ILU(0): rows as "supernodes", its levels, no dense fronts, its entries
    const Ilu0& I = P.prec->ilu;
    out[0] = double(I.n);
    out[1] = double(I.off_f.size() - 1);
    out[2] = double(I.off_b.size() - 1);
    out[3] = 1.0;
    out[4] = double(I.lu.size());
    out[5] = 0.0;
    out[6] = 0.0;
    out[7] = P.prec->seconds_upload;
    return LRC_OK;
  }
  out[0] = F.nsn;
  out[1] = F.nlev_fwd;
  out[2] = F.nlev_bwd;
  out[3] = double(F.max_front);
  out[4] = F.dense_entries;
  out[5] = F.seconds_order;
  out[6] = F.seconds_factor;
  out[7] = P.prec->seconds_upload;
  return LRC_OK;
}

lrc_status lrc_prob_prec_apply_dev(lrc_prob prob, int dtype, int k, const void* R, int ldr,
                                   void* Z, int ldz) {
  if (!prob) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    LRC_CHECK(P.prec != nullptr, ST_EINVAL, "prec_apply: no preconditioner");
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "prec_apply: dtype must be 0 or 1");
    LRC_CHECK(k >= 1 && k <= kPrecCols && ldr >= k && ldz >= k && R && Z, ST_EINVAL,
              "prec_apply: bad arguments");
    const int64_t n = P.ops->n;
    const int ld = ld_for(k);
    const size_t es = dtype == 0 ? 8 : 4;
    DevBuf y(size_t(n) * ld * es), x(size_t(n) * ld * es),
        cb(size_t(std::max<int64_t>(P.prec->cb_rows, 1)) * ld * es),
        st(size_t(std::max<int64_t>(P.prec->stage_rows, 1)) * ld * es);
    hipStream_t s = P.ctx->stream;
    if (dtype == 0)
      launch_prec_apply<double>(P.prec->p64, P.prec->fwd, P.prec->bwd,
                                static_cast<const double*>(R), ldr, static_cast<double*>(Z), ldz,
                                nullptr, k, k, y.as<double>(), x.as<double>(), cb.as<double>(),
                                st.as<double>(), ld, s);
    else
      launch_prec_apply<float>(P.prec->p32, P.prec->fwd, P.prec->bwd,
                               static_cast<const float*>(R), ldr, static_cast<float*>(Z), ldz,
                               nullptr, k, k, y.as<float>(), x.as<float>(), cb.as<float>(),
                               st.as<float>(), ld, s);
    LRC_HIP(hipStreamSynchronize(s));   // scratch buffers are released on return
    return LRC_OK;
  });
}

lrc_status lrc_solve(lrc_prob prob, const lrc_opts* opts, int r0, const double* U0,
                     const double* s0, const double* V0, lrc_info* info) {
  if (!prob || !opts) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    LRC_HIP(hipSetDevice(P.ctx->device));
    return solve_problem(P, *opts, r0, U0, s0, V0, info);
  });
}

lrc_status lrc_solve_x0_dev(lrc_prob prob, const lrc_opts* opts, int r0, const double* U0_dev,
                            int ldu, const double* s0, const double* V0_dev, int ldv,
                            lrc_info* info) {
  if (!prob || !opts) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    LRC_HIP(hipSetDevice(P.ctx->device));
    LRC_CHECK((opts->init == LRC_INIT_GIVEN || opts->init == LRC_INIT_GIVEN_JUDGED ||
               opts->init == LRC_INIT_NEWTON) && r0 >= 1,
              ST_EINVAL, "lrc_solve_x0_dev: needs a given initial term (init GIVEN, "
                         "GIVEN_JUDGED or NEWTON) and r0 >= 1");
    const X0Dev xd{U0_dev, ldu, V0_dev, ldv};
    return solve_problem(P, *opts, r0, nullptr, s0, nullptr, info, &xd);
  });
}

lrc_status lrc_solve_batched(lrc_prob* probs, int K, const lrc_opts* opts, lrc_info* infos) {
  if (!probs || K < 1 || !opts) return LRC_EINVAL;
  for (int k = 0; k < K; ++k)
    if (!probs[k]) return LRC_EINVAL;
  Ctx* cx = probs[0]->p.ctx;
  return guarded(cx, [&]() -> lrc_status {
    LRC_HIP(hipSetDevice(cx->device));
    LRC_CHECK(opts->init == LRC_INIT_ZERO || opts->init == LRC_INIT_MEDIAN, ST_EINVAL,
              "lrc_solve_batched: given initial terms are not supported (use lrc_solve)");
    std::vector<Prob*> ps(K);
    for (int k = 0; k < K; ++k) ps[k] = &probs[k]->p;
    std::vector<lrc_info> inf(K);
    const auto st = solve_batched(ps, *opts, inf.data());
    lrc_status worst = LRC_OK;
    for (int k = 0; k < K; ++k) {
      inf[k].status = st[k];
      worst = std::max(worst, lrc_status(st[k]));
      if (infos) infos[k] = inf[k];
    }
    return worst;
  });
}

lrc_status lrc_get_solution(lrc_prob prob, int* rank, double* U, double* s, double* V) {
  if (!prob || !rank) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    LRC_CHECK(P.S.U.p != nullptr, ST_EINVAL, "lrc_get_solution: nothing solved yet");
    const int r0 = P.rank_x0, rs = P.rank_s;
    *rank = r0 + rs;
    if (!U && !s && !V) return LRC_OK;
    LRC_CHECK(U && s && V, ST_EINVAL, "lrc_get_solution: U, s and V are all required");
    const int64_t n = P.ops->n, m = P.m;
    hipStream_t st = P.ctx->stream;
    auto fetch = [&](const LR<double>& X, int r, int col0) {
      if (r == 0) return;
      std::vector<double> u(size_t(n) * X.ld), v(size_t(m) * X.ld), sv(r);
      LRC_HIP(hipMemcpyAsync(u.data(), X.U.p, u.size() * 8, hipMemcpyDeviceToHost, st));
      LRC_HIP(hipMemcpyAsync(v.data(), X.V.p, v.size() * 8, hipMemcpyDeviceToHost, st));
      LRC_HIP(hipMemcpyAsync(sv.data(), X.s.p, size_t(r) * 8, hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      for (int a = 0; a < r; ++a) {
        for (int64_t i = 0; i < n; ++i) U[size_t(col0 + a) * n + i] = u[size_t(i) * X.ld + a];
        for (int64_t j = 0; j < m; ++j) V[size_t(col0 + a) * m + j] = v[size_t(j) * X.ld + a];
        s[col0 + a] = sv[a];
      }
    };
    fetch(P.X0, r0, 0);
    fetch(P.S, rs, r0);
    return LRC_OK;
  });
}

lrc_status lrc_residual(lrc_prob prob, double* relres, double* colres) {
  if (!prob || !relres) return LRC_EINVAL;
  Prob& P = prob->p;
  return guarded(P.ctx, [&]() -> lrc_status {
    LRC_CHECK(P.S.U.p != nullptr, ST_EINVAL, "lrc_residual: nothing solved yet");
    // the last solve's convention: a Newton step's linearisation point is not
    // part of its equation; residuals relative to its reference norm
    *relres = residual_fp64(P, P.X0, P.newton_point ? 0 : P.rank_x0, P.S, colres) /
              (P.ref > 0.0 ? P.ref : P.fnorm);
    return LRC_OK;
  });
}

lrc_status lrc_truncate_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m, int k,
                            const void* A, int lda, const double* c, const void* B, int ldb,
                            int rank_cap, double tol, void* U, int ldu, double* s, void* V,
                            int ldv, int* rank) {
  if (!ctx) return LRC_EINVAL;
  return guarded(&ctx->c, [&]() -> lrc_status {
    LRC_CHECK(dtype == 0 || dtype == 1 || dtype == 2, ST_EINVAL, "truncate: dtype must be 0, 1 or 2");
    LRC_CHECK(n >= 1 && m >= 1 && k >= 1 && k <= kTruncCap, ST_EINVAL,
              "truncate: need n, m >= 1 and 1 <= k <= 128");
    LRC_CHECK(rank_cap >= 1 && rank_cap <= 64 && rank_cap <= ldu && rank_cap <= ldv, ST_EINVAL,
              "truncate: rank_cap in [1, 64] and <= ldu, ldv");
    LRC_CHECK(A && B && c && U && V && s && rank && lda >= k && ldb >= k, ST_EINVAL,
              "truncate: bad pointers or leading dimensions");
    hipStream_t st = ctx->c.stream;
    std::vector<double> ch(c, c + k);
    DevBuf cd = upload(ch, st), sd(64 * 8), outs(16 * 8);
    CoreView cv{};
    cv.nb = 1;
    cv.s[0] = cd.as<double>();
    cv.coef[0] = 1.0;
    cv.wdev[0] = nullptr;
    cv.wconst[0] = k;
    auto run = [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      Truncator<T> tr;
      tr.alloc(n, m, st);
      tr.bf16 = dtype == 2;
      BlockView<T> av = view1<T>(static_cast<const T*>(A), lda, nullptr, k);
      BlockView<T> bv = view1<T>(static_cast<const T*>(B), ldb, nullptr, k);
      int* rk = reinterpret_cast<int*>(outs.as<double>() + 2);
      tr.run(av, n, bv, m, cv, rank_cap, tol, static_cast<T*>(U), ldu, static_cast<T*>(V), ldv,
             sd.as<double>(), rk, outs.as<double>(), st);
      LRC_HIP(hipMemcpyAsync(rank, rk, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (*rank > 0)
        LRC_HIP(hipMemcpyAsync(s, sd.p, size_t(*rank) * 8, hipMemcpyDeviceToHost, st));
      int flags = 0;
      LRC_HIP(hipMemcpyAsync(&flags, tr.st.info, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (flags & 2) throw Error(ST_EBREAKDOWN, "truncate: Cholesky breakdown");
    };
    if (dtype == 0) run(static_cast<double*>(nullptr));
    else run(static_cast<float*>(nullptr));
    return LRC_OK;
  });
}

lrc_status lrc_truncate_scaled_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m, int k, int k1,
                                   const void* A, int lda, const double* c, const void* B,
                                   int ldb, const double* w_dev, int rank_cap, double tol, void* U,
                                   int ldu, double* s, void* V, int ldv, int* rank) {
  if (!ctx) return LRC_EINVAL;
  return guarded(&ctx->c, [&]() -> lrc_status {
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "truncate: dtype must be 0 or 1");
    LRC_CHECK(n >= 1 && m >= 1 && k >= 1 && k <= kTruncCap, ST_EINVAL,
              "truncate: need n, m >= 1 and 1 <= k <= 128");
    LRC_CHECK(rank_cap >= 1 && rank_cap <= 64 && rank_cap <= ldu && rank_cap <= ldv, ST_EINVAL,
              "truncate: rank_cap in [1, 64] and <= ldu, ldv");
    LRC_CHECK(A && B && c && U && V && s && rank && lda >= k && ldb >= k, ST_EINVAL,
              "truncate: bad pointers or leading dimensions");
    LRC_CHECK(w_dev && k1 >= 0 && k1 < k, ST_EINVAL, "truncate: need a row scale and 0 <= k1 < k");
    hipStream_t st = ctx->c.stream;
    std::vector<double> ch(c, c + k);
    DevBuf cd = upload(ch, st), sd(64 * 8), outs(16 * 8);
    CoreView cv{};
    cv.nb = 1;
    cv.s[0] = cd.as<double>();
    cv.coef[0] = 1.0;
    cv.wdev[0] = nullptr;
    cv.wconst[0] = k;
    auto run = [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      Truncator<T> tr;
      tr.alloc(n, m, st);
      // two blocks per side; the second block of B is row-scaled by w
      const T* a = static_cast<const T*>(A);
      const T* b = static_cast<const T*>(B);
      BlockView<T> av{}, bv{};
      av.nb = bv.nb = 2;
      av.ptr[0] = a;
      av.ptr[1] = a + k1;
      bv.ptr[0] = b;
      bv.ptr[1] = b + k1;
      av.ld[0] = av.ld[1] = lda;
      bv.ld[0] = bv.ld[1] = ldb;
      av.wconst[0] = bv.wconst[0] = av.cap[0] = bv.cap[0] = k1;
      av.wconst[1] = bv.wconst[1] = av.cap[1] = bv.cap[1] = k - k1;
      bv.rowscale[1] = w_dev;
      int* rk = reinterpret_cast<int*>(outs.as<double>() + 2);
      tr.run(av, n, bv, m, cv, rank_cap, tol, static_cast<T*>(U), ldu, static_cast<T*>(V), ldv,
             sd.as<double>(), rk, outs.as<double>(), st);
      LRC_HIP(hipMemcpyAsync(rank, rk, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (*rank > 0)
        LRC_HIP(hipMemcpyAsync(s, sd.p, size_t(*rank) * 8, hipMemcpyDeviceToHost, st));
      int flags = 0;
      LRC_HIP(hipMemcpyAsync(&flags, tr.st.info, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (flags & 2) throw Error(ST_EBREAKDOWN, "truncate: Cholesky breakdown");
    };
    if (dtype == 0) run(static_cast<double*>(nullptr));
    else run(static_cast<float*>(nullptr));
    return LRC_OK;
  });
}

lrc_status lrc_newton_subsets(lrc_ops ops, int64_t m, const double* d, int K,
                              const int64_t* sizes, const double* f, const double* x_init,
                              lrc_linearize_fn cb, void* user, double eps_newton,
                              int newton_max, int picard, int kind, const lrc_opts* opts,
                              lrc_prob* out, lrc_info* info, int64_t* sizes_out) {
  if (!ops || !opts || !out || !d) return LRC_EINVAL;
  Ops& base = ops->o;
  return guarded(base.ctx, [&]() -> lrc_status {
    LRC_CHECK(K >= 1 && K <= m, ST_EINVAL, "newton_subsets: need 1 <= K <= m");
    LRC_CHECK(cb || f, ST_EINVAL, "newton_subsets: a callback or the load vector f is required");
    LRC_CHECK(eps_newton > 0.0 && newton_max >= 1, ST_EINVAL,
              "newton_subsets: need eps_newton > 0 and newton_max >= 1");
    std::vector<int64_t> sz(K);
    if (sizes) {
      int64_t tot = 0;
      for (int k = 0; k < K; ++k) {
        LRC_CHECK(sizes[k] >= 1, ST_EINVAL, "newton_subsets: empty subset");
        sz[k] = sizes[k];
        tot += sz[k];
      }
      LRC_CHECK(tot == m, ST_EINVAL, "newton_subsets: sizes must sum to m");
    } else {
      // eq. clustering1: floor(m / K) for the first K - 1 subsets, the rest last
      for (int k = 0; k < K - 1; ++k) sz[k] = m / K;
      sz[K - 1] = m - (K - 1) * (m / K);
    }
    if (sizes_out) std::copy(sz.begin(), sz.end(), sizes_out);
    for (int k = 0; k < K; ++k) out[k] = nullptr;
    const int q = base.q;
    const int64_t n = base.n;
    constexpr int kMaxRb = 8;
    lrc_ctx_s* cx = static_cast<lrc_ctx_s*>(base.ctx->handle);
    // the point of the first median Newton iteration, then x~^{k-1}
    std::vector<double> x(n, 0.0);
    if (x_init) std::copy(x_init, x_init + n, x.begin());
    double fnrm = 0.0;
    if (f)
      for (int64_t i = 0; i < n; ++i) fnrm += f[i] * f[i];
    fnrm = std::sqrt(fnrm);
    lrc_status worst = LRC_OK;
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t mk = sz[k];
      const double* dk = d + size_t(off) * q;
      const int jmed = int(mk / 2);   // upper median (Sec. 3.3)
      // private operators for this subset's linearisation point
      std::unique_ptr<lrc_ops_s> so;
      {
        std::vector<const int64_t*> rp(q);
        std::vector<const int32_t*> cl(q);
        std::vector<const double*> vl(q);
        for (int i = 0; i < q; ++i) {
          rp[i] = base.host[i].rowptr.data();
          cl[i] = base.host[i].col.data();
          vl[i] = base.host[i].val.data();
        }
        lrc_ops tmp = nullptr;
        const lrc_status st = lrc_ops_create(cx, n, q, rp.data(), cl.data(), vl.data(), &tmp);
        if (st != LRC_OK) return st;
        so.reset(tmp);
      }
      std::vector<std::vector<double>> vals(q);
      std::vector<double*> vp(q);
      std::vector<double> BU(size_t(n) * kMaxRb), BV(size_t(mk) * kMaxRb);
      int rB = 0;
      double bnorm = 0.0;
      std::vector<double> W;
      // one linearisation at x: operator values (uploaded when changed) and
      // the right-hand side factors; returns whether the values changed
      auto linearize = [&](int stage) -> bool {
        for (int i = 0; i < q; ++i) {
          vals[i] = so->o.host[i].val;
          vp[i] = vals[i].data();
        }
        if (cb) {
          rB = 0;
          bnorm = 0.0;
          const int rc = cb(user, k, stage, x.data(), vp.data(), &rB, BU.data(), BV.data(), &bnorm);
          if (rc != 0) throw Error(ST_ECALLBACK, "newton_subsets: callback returned non-zero");
          LRC_CHECK(rB >= 1 && rB <= kMaxRb, ST_EINVAL,
                    "newton_subsets: callback right-hand side rank must be in [1, 8]");
          LRC_CHECK(std::isfinite(bnorm) && bnorm > 0.0, ST_EINVAL,
                    "newton_subsets: callback must give a positive ||b||");
        } else {
          // linear operators: B_k(x) = f 1^T - sum_i (K_i x) d_i^T (stage 0),
          // b 1^T = f 1^T (stage 1)
          bnorm = fnrm;
          std::copy(f, f + n, BU.begin());
          for (int64_t j = 0; j < mk; ++j) BV[size_t(j)] = 1.0;
          rB = 1;
          bool nz = false;
          for (int64_t i = 0; i < n && !nz; ++i) nz = x[i] != 0.0;
          if (stage == 0 && nz) {
            ops_apply_vector(so->o, x, W);
            for (int i = 0; i < q; ++i) {
              for (int64_t r = 0; r < n; ++r) BU[size_t(1 + i) * n + r] = -W[size_t(i) * n + r];
              for (int64_t j = 0; j < mk; ++j) BV[size_t(1 + i) * mk + j] = dk[size_t(j) * q + i];
            }
            rB = 1 + q;
          }
        }
        bool changed = false;
        for (int i = 0; i < q; ++i)
          if (vals[i] != so->o.host[i].val) {
            for (double v : vals[i])
              LRC_CHECK(std::isfinite(v), ST_EINVAL, "newton_subsets: non-finite operator value");
            std::copy(vals[i].begin(), vals[i].end(), so->o.host[i].val.begin());
            so->o.upload_values(i);
            changed = true;
          }
        return changed;
      };
      // a problem on the current operators with F = BU BV^T (rank rB); the
      // factorisation is carried over from `keep` unless the values changed
      std::unique_ptr<lrc_prob_s> pb;
      auto make_prob = [&](bool refactor) {
        lrc_prob tmp = nullptr;
        lrc_status st = lrc_prob_create(so.get(), mk, dk, rB, BU.data(), nullptr, BV.data(), &tmp);
        if (st != LRC_OK) throw Error(st, lrc_last_error(cx));
        std::unique_ptr<lrc_prob_s> np(tmp);
        if (refactor || !pb || !pb->p.prec) {
          st = lrc_prob_precondition(np.get(), nullptr, 0, kind);
          if (st != LRC_OK) throw Error(st, lrc_last_error(cx));
        } else {
          np->p.prec = std::move(pb->p.prec);
          np->p.seconds_setup = pb->p.seconds_setup;
        }
        pb = std::move(np);
      };
      // 1. Newton on the upper-median column from x~^{k-1}
      int steps = 0, med_iters = 0;
      bool refactor = true;
      for (;;) {
        refactor = linearize(0) || refactor;
        make_prob(refactor);
        refactor = false;
        // the median column's nonlinear residual B_k(x) e_med
        std::vector<double> r(n, 0.0);
        for (int a = 0; a < rB; ++a) {
          const double w = BV[size_t(a) * mk + jmed];
          for (int64_t i = 0; i < n; ++i) r[i] += w * BU[size_t(a) * n + i];
        }
        double rn = 0.0;
        for (double v : r) rn += v * v;
        rn = std::sqrt(rn);
        LRC_CHECK(std::isfinite(rn), ST_EINVAL, "newton_subsets: non-finite median residual");
        if (rn <= eps_newton || steps >= newton_max) break;
        std::vector<double> dx;
        int it = 0;
        median_column_solve(pb->p, r, opts->median_tol > 0 ? opts->median_tol : 1e-6,
                            opts->eager != 0, dx, &it);
        med_iters += it;
        for (int64_t i = 0; i < n; ++i) x[i] += dx[i];
        ++steps;
      }
      // 2./3. the subset's step at x~^k
      lrc_opts o = *opts;
      o.res_ref = bnorm * std::sqrt(double(mk));
      lrc_status st;
      lrc_info inf{};
      if (!picard) {
        // Newton: L(S) = B_k(x~^k), X^k = x~^k 1^T + S
        o.init = LRC_INIT_NEWTON;
        std::vector<double> ones(size_t(mk), 1.0);
        st = lrc_solve(pb.get(), &o, 1, x.data(), nullptr, ones.data(), &inf);
      } else {
        // fixed point: L_F(X) = b 1^T from zero with the stage-1 operators
        make_prob(linearize(1));
        o.init = LRC_INIT_ZERO;
        st = lrc_solve(pb.get(), &o, 0, nullptr, nullptr, nullptr, &inf);
      }
      if (st < 0) return st;
      if (st > worst) worst = st;
      inf.newton_steps = steps;
      inf.median_iters = med_iters;
      if (info) info[k] = inf;
      pb->owned_ops = std::move(so);
      out[k] = pb.release();
      off += mk;
    }
    return worst;
  });
}

}  // extern "C"
