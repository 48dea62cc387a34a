// Host runtime of libspider: contexts, catalog and network loading, device
// memory, and the per-step pipeline behind the C ABI of include/spider.h.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "index_limits.h"
#include "spider.h"

using namespace spider;

namespace {

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    // growth happens between steps: wait for work that may still use p
    if (p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  // Grow to at least n bytes (contents are not kept).
  hipError_t reserve(size_t n) { return bytes >= n ? hipSuccess : alloc(n); }
  template <typename T>
  T* as() const { return (T*)p; }
};

struct Catalog {
  int32_t M = 0, L = 0, P = 0;
  int64_t N = 0;
  uint32_t stream = 0;
  int whiten = SPIDER_WHITEN_EXACT;
  double sigma = 0, kappa = 0, prior_sigma[4] = {}, centroid_sigma[4] = {};
  // two phases: L = 2 L_p groups (station + L_p phase), stations duplicated
  int32_t L_p = 0;
  double zscale_s = 1.0;  // sigma_P^2 / sigma_S^2
  int net_s = -1;         // S-phase network (spider_set_phase_net)
  double* samples = nullptr;  // caller's sample buffer (spider_set_sample_buffer)
  int64_t sample_cap = 0;
  DevBuf hypo0, stations, pairs, w_pair, obs, inv_mean, mu_c;
  DevBuf rec;  // packed observation records (the 12-byte ones are freed after load)
  int C = 0;  // chains allocated
  DevBuf theta, v, mean, m2, steps, mcount;
  DevBuf adam_m, adam_v;      // Stage 1 optimiser moments, allocated on first use
  bool adam_zeroed = false;   // cleared by spider_reset_chains

  CatView view() const {
    CatView c;
    c.M = M;
    c.L = L;
    c.N = N;
    c.hypo0 = hypo0.as<double>();
    c.stations = stations.as<double>();
    c.pairs = pairs.as<int2>();
    c.w_pair = w_pair.as<double>();
    c.rec = rec.as<ObsRec>();
    c.inv_mean = inv_mean.as<double>();
    c.mu_c = mu_c.as<double>();
    c.stream = stream;
    c.sigma = sigma;
    c.kappa = kappa;
    c.L_p = L_p;
    c.zscale_s = zscale_s;
    for (int k = 0; k < 4; ++k) {
      c.prior_sigma[k] = prior_sigma[k];
      c.centroid_sigma[k] = centroid_sigma[k];
    }
    return c;
  }
};

struct Net {
  int D = 0, H = 0;
  double v0 = 0, center[3] = {}, half[3] = {};
  float bout = 0;
  DevBuf W0, bias, W0s, bias_s, Wt, wout;
  DevBuf pack_fwd[2], pack_bwd[2];  // by precision

  NetView view(int prec) const {
    NetView v;
    v.D = D;
    v.H = H;
    v.W0 = W0.as<float>();
    v.bias = bias.as<float>();
    v.W0s = W0s.as<float>();
    v.bias_s = bias_s.as<float>();
    v.Wt = Wt.as<float>();
    v.wout = wout.as<float>();
    v.bout = bout;
    v.v0 = v0;
    v.inv_v0 = 1.0 / v0;
    for (int a = 0; a < 3; ++a) {
      v.center[a] = center[a];
      v.half[a] = half[a];
      v.inv_half[a] = 1.0 / half[a];
    }
    v.pack_fwd = pack_fwd[prec].p;
    v.pack_bwd = pack_bwd[prec].p;
    return v;
  }
};

// Where one chain set of a fused step keeps its step scratch: offsets of its
// part of the entry-indexed solver arrays (e_off = its first entry), of the
// system lists, spill flags and scan scratch, and of the per-event gradient
// (in (chain, event) keys), reduction parts (bytes), centroid partials and
// centroids (double4 units).  Sets with disjoint parts can run side by side.
struct SetLayout {
  int64_t e_off = 0, sys_off = 0, spill_off = 0, scan_off = 0, g_off = 0, rpart_off = 0,
          partial_off = 0, tb_off = 0;
};

// Scratch of one minibatch pipeline, grown on demand.  Entry- and
// slot-indexed arrays hold every chain set of a fused step side by side
// (obs_total slots); the count and system arrays hold each set's keys and
// systems side by side; the solver scratch holds one set at a time.
struct Workspace {
  DevBuf obs, ev, sta, tau, w, start, csr, ckey, hd, pev, pgr, nend, rows, net_out, tr, gT, gT64,
      r, z, zp, wr;
  DevBuf act, sys, list, ent, vec, ivec, nrec, scan_part, bucket, phase_flags, n_p;
  DevBuf G, partial, thetabar, lp_tmp, err, rpart;
  int64_t e_cur = 0;  // entries of the last reserve: the layout of ivec

  // A second copy of what the selection and the CSR build write (and their
  // scratch), so that the next step's minibatch can be built while the
  // current step still reads its own (graph replays of sampler steps).
  struct Ahead {
    DevBuf obs, ev, sta, tau, w, start, csr, ckey, hd, pev, pgr, nend, bucket, scan_part;
    DevBuf scan_part0;  // scan scratch of a side-0 build beside the whitening's scans
  } ahead;
  hipError_t reserve_ahead(int64_t obs_total, int64_t keys_total, int64_t bucket_words) {
    const int64_t Cn = obs_total, E = 2 * obs_total;
    hipError_t e;
#define RES(buf, bytes)                                     \
  if ((e = buf.reserve((size_t)(bytes))) != hipSuccess) return e;
    RES(ahead.obs, Cn * 8);
    RES(ahead.ev, E * 4);
    RES(ahead.sta, E * 4);
    RES(ahead.tau, Cn * 8);
    RES(ahead.w, Cn * 8);
    RES(ahead.start, keys_total * 4);
    RES(ahead.csr, E * 4);
    RES(ahead.ckey, E * 8);
    RES(ahead.hd, E * 4);
    RES(ahead.pev, E * 4);
    RES(ahead.pgr, E * 4);
    RES(ahead.nend, E * 4);
    RES(ahead.bucket, bucket_words * 4);
    int64_t sp = scan_part_size(bucket_words);
    if (scan_part_size(keys_total) > sp) sp = scan_part_size(keys_total);
    RES(ahead.scan_part, sp * 4);
    RES(ahead.scan_part0, sp * 4);
#undef RES
    return hipSuccess;
  }
  // the batch buffers with the selection and CSR arrays of side 0 (the
  // usual ones) or side 1 (ahead)
  BatchBufs batch_side(int side) const {
    BatchBufs b = batch();
    if (side == 0) return b;
    b.obs = ahead.obs.as<int64_t>();
    b.ev = ahead.ev.as<int32_t>();
    b.sta = ahead.sta.as<int32_t>();
    b.tau = ahead.tau.as<double>();
    b.w = ahead.w.as<double>();
    b.start = ahead.start.as<int32_t>();
    b.csr = ahead.csr.as<int32_t>();
    b.ckey = ahead.ckey.as<uint64_t>();
    b.hd = ahead.hd.as<int32_t>();
    b.pev = ahead.pev.as<int32_t>();
    b.pgr = ahead.pgr.as<int32_t>();
    b.nend = ahead.nend.as<int32_t>();
    return b;
  }
  // CSR-build scratch of a side: side 0 outside the look-ahead branch uses
  // the common scan scratch, inside it (beside the whitening) its own
  int32_t* bucket_side(int side) const {
    return side == 0 ? bucket.as<int32_t>() : ahead.bucket.as<int32_t>();
  }
  int32_t* scan_part_side(int side, bool branch = false) const {
    return side == 1 ? ahead.scan_part.as<int32_t>()
                     : branch ? ahead.scan_part0.as<int32_t>() : scan_part.as<int32_t>();
  }

  // obs_total: slots of all sets; keys_total: sum of (C M + 1); sys_total:
  // the largest set's system-list counts (C L nb + 1); C, CM: the largest
  // set's chains and C M; bucket_words: the largest set's CSR-build buckets
  hipError_t reserve(int64_t C, int64_t obs_total, int64_t keys_total, int64_t sys_total,
                     int64_t CM, int64_t bucket_words) {
    const int64_t Cn = obs_total, E = 2 * obs_total;
    hipError_t e;
#define RES(buf, bytes)                                     \
  if ((e = buf.reserve((size_t)(bytes))) != hipSuccess) return e;
    RES(obs, Cn * 8);
    RES(ev, E * 4);
    RES(sta, E * 4);
    RES(tau, Cn * 8);
    RES(w, Cn * 8);
    RES(start, keys_total * 4);
    RES(csr, E * 4);
    RES(ckey, E * 8);
    RES(hd, E * 4);
    RES(pev, E * 4);
    RES(pgr, E * 4);
    RES(nend, E * 4);
    RES(rows, E * 4);
    RES(net_out, E * sizeof(RowOut));
    RES(tr, E * sizeof(TRec));
    RES(gT, E * 12);
    RES(gT64, E * 24);
    RES(r, Cn * 8);
    RES(z, Cn * 8);
    RES(zp, E * 8);
    RES(wr, Cn * sizeof(WRec));
    RES(act, E * 4);
    RES(sys, sys_total * 4);
    RES(list, E * 4);
    RES(ent, E * sizeof(ERec));
    RES(vec, E * 8 * 7);
    RES(ivec, E * 4 * 6 + sys_total * 4);
    RES(nrec, E * sizeof(NodeRec));
    e_cur = E;
    int64_t sp = scan_part_size(E + 1);
    if (scan_part_size(keys_total) > sp) sp = scan_part_size(keys_total);
    if (scan_part_size(sys_total) > sp) sp = scan_part_size(sys_total);
    if (scan_part_size(bucket_words) > sp) sp = scan_part_size(bucket_words);
    RES(scan_part, sp * 4);
    RES(bucket, bucket_words * 4);
    RES(phase_flags, (E + 1) * 4);
    RES(n_p, 16);
    RES(G, CM * 32);
    RES(rpart, reduce_part_bytes(2 * obs_total));
    RES(partial, (CM / 4096 + C + 1) * 32);
    RES(thetabar, C * 32);
    RES(lp_tmp, 4096 * 8);
    RES(err, 64);
#undef RES
    return hipSuccess;
  }

  BatchBufs batch() const {
    BatchBufs b;
    b.obs = obs.as<int64_t>();
    b.ev = ev.as<int32_t>();
    b.sta = sta.as<int32_t>();
    b.tau = tau.as<double>();
    b.w = w.as<double>();
    b.start = start.as<int32_t>();
    b.csr = csr.as<int32_t>();
    b.ckey = ckey.as<uint64_t>();
    b.hd = hd.as<int32_t>();
    b.pev = pev.as<int32_t>();
    b.pgr = pgr.as<int32_t>();
    b.nend = nend.as<int32_t>();
    b.rows = rows.as<int32_t>();
    b.net_out = net_out.as<RowOut>();
    b.tr = tr.as<TRec>();
    b.gT = gT.as<float>();
    b.gT64 = gT64.as<double>();
    b.r = r.as<double>();
    b.z = z.as<double>();
    b.zp = zp.as<double>();
    b.wr = wr.as<WRec>();
    return b;
  }
  // a chain set's part of the step scratch (see SetLayout)
  struct SetScratch {
    SolveBufs sv;
    double* G;
    void* rpart;
    double* partial;
    double* thetabar;
  };
  SetScratch set_scratch(const SetLayout& l) const {
    SetScratch x;
    x.sv = solve(l.sys_off);
    x.sv.act += l.e_off;
    x.sv.list += l.e_off;
    x.sv.ent += l.e_off;
    x.sv.vec += 7 * l.e_off;   // its seven arrays of its own entry count
    x.sv.ivec += 5 * l.e_off;  // its five arrays of its own entry count
    x.sv.lidx += l.e_off;
    x.sv.spill += l.spill_off;
    x.sv.nrec += l.e_off;
    x.sv.scan_part += l.scan_off;
    x.G = G.as<double>() + 4 * l.g_off;
    x.rpart = rpart.as<char>() + l.rpart_off;
    x.partial = partial.as<double>() + 4 * l.partial_off;
    x.thetabar = thetabar.as<double>() + 4 * l.tb_off;
    return x;
  }
  // grows the reduction parts and the scan scratch to the totals of the sets
  hipError_t reserve_sets(int64_t rpart_bytes, int64_t scan_ints) {
    hipError_t e = rpart.reserve((size_t)rpart_bytes);
    if (e == hipSuccess) e = scan_part.reserve((size_t)scan_ints * 4);
    return e;
  }
  SolveBufs solve(int64_t sys_off) const {
    SolveBufs v;
    v.act = act.as<int32_t>();
    v.sys = sys.as<int32_t>() + sys_off;
    v.list = list.as<int32_t>();
    v.ent = ent.as<ERec>();
    v.vec = vec.as<double>();
    v.ivec = ivec.as<int32_t>();
    v.lidx = ivec.as<int32_t>() + 5 * e_cur;
    v.spill = ivec.as<int32_t>() + 6 * e_cur;
    v.nrec = nrec.as<NodeRec>();
    v.scan_part = scan_part.as<int32_t>();
    return v;
  }
};

}  // namespace

struct spider_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool profiling = false;
  // autotuned matrix-core variant per (precision, H, D)
  std::map<std::tuple<int, int, int>, int> tuned;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  std::vector<int64_t> prof_rows;
  std::vector<std::unique_ptr<Catalog>> cats;
  std::vector<std::unique_ptr<Net>> nets;
  Workspace ws;
  RowOut* noalloc_scratch = nullptr;  // this device's copy of the static scratch array
  bool graphs = true;                 // replay sampler steps from a captured HIP graph
  hipStream_t cap_stream = nullptr;   // the stream graphs are captured on
  hipStream_t side_stream = nullptr;  // a second branch of the captured step
  hipEvent_t fork = nullptr, join = nullptr;
  // branches of the fused sets' post-network work (besides the main stream)
  hipStream_t branch[2] = {nullptr, nullptr};
  hipEvent_t bjoin[2] = {nullptr, nullptr};
};

namespace {

int fail(spider_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(spider_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? SPIDER_E_OOM : SPIDER_E_HIP, m);
}

#define HIPCK(call, what)                                 \
  do {                                                    \
    hipError_t _e = (call);                               \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

// Select the context's device for the duration of a call.  A failure here
// surfaces as the error of the call's first HIP operation.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return;
    if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
  }
};

Catalog* get_cat(spider_ctx* ctx, int32_t id) {
  if (id < 0 || id >= (int32_t)ctx->cats.size()) return nullptr;
  return ctx->cats[id].get();
}
Net* get_net(spider_ctx* ctx, int32_t id) {
  if (id < 0 || id >= (int32_t)ctx->nets.size()) return nullptr;
  return ctx->nets[id].get();
}

// Copy `bytes` from a host or device source into a device buffer.
hipError_t upload(DevBuf& dst, const void* src, size_t bytes, int mem, hipStream_t s) {
  hipError_t e = dst.alloc(bytes);
  if (e != hipSuccess) return e;
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst.p, src, bytes, mem == SPIDER_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                                     : hipMemcpyHostToDevice, s);
}

// Fetch an array from host or device memory into a host vector.
template <typename T>
hipError_t fetch(std::vector<T>& out, const T* src, size_t count, int mem, hipStream_t s) {
  out.resize(count);
  if (count == 0) return hipSuccess;
  if (mem == SPIDER_MEM_DEVICE) {
    hipError_t e = hipMemcpyAsync(out.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  std::memcpy(out.data(), src, count * sizeof(T));
  return hipSuccess;
}

constexpr int64_t kTuneRows = 1 << 16;  // tune on launches at least this large

// Matrix-core variant for this launch.  On the first launch of at least
// kTuneRows rows for a (precision, H, D), every variant is timed on these
// very rows (one warm-up and two timed launches each, HIP events on the
// context stream) and the fastest is kept for the context.  The variants
// give identical results, so tuning never changes an answer.
// SPIDER_MLP_VARIANT=<index> pins a variant (measurement runs).
int pick_variant(spider_ctx* ctx, const NetView& nv, int prec, const RowSource& src, RowOut* out,
                 const MlpVariant* vl, int nvar, int* chosen) {
  *chosen = 0;
  if (const char* env = std::getenv("SPIDER_MLP_VARIANT")) {
    const int k = std::atoi(env);
    *chosen = (k >= 0 && k < nvar) ? k : 0;
    return SPIDER_OK;
  }
  const auto key = std::make_tuple(prec, nv.H, nv.D);
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    *chosen = it->second;
    return SPIDER_OK;
  }
  if (nvar == 1 || src.rows < kTuneRows) return SPIDER_OK;
  hipEvent_t a, b;
  HIPCK(hipEventCreate(&a), "event");
  HIPCK(hipEventCreate(&b), "event");
  // one untimed launch of each variant, then two timed rounds over all of
  // them in turn, so that the clock's drift over the first launches of a run
  // does not favour the variants timed first
  std::vector<float> total(nvar, 0.0f);
  for (int k = 0; k < nvar; ++k)
    HIPCK(vl[k].launch(src, nv, out, ctx->stream), "network kernel (tuning)");
  for (int round = 0; round < 2; ++round)
    for (int k = 0; k < nvar; ++k) {
      HIPCK(hipEventRecord(a, ctx->stream), "event");
      HIPCK(vl[k].launch(src, nv, out, ctx->stream), "network kernel (tuning)");
      HIPCK(hipEventRecord(b, ctx->stream), "event");
      HIPCK(hipEventSynchronize(b), "event");
      float ms = 0.0f;
      HIPCK(hipEventElapsedTime(&ms, a, b), "event");
      total[k] += ms;
    }
  float best = 1e30f;
  for (int k = 0; k < nvar; ++k)
    if (total[k] < best) {
      best = total[k];
      *chosen = k;
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ctx->tuned[key] = *chosen;
  return SPIDER_OK;
}

// The variant a launch uses without tuning: SPIDER_MLP_VARIANT, else the
// context's tuned choice, else the first one (all give identical results).
int untuned_variant(const spider_ctx* ctx, int prec, const Net& net, int nvar) {
  if (const char* env = std::getenv("SPIDER_MLP_VARIANT")) {
    const int k = std::atoi(env);
    return (k >= 0 && k < nvar) ? k : 0;
  }
  auto it = ctx->tuned.find(std::make_tuple(prec, net.H, net.D));
  return it == ctx->tuned.end() ? 0 : it->second;
}

// Network forward/backward over the rows of src.  With may_allocate false
// the launch is never tuned or profiled (both create HIP events), so it
// enqueues the kernel and nothing else.
int run_network(spider_ctx* ctx, const Net& net, int prec, const RowSource& src, RowOut* out,
                bool may_allocate = true) {
  const NetView nv = net.view(prec);
  hipError_t e;
  const MlpVariant* vl = nullptr;
  const int nvar = mlp_variants(prec, net.H, net.D, &vl);
  int vi = 0;
  if (nvar > 0 && src.rows > 0) {
    if (may_allocate) {
      int rc = pick_variant(ctx, nv, prec, src, out, vl, nvar, &vi);
      if (rc != SPIDER_OK) return rc;
    } else {
      vi = untuned_variant(ctx, prec, net, nvar);
    }
  }
  const bool prof = ctx->profiling && may_allocate;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (prof) {
    HIPCK(hipEventCreate(&ev0), "event");
    HIPCK(hipEventCreate(&ev1), "event");
    HIPCK(hipEventRecord(ev0, ctx->stream), "event");
  }
  if (nvar > 0) {
    e = src.rows > 0 ? vl[vi].launch(src, nv, out, ctx->stream) : hipSuccess;
  } else if (prec == SPIDER_FP32) {
    e = launch_mlp_tangent(src, nv, out, ctx->stream);
  } else {
    return fail(ctx, SPIDER_E_UNSUPPORTED, "no BF16 matrix-core kernel for this network shape");
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "network kernel");
  if (prof) {
    HIPCK(hipEventRecord(ev1, ctx->stream), "event");
    ctx->prof_events.emplace_back(ev0, ev1);
    ctx->prof_rows.push_back(src.rows);
  }
  return SPIDER_OK;
}

void clear_profile(spider_ctx* ctx) {
  for (auto& pr : ctx->prof_events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  ctx->prof_events.clear();
  ctx->prof_rows.clear();
}

// The batch buffers of a chain set whose slots start at obs_off (entries and
// network rows at 2 obs_off) and whose (chain, event) counts start at key_off.
BatchBufs batch_at(const BatchBufs& b, int64_t obs_off, int64_t key_off) {
  BatchBufs o = b;
  o.obs += obs_off;
  o.tau += obs_off;
  o.w += obs_off;
  o.r += obs_off;
  o.z += obs_off;
  o.wr += obs_off;
  o.ev += 2 * obs_off;
  o.sta += 2 * obs_off;
  o.csr += 2 * obs_off;
  o.ckey += 2 * obs_off;
  o.hd += 2 * obs_off;
  o.pev += 2 * obs_off;
  o.pgr += 2 * obs_off;
  o.zp += 2 * obs_off;
  o.nend += 2 * obs_off;
  o.rows += 2 * obs_off;
  o.net_out += 2 * obs_off;
  o.tr += 2 * obs_off;
  o.gT += 6 * obs_off;
  o.gT64 += 6 * obs_off;
  o.start += key_off;
  return o;
}

// The same buffers with the residuals not kept (sampler steps read only z).
BatchBufs without_r(BatchBufs b) {
  b.r = nullptr;
  return b;
}

// The same buffers with the selected observation indices not kept (sampler
// steps use the gathered fields only).
BatchBufs without_obs(BatchBufs b) {
  b.obs = nullptr;
  return b;
}

// Before the network: the minibatch of each chain and its CSR order.
void pre_network(spider_ctx* ctx, const Catalog& cat, int C, int64_t n, const int64_t* idx,
                 uint64_t seed, const int64_t* steps_dev, int64_t step_scalar, int chain0,
                 const BatchBufs& b, int side = 0, bool branch = false) {
  Workspace& ws = ctx->ws;
  const CatView cv = cat.view();
  launch_select(cv, C, n, idx, seed, steps_dev, step_scalar, chain0, b, ws.err.as<int>(),
                ctx->stream);
  launch_build_csr(cv, C, n, b, ws.bucket_side(side), ws.scan_part_side(side, branch),
                   ctx->stream);
}

// The network's row source of a chain set: its entries in CSR order (row p
// is CSR position p: event pev[p], group pgr[p], chain p / 2n).
RowSource csr_rows(const Catalog& cat, int64_t n, int64_t E, const double* theta,
                   int64_t theta_stride, const BatchBufs& b) {
  RowSource src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  src.rows = E;
  src.ev = b.pev;
  src.sta = b.pgr;
  src.theta = theta;
  src.rows_per_chain = 2 * n;
  src.theta_chain_stride = theta_stride;
  src.stations = cat.stations.as<double>();
  return src;
}

// After the network: travel times, residuals, whitening and (if grad) the
// scaled per-event likelihood gradient into ws.G.  rows: the network's row
// order when it is not the CSR order (two-phase catalogs), else null.
int post_network(spider_ctx* ctx, const Catalog& cat, const Net& net, const Net& net_s, int prec,
                 int C, int64_t n, const double* theta, int64_t theta_stride, const int32_t* rows,
                 const BatchBufs& b, bool grad, double scale, bool l1,
                 const Workspace::SetScratch* sc = nullptr) {
  Workspace& ws = ctx->ws;
  const Workspace::SetScratch x = sc ? *sc : ws.set_scratch(SetLayout{});
  const CatView cv = cat.view();
  const int whiten = l1 ? kWhitenL1 : cat.kappa == 0.0 ? SPIDER_WHITEN_NONE : cat.whiten;
  // per-entry gradients in FP64 for the calls that return them (no gradient
  // sums); the assembly also clears the exact whitening's node flags
  launch_assemble(cv, net.view(prec), net_s.view(prec), C, n, theta, theta_stride, rows, b, !grad,
                  whiten == SPIDER_WHITEN_EXACT ? x.sv.act : nullptr, ctx->stream);
  launch_residual(cv, C, n, theta, theta_stride, whiten, b, x.sv, ctx->stream);
  if (whiten == SPIDER_WHITEN_EXACT)
    HIPCK(exact_whiten(cv, C, n, b, x.sv, ws.err.as<int>(), ctx->stream), "exact whitening");
  if (grad) launch_reduce(cv, C, n, scale, b, x.G, x.rpart, ctx->stream);
  HIPCK(hipGetLastError(), "step kernels");
  return SPIDER_OK;
}

// One minibatch for C chains: selection, network, residuals, whitening and
// (if grad) the scaled per-event likelihood gradient into ws.G.  With l1, z
// is sign(r) instead of the whitened residual (the Stage 1 loss).
int run_batch(spider_ctx* ctx, Catalog& cat, Net& net, int prec, int C, int64_t n,
              const double* theta, int64_t theta_stride, const int64_t* idx, uint64_t seed,
              const int64_t* steps_dev, int64_t step_scalar, int chain0, bool grad, double scale,
              bool l1 = false) {
  Workspace& ws = ctx->ws;
  const int64_t Cn = (int64_t)C * n, E = 2 * Cn;
  const BucketShape bs = bucket_shape(C, n, cat.M);
  if (!bs.ok) return fail(ctx, SPIDER_E_UNSUPPORTED, "chains x events too large for the CSR build");
  HIPCK(ws.reserve(C, Cn, (int64_t)C * cat.M + 1,
                   (int64_t)C * cat.L * list_blocks(C, n, cat.L) + 1, (int64_t)C * cat.M,
                   bs.words),
        "workspace");
  const BatchBufs b = ws.batch();
  pre_network(ctx, cat, C, n, idx, seed, steps_dev, step_scalar, chain0, b);
  RowSource src = csr_rows(cat, n, E, theta, theta_stride, b);
  Net* net_s = &net;
  const int32_t* rows = nullptr;
  int rc;
  if (cat.L_p < cat.L) {
    // two phases: the P rows through net and the S rows through the
    // catalog's S network, each launch over its part of the row list
    net_s = get_net(ctx, cat.net_s);
    if (!net_s)
      return fail(ctx, SPIDER_E_STATE, "two-phase catalog without an S network "
                                       "(spider_set_phase_net)");
    launch_phase_rows(cat.view(), E, b, ws.phase_flags.as<int32_t>(), ws.scan_part.as<int32_t>(),
                      ws.n_p.as<int64_t>(), ctx->stream);
    int64_t n_p = 0;
    HIPCK(hipMemcpyAsync(&n_p, ws.n_p.p, 8, hipMemcpyDeviceToHost, ctx->stream), "phase count");
    HIPCK(hipStreamSynchronize(ctx->stream), "phase count");
    rows = b.rows;
    src.mode = 3;  // rows listed by CSR position, P first
    src.list = b.rows;
    src.rows = n_p;
    rc = run_network(ctx, net, prec, src, b.net_out);
    if (rc != SPIDER_OK) return rc;
    src.list = b.rows + n_p;
    src.rows = E - n_p;
    rc = run_network(ctx, *net_s, prec, src, b.net_out + n_p);
    if (rc != SPIDER_OK) return rc;
  } else {
    rc = run_network(ctx, net, prec, src, b.net_out);
    if (rc != SPIDER_OK) return rc;
  }
  return post_network(ctx, cat, net, *net_s, prec, C, n, theta, theta_stride, rows, b, grad, scale,
                      l1);
}

// The update arguments with the catalog's sample buffer.
UpdateArgs with_samples(UpdateArgs a, const Catalog& cat) {
  a.samples = cat.samples;
  a.sample_cap = cat.samples ? cat.sample_cap : 0;
  a.sample_C = cat.C;
  return a;
}

// Chain sets that share one network and precision, advanced together: every
// set's minibatch and CSR order are built in its own slice of the workspace,
// one network launch evaluates the rows of all sets (row source mode 2), and
// the residual, whitening, per-event reduction and update of each set follow.
// The results equal those of advancing each set on its own.
struct FusedSets {
  std::vector<int64_t> obs_off;  // first slot of each set in the workspace
  std::vector<int64_t> key_off;  // first (chain, event) count of each set
  int64_t total_obs = 0;
  int64_t bucket_words = 0;      // the largest set's CSR-build buckets
  DevBuf subs, row0;             // device RowSource table and its row offsets
  DevBuf subs_ahead;             // the same over the second buffer side
  std::vector<SetLayout> lay;    // each set's part of the step scratch
  std::vector<int> branch;       // graph branch of each set's post-network work
  int n_branches = 1;
};

// Graph branches over which the post-network work of fused sets is spread
// (each a stream of its own while capturing; the hardware runs four queues).
constexpr int kPostBranches = 3;

// The network's row-source table of the fused sets over the selection and
// CSR arrays of one buffer side.
int upload_subs(spider_ctx* ctx, const spider_chainset* sets, int n_sets, const FusedSets& f,
                int side, DevBuf& dst) {
  const BatchBufs b = ctx->ws.batch_side(side);
  std::vector<RowSource> subs(n_sets);
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    const BatchBufs bk = batch_at(b, f.obs_off[k], f.key_off[k]);
    subs[k] = csr_rows(cat, sets[k].batch, 2 * (f.obs_off[k + 1] - f.obs_off[k]),
                       cat.theta.as<double>(), (int64_t)cat.M * 4, bk);
  }
  HIPCK(upload(dst, subs.data(), subs.size() * sizeof(RowSource), SPIDER_MEM_HOST, ctx->stream),
        "row sources");
  HIPCK(hipStreamSynchronize(ctx->stream), "row sources");
  return SPIDER_OK;
}

int prepare_fused(spider_ctx* ctx, const spider_chainset* sets, int n_sets, FusedSets& f) {
  int64_t sumC = 0, maxB = 1;
  f.obs_off.assign(n_sets + 1, 0);
  f.key_off.assign(n_sets + 1, 0);
  f.lay.assign(n_sets, SetLayout{});
  SetLayout end;  // the running offsets: the totals after the last set
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    const int64_t C = sets[k].n_chains, n = sets[k].batch, Cn = C * n;
    f.obs_off[k + 1] = f.obs_off[k] + Cn;
    f.key_off[k + 1] = f.key_off[k] + C * cat.M + 1;
    sumC += C;
    const int64_t S = C * cat.L * list_blocks(C, n, cat.L) + 1;
    SetLayout& l = f.lay[k];
    l = end;
    l.e_off = 2 * f.obs_off[k];
    end.sys_off += S;
    end.spill_off += C * cat.L;
    end.scan_off += scan_part_size(S);
    end.g_off += C * cat.M;
    end.rpart_off += reduce_part_bytes(2 * Cn);
    end.partial_off += C * cat.M / 4096 + C + 1;
    end.tb_off += C;
    const BucketShape bs = bucket_shape(C, n, cat.M);
    if (!bs.ok)
      return fail(ctx, SPIDER_E_UNSUPPORTED, "chains x events too large for the CSR build");
    maxB = std::max(maxB, bs.words);
  }
  f.total_obs = f.obs_off[n_sets];
  f.bucket_words = maxB;
  // post-network branches: the sets by decreasing entries, each to the
  // least loaded branch
  f.n_branches = std::min(n_sets, kPostBranches);
  f.branch.assign(n_sets, 0);
  {
    std::vector<int> order(n_sets);
    for (int k = 0; k < n_sets; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return f.obs_off[a + 1] - f.obs_off[a] > f.obs_off[b + 1] - f.obs_off[b];
    });
    std::vector<int64_t> load(f.n_branches, 0);
    for (int k : order) {
      const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      f.branch[k] = br;
      load[br] += f.obs_off[k + 1] - f.obs_off[k];
    }
  }
  Workspace& ws = ctx->ws;
  // sizes: every set's part side by side (the partial and centroid counts
  // of reserve take sum C + n_sets chains)
  HIPCK(ws.reserve(sumC + n_sets, f.total_obs, f.key_off[n_sets], end.sys_off, end.g_off, maxB),
        "workspace");
  HIPCK(ws.reserve_sets(end.rpart_off, end.scan_off), "workspace");
  const BatchBufs b = ws.batch();
  std::vector<RowSource> subs(n_sets);
  std::vector<int64_t> row0(n_sets + 1);
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    const BatchBufs bk = batch_at(b, f.obs_off[k], f.key_off[k]);
    subs[k] = csr_rows(cat, sets[k].batch, 2 * (f.obs_off[k + 1] - f.obs_off[k]),
                       cat.theta.as<double>(), (int64_t)cat.M * 4, bk);
    row0[k] = 2 * f.obs_off[k];
  }
  row0[n_sets] = 2 * f.total_obs;
  HIPCK(upload(f.subs, subs.data(), subs.size() * sizeof(RowSource), SPIDER_MEM_HOST, ctx->stream),
        "row sources");
  HIPCK(upload(f.row0, row0.data(), row0.size() * 8, SPIDER_MEM_HOST, ctx->stream), "row sources");
  HIPCK(hipStreamSynchronize(ctx->stream), "row sources");
  return SPIDER_OK;
}

int fused_step(spider_ctx* ctx, const spider_chainset* sets, int n_sets, const FusedSets& f,
               const UpdateArgs& ua) {
  Workspace& ws = ctx->ws;
  const BatchBufs b = ws.batch();
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    pre_network(ctx, cat, sets[k].n_chains, sets[k].batch, nullptr, ua.seed,
                cat.steps.as<int64_t>(), 0, 0,
                without_obs(batch_at(b, f.obs_off[k], f.key_off[k])));
  }
  RowSource src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 2;
  src.nsub = n_sets;
  src.sub = f.subs.as<RowSource>();
  src.sub_row0 = f.row0.as<int64_t>();
  src.rows = 2 * f.total_obs;
  int rc = run_network(ctx, *get_net(ctx, sets[0].net_id), sets[0].precision, src, b.net_out);
  if (rc != SPIDER_OK) return rc;
  for (int k = 0; k < n_sets; ++k) {
    const spider_chainset& st = sets[k];
    Catalog& cat = *get_cat(ctx, st.cat_id);
    const Net& net = *get_net(ctx, st.net_id);
    const int C = st.n_chains;
    const int64_t n = st.batch;
    const Workspace::SetScratch sc = ws.set_scratch(f.lay[k]);
    rc = post_network(ctx, cat, net, net, st.precision, C, n, cat.theta.as<double>(),
                      (int64_t)cat.M * 4, nullptr,
                      without_r(batch_at(b, f.obs_off[k], f.key_off[k])), true,
                      (double)cat.N / (double)n, false, &sc);
    if (rc != SPIDER_OK) return rc;
    launch_centroid(cat.theta.as<double>(), C, cat.M, sc.partial, sc.thetabar, ctx->stream);
    launch_update(cat.view(), C, cat.theta.as<double>(), cat.v.as<double>(), sc.G, sc.thetabar,
                  cat.steps.as<int64_t>(), cat.mcount.as<int64_t>(), with_samples(ua, cat),
                  cat.mean.as<double>(), cat.m2.as<double>(), ctx->stream);
    HIPCK(hipGetLastError(), "update");
  }
  return SPIDER_OK;
}

// One fused step whose selection and CSR arrays are on buffer side `side`
// (built by the previous step), which also builds the next step's on the
// other side: after the network launch, the next minibatch's selection and
// CSR build (step counter + 1) run on a second branch beside the residual,
// whitening, reduction and update of this one, and the step counters
// advance once both branches are done.  The results equal those of
// fused_step: the same kernels on the same inputs.
int fused_step_ahead(spider_ctx* ctx, const spider_chainset* sets, int n_sets, const FusedSets& f,
                     const UpdateArgs& ua, int side) {
  Workspace& ws = ctx->ws;
  const BatchBufs b = ws.batch_side(side), bn = ws.batch_side(1 - side);
  RowSource src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 2;
  src.nsub = n_sets;
  src.sub = (side == 0 ? f.subs : f.subs_ahead).as<RowSource>();
  src.sub_row0 = f.row0.as<int64_t>();
  src.rows = 2 * f.total_obs;
  int rc = run_network(ctx, *get_net(ctx, sets[0].net_id), sets[0].precision, src, b.net_out);
  if (rc != SPIDER_OK) return rc;
  // the second branch: the next step's minibatches and CSR orders
  const hipStream_t main = ctx->stream;
  HIPCK(hipEventRecord(ctx->fork, main), "fork");
  HIPCK(hipStreamWaitEvent(ctx->side_stream, ctx->fork, 0), "fork");
  ctx->stream = ctx->side_stream;
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    pre_network(ctx, cat, sets[k].n_chains, sets[k].batch, nullptr, ua.seed,
                cat.steps.as<int64_t>(), 1, 0,
                without_obs(batch_at(bn, f.obs_off[k], f.key_off[k])), 1 - side, true);
  }
  ctx->stream = main;
  const hipError_t eb = hipGetLastError();
  HIPCK(hipEventRecord(ctx->join, ctx->side_stream), "join");
  if (eb != hipSuccess) return hip_fail(ctx, eb, "next minibatch");
  // the sets' residual, whitening, reduction and update: branch 0 on the
  // main stream, the others on branch streams (each set has its own scratch)
  for (int br = 0; br < f.n_branches; ++br) {
    const hipStream_t bs = br == 0 ? main : ctx->branch[br - 1];
    if (br > 0) HIPCK(hipStreamWaitEvent(bs, ctx->fork, 0), "fork");
    ctx->stream = bs;
    for (int k = 0; k < n_sets; ++k) {
      if (f.branch[k] != br) continue;
      const spider_chainset& st = sets[k];
      Catalog& cat = *get_cat(ctx, st.cat_id);
      const Net& net = *get_net(ctx, st.net_id);
      const int C = st.n_chains;
      const int64_t n = st.batch;
      const Workspace::SetScratch sc = ws.set_scratch(f.lay[k]);
      rc = post_network(ctx, cat, net, net, st.precision, C, n, cat.theta.as<double>(),
                        (int64_t)cat.M * 4, nullptr,
                        without_r(batch_at(b, f.obs_off[k], f.key_off[k])), true,
                        (double)cat.N / (double)n, false, &sc);
      if (rc != SPIDER_OK) {
        ctx->stream = main;
        return rc;
      }
      launch_centroid(cat.theta.as<double>(), C, cat.M, sc.partial, sc.thetabar, ctx->stream);
      launch_update(cat.view(), C, cat.theta.as<double>(), cat.v.as<double>(), sc.G, sc.thetabar,
                    cat.steps.as<int64_t>(), cat.mcount.as<int64_t>(), with_samples(ua, cat),
                    cat.mean.as<double>(), cat.m2.as<double>(), ctx->stream, false);
    }
    ctx->stream = main;
    const hipError_t eu = hipGetLastError();
    if (eu != hipSuccess) return hip_fail(ctx, eu, "update");
    if (br > 0) {
      HIPCK(hipEventRecord(ctx->bjoin[br - 1], bs), "join");
      HIPCK(hipStreamWaitEvent(main, ctx->bjoin[br - 1], 0), "join");
    }
  }
  HIPCK(hipStreamWaitEvent(ctx->stream, ctx->join, 0), "join");
  for (int k = 0; k < n_sets; ++k) {
    Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    launch_advance(sets[k].n_chains, cat.steps.as<int64_t>(), cat.mcount.as<int64_t>(), ua,
                   ctx->stream);
  }
  HIPCK(hipGetLastError(), "advance");
  return SPIDER_OK;
}

// Captures fused_step_ahead(side) on the context's capture stream.
int capture_ahead(spider_ctx* ctx, const spider_chainset* sets, int n_sets, const FusedSets& f,
                  const UpdateArgs& ua, int side, hipGraphExec_t* out) {
  const hipStream_t main = ctx->stream;
  ctx->stream = ctx->cap_stream;
  hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    ctx->stream = main;
    return hip_fail(ctx, e, "graph capture");
  }
  const int rc = fused_step_ahead(ctx, sets, n_sets, f, ua, side);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(ctx->cap_stream, &g);
  ctx->stream = main;
  if (rc != SPIDER_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != SPIDER_OK ? rc : hip_fail(ctx, e, "graph capture");
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(ctx, e, "graph instantiate");
  return SPIDER_OK;
}

// n fused steps replayed from HIP graphs, launched on the context's stream.
// The minibatch of the first replayed step is built eagerly on buffer side
// 1; then two graphs alternate: the one for side s runs the step on side s
// and builds the next minibatch on side 1 - s (fused_step_ahead).  Every
// kernel reads the chains' step counters on the device, so each replay is
// the next step; a step holds no host synchronisation, allocation or memset.
int graph_steps(spider_ctx* ctx, const spider_chainset* sets, int n_sets, FusedSets& f,
                const UpdateArgs& ua, int64_t n) {
  if (n <= 0) return SPIDER_OK;
  if (!ctx->cap_stream)
    HIPCK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "capture stream");
  if (!ctx->side_stream)
    HIPCK(hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking), "side stream");
  if (!ctx->fork) HIPCK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming), "fork event");
  if (!ctx->join) HIPCK(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming), "join event");
  for (int k = 0; k + 1 < kPostBranches; ++k) {
    if (!ctx->branch[k])
      HIPCK(hipStreamCreateWithFlags(&ctx->branch[k], hipStreamNonBlocking), "branch stream");
    if (!ctx->bjoin[k])
      HIPCK(hipEventCreateWithFlags(&ctx->bjoin[k], hipEventDisableTiming), "branch event");
  }
  Workspace& ws = ctx->ws;
  HIPCK(ws.reserve_ahead(f.total_obs, f.key_off[n_sets], f.bucket_words), "workspace");
  int rc = upload_subs(ctx, sets, n_sets, f, 1, f.subs_ahead);
  if (rc) return rc;
  // the first replayed step's minibatch, on side 1
  const BatchBufs b1 = ws.batch_side(1);
  for (int k = 0; k < n_sets; ++k) {
    const Catalog& cat = *get_cat(ctx, sets[k].cat_id);
    pre_network(ctx, cat, sets[k].n_chains, sets[k].batch, nullptr, ua.seed,
                cat.steps.as<int64_t>(), 0, 0,
                without_obs(batch_at(b1, f.obs_off[k], f.key_off[k])), 1);
  }
  HIPCK(hipGetLastError(), "next minibatch");
  hipGraphExec_t x[2] = {nullptr, nullptr};
  rc = capture_ahead(ctx, sets, n_sets, f, ua, 1, &x[1]);
  if (rc == SPIDER_OK) rc = capture_ahead(ctx, sets, n_sets, f, ua, 0, &x[0]);
  hipError_t e = hipSuccess;
  if (rc == SPIDER_OK)
    for (int64_t t = 0; t < n && e == hipSuccess; ++t) e = hipGraphLaunch(x[t % 2 == 0 ? 1 : 0], ctx->stream);
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  for (int k = 0; k < 2; ++k)
    if (x[k]) (void)hipGraphExecDestroy(x[k]);
  if (rc != SPIDER_OK) return rc;
  if (e != hipSuccess) return hip_fail(ctx, e, "graph launch");
  if (es != hipSuccess) return hip_fail(ctx, es, "graph steps");
  return SPIDER_OK;
}

int check_select_flag(spider_ctx* ctx) {
  int flag = 0;
  HIPCK(hipMemcpyAsync(&flag, ctx->ws.err.as<int>(), sizeof(int), hipMemcpyDeviceToHost,
                       ctx->stream),
        "read flag");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  if (flag & kErrSelect)
    return fail(ctx, SPIDER_E_INVALID,
                "observation index out of range (or the minibatch permutation walk failed)");
  if (flag & kErrSolve)
    return fail(ctx, SPIDER_E_NUMERIC,
                "exact whitening: the CG solve of a cyclic core stayed above 1e-8 relative "
                "residual after 200 iterations");
  return SPIDER_OK;
}

int reset_err_flag(spider_ctx* ctx) {
  HIPCK(ctx->ws.err.reserve(64), "workspace");
  HIPCK(hipMemsetAsync(ctx->ws.err.p, 0, sizeof(int), ctx->stream), "flag reset");
  return SPIDER_OK;
}

// ---- scratch of the allocation-free travel-time call
// The network kernel's per-row outputs for spider_travel_time_noalloc, at
// most SPIDER_NOALLOC_MAX_ROWS rows (16 MiB).  Every device the library runs
// on holds its own copy of this array until the process ends.  In host code
// the name `scratch` is only a host-side stand-in: kernels are given the
// device address that hipGetSymbolAddress returns for the current device
// (kept per device in g_scratch by noalloc_setup), never the name itself.
static __device__ __align__(256) RowOut scratch[SPIDER_NOALLOC_MAX_ROWS];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
RowOut* g_scratch[kMaxScratchDevices] = {};

// Resolves this device's copy of `scratch` once per device; the device must
// be current.
hipError_t noalloc_setup(int device, RowOut** out) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = (RowOut*)p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

// T and dT/dx (or vjp_w dT/dx) of explicit rows: the network kernel into
// the RowOut buffer `net_out`, then the FP64 assembly.
int travel_time_rows(spider_ctx* ctx, Net& net, int32_t precision, const double* x_src,
                     const double* s, int64_t rows, RowOut* net_out, bool may_allocate,
                     double* T, double* gradT, const double* vjp_w) {
  RowSource src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 1;
  src.rows = rows;
  src.x = x_src;
  src.s = s;
  int rc = run_network(ctx, net, precision, src, net_out, may_allocate);
  if (rc != SPIDER_OK) return rc;
  launch_tt_assemble(net.view(precision), rows, x_src, s, net_out, T, gradT, vjp_w, ctx->stream);
  HIPCK(hipGetLastError(), "travel time");
  return SPIDER_OK;
}

// Common checks of the travel-time calls; *skip is set when rows == 0.
int travel_time_args(spider_ctx* ctx, int32_t net_id, int32_t precision, int64_t rows,
                     Net** net, bool* skip) {
  *net = get_net(ctx, net_id);
  *skip = false;
  if (!*net) return fail(ctx, SPIDER_E_INVALID, "unknown network id");
  if (precision != SPIDER_FP32 && precision != SPIDER_BF16)
    return fail(ctx, SPIDER_E_INVALID, "unknown precision");
  if (rows < 0) return fail(ctx, SPIDER_E_INVALID, "rows < 0");
  *skip = rows == 0;
  return SPIDER_OK;
}

}  // namespace

extern "C" {

int spider_version(void) { return 100; }

int spider_create(spider_ctx** out, int device, void* hip_stream) {
  if (!out) return SPIDER_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SPIDER_E_INVALID;
  RowOut* scr = nullptr;
  {
    DeviceGuard g(device);
    if (noalloc_setup(device, &scr) != hipSuccess) return SPIDER_E_HIP;
  }
  auto* ctx = new (std::nothrow) spider_ctx();
  if (!ctx) return SPIDER_E_OOM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->noalloc_scratch = scr;
  *out = ctx;
  return SPIDER_OK;
}

void spider_destroy(spider_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  clear_profile(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->side_stream) (void)hipStreamDestroy(ctx->side_stream);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  for (int k = 0; k < 2; ++k) {
    if (ctx->branch[k]) (void)hipStreamDestroy(ctx->branch[k]);
    if (ctx->bjoin[k]) (void)hipEventDestroy(ctx->bjoin[k]);
  }
  delete ctx;
}

int spider_set_graphs(spider_ctx* ctx, int enable) {
  if (!ctx) return SPIDER_E_INVALID;
  ctx->graphs = enable != 0;
  return SPIDER_OK;
}

int spider_profile(spider_ctx* ctx, int enable) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  clear_profile(ctx);
  ctx->profiling = enable != 0;
  return SPIDER_OK;
}

int spider_network_variant(spider_ctx* ctx, int32_t net_id, int32_t precision, int32_t* waves,
                           int32_t* row_tiles, int32_t* schedule) {
  if (!ctx) return SPIDER_E_INVALID;
  Net* net = get_net(ctx, net_id);
  if (!net) return fail(ctx, SPIDER_E_INVALID, "unknown network id");
  const MlpVariant* vl = nullptr;
  const int nvar = mlp_variants(precision, net->H, net->D, &vl);
  int32_t w = 0, r = 0, sc = 0;
  if (nvar > 0) {
    auto it = ctx->tuned.find(std::make_tuple((int)precision, net->H, net->D));
    int k = it == ctx->tuned.end() ? 0 : it->second;
    if (const char* env = std::getenv("SPIDER_MLP_VARIANT")) {
      const int e = std::atoi(env);
      k = (e >= 0 && e < nvar) ? e : 0;
    }
    w = vl[k].nw;
    r = vl[k].rt;
    sc = vl[k].schedule;
  }
  if (waves) *waves = w;
  if (row_tiles) *row_tiles = r;
  if (schedule) *schedule = sc;
  return SPIDER_OK;
}

int spider_profile_read(spider_ctx* ctx, double* ms, int64_t* launches, int64_t* rows) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  double tot = 0.0;
  int64_t nr = 0;
  for (size_t k = 0; k < ctx->prof_events.size(); ++k) {
    float t = 0.0f;
    HIPCK(hipEventElapsedTime(&t, ctx->prof_events[k].first, ctx->prof_events[k].second),
          "event time");
    tot += t;
    nr += ctx->prof_rows[k];
  }
  if (ms) *ms = tot;
  if (launches) *launches = (int64_t)ctx->prof_events.size();
  if (rows) *rows = nr;
  return SPIDER_OK;
}

const char* spider_last_error(const spider_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int spider_sync(spider_ctx* ctx) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  HIPCK(hipStreamSynchronize(ctx->stream), "stream synchronize");
  return SPIDER_OK;
}

int spider_load_catalog(spider_ctx* ctx, const spider_catalog_desc* d, int32_t* cat_id) {
  if (!ctx || !d || !cat_id) return fail(ctx, SPIDER_E_INVALID, "null argument");
  DeviceGuard g(ctx->device);
  if (d->M < 2 || d->L < 1 || d->P < 1 || d->N < 1)
    return fail(ctx, SPIDER_E_INVALID, "need M >= 2, L >= 1, P >= 1, N >= 1");
  if (d->N > (int64_t)INT32_MAX * 2 || (int64_t)d->M * 4 > INT32_MAX)
    return fail(ctx, SPIDER_E_UNSUPPORTED, "catalog too large");
  if (d->mem != SPIDER_MEM_HOST && d->mem != SPIDER_MEM_DEVICE)
    return fail(ctx, SPIDER_E_INVALID, "mem must be SPIDER_MEM_HOST or SPIDER_MEM_DEVICE");
  if (!d->hypo0 || !d->stations || !d->pair_i || !d->pair_j || !d->obs_pair || !d->obs_sta ||
      !d->obs_dt)
    return fail(ctx, SPIDER_E_INVALID, "null catalog array");
  if (!(d->sigma > 0) || !(d->kappa >= 0) || !(d->ell > 0) || !(d->eps_w > 0) ||
      !std::isfinite(d->p) || !std::isfinite(d->kappa))
    return fail(ctx, SPIDER_E_INVALID, "need sigma > 0, kappa >= 0, ell > 0, eps_w > 0, finite p");
  for (int k = 0; k < 4; ++k)
    if (!(d->prior_sigma[k] > 0) || !(d->centroid_sigma[k] > 0) ||
        !std::isfinite(d->prior_sigma[k]) || !std::isfinite(d->centroid_sigma[k]))
      return fail(ctx, SPIDER_E_INVALID, "prior and centroid s.d. must be positive and finite");
  if (d->stream >= (1u << 24)) return fail(ctx, SPIDER_E_INVALID, "stream id must be < 2^24");
  if (d->whiten < SPIDER_WHITEN_NONE || d->whiten > SPIDER_WHITEN_EXACT)
    return fail(ctx, SPIDER_E_INVALID, "unknown whitening mode");
  std::vector<int8_t> phase;
  bool two_phase = false;
  if (d->obs_phase) {
    HIPCK(fetch(phase, d->obs_phase, d->N, d->mem, ctx->stream), "read obs_phase");
    for (int8_t ph : phase) {
      if (ph != 0 && ph != 1) return fail(ctx, SPIDER_E_INVALID, "phase must be 0 (P) or 1 (S)");
      two_phase |= ph == 1;
    }
  }
  if (two_phase && (!(d->sigma_s > 0) || !(d->kappa_s >= 0) || !std::isfinite(d->sigma_s) ||
                    !std::isfinite(d->kappa_s) || (d->kappa_s > 0) != (d->kappa > 0)))
    return fail(ctx, SPIDER_E_INVALID,
                "need sigma_s > 0, kappa_s >= 0, and kappa_s > 0 exactly when kappa > 0");
  const int32_t Lg = two_phase ? 2 * d->L : d->L;  // station-phase groups
  if (Lg > kMaxGroups)
    return fail(ctx, SPIDER_E_UNSUPPORTED, "more than 40,960 station-phase groups");

  auto cat = std::make_unique<Catalog>();
  cat->M = d->M;
  cat->L = Lg;
  cat->L_p = d->L;
  if (two_phase) cat->zscale_s = (d->sigma * d->sigma) / (d->sigma_s * d->sigma_s);
  cat->P = d->P;
  cat->N = d->N;
  cat->stream = d->stream;
  cat->whiten = d->whiten;
  cat->sigma = d->sigma;
  cat->kappa = d->kappa;
  for (int k = 0; k < 4; ++k) {
    cat->prior_sigma[k] = d->prior_sigma[k];
    cat->centroid_sigma[k] = d->centroid_sigma[k];
  }
  hipStream_t s = ctx->stream;
  HIPCK(upload(cat->hypo0, d->hypo0, (size_t)d->M * 32, d->mem, s), "upload hypo0");
  if (two_phase) {  // the S groups' rows of the station table repeat the P ones
    std::vector<double> st;
    HIPCK(fetch(st, d->stations, (size_t)d->L * 3, d->mem, s), "read stations");
    st.insert(st.end(), st.begin(), st.end());
    HIPCK(upload(cat->stations, st.data(), st.size() * 8, SPIDER_MEM_HOST, s), "upload stations");
    HIPCK(hipStreamSynchronize(s), "sync");
  } else {
    HIPCK(upload(cat->stations, d->stations, (size_t)d->L * 24, d->mem, s), "upload stations");
  }

  // pairs and observations are re-packed on the host (12-byte records)
  {
    std::vector<int32_t> pi, pj;
    HIPCK(fetch(pi, d->pair_i, d->P, d->mem, s), "read pair_i");
    HIPCK(fetch(pj, d->pair_j, d->P, d->mem, s), "read pair_j");
    std::vector<int2> pairs(d->P);
    for (int32_t e = 0; e < d->P; ++e) pairs[e] = make_int2(pi[e], pj[e]);
    HIPCK(upload(cat->pairs, pairs.data(), pairs.size() * sizeof(int2), SPIDER_MEM_HOST, s),
          "upload pairs");
    HIPCK(hipStreamSynchronize(s), "sync");
  }
  {
    std::vector<int32_t> op;
    std::vector<int16_t> os;
    std::vector<float> od;
    HIPCK(fetch(op, d->obs_pair, d->N, d->mem, s), "read obs_pair");
    HIPCK(fetch(os, d->obs_sta, d->N, d->mem, s), "read obs_sta");
    HIPCK(fetch(od, d->obs_dt, d->N, d->mem, s), "read obs_dt");
    std::vector<Obs> obs(d->N);
    for (int64_t q = 0; q < d->N; ++q) obs[q] = Obs{op[q], od[q], (int32_t)os[q]};
    if (two_phase)
      for (int64_t q = 0; q < d->N; ++q) {
        if (os[q] < 0 || os[q] >= d->L)
          return fail(ctx, SPIDER_E_INVALID, "event, pair or station id out of range, or i == j");
        obs[q].sta += d->L * phase[q];
      }
    HIPCK(upload(cat->obs, obs.data(), obs.size() * sizeof(Obs), SPIDER_MEM_HOST, s),
          "upload observations");
    HIPCK(hipStreamSynchronize(s), "sync");
  }
  // validation on the device
  DevBuf bad;
  HIPCK(bad.alloc(16), "alloc");
  HIPCK(hipMemsetAsync(bad.p, 0, 16, s), "memset");
  launch_validate(cat->hypo0.as<double>(), d->M, cat->stations.as<double>(), Lg,
                  cat->pairs.as<int2>(), d->P, cat->obs.as<Obs>(), d->N, bad.as<int>(), s);
  int flag = 0;
  HIPCK(hipMemcpyAsync(&flag, bad.p, sizeof(int), hipMemcpyDeviceToHost, s), "read flag");
  HIPCK(hipStreamSynchronize(s), "validate");
  if (flag & 1) return fail(ctx, SPIDER_E_INVALID, "event, pair or station id out of range, or i == j");
  if (flag & 2) return fail(ctx, SPIDER_E_INVALID, "non-finite coordinate or observation");
  if (flag & 4) return fail(ctx, SPIDER_E_INVALID, "an initial source lies within 1e-3 km of its station");

  HIPCK(cat->w_pair.alloc((size_t)d->P * 8), "alloc w_pair");
  HIPCK(cat->inv_mean.alloc((size_t)Lg * 8), "alloc inv_mean");
  HIPCK(cat->mu_c.alloc(32), "alloc mu_c");
  launch_pair_weights(cat->hypo0.as<double>(), cat->pairs.as<int2>(), d->P, d->ell, d->p, d->eps_w,
                      cat->w_pair.as<double>(), s);
  HIPCK(group_inverse_mean(cat->obs.as<Obs>(), d->N, Lg, cat->w_pair.as<double>(),
                           cat->inv_mean.as<double>(), s),
        "group means");
  if (two_phase && d->kappa > 0) {
    // Sigma_g of an S group = (sigma_S^2 / sigma_P^2) times the P-phase form
    // sigma_P^2 I + kappa_P^2 W'^1/2 A A^T W'^1/2 with W' = rho W: the S
    // weights carry rho, and z of an S row is scaled by sigma_P^2 / sigma_S^2
    const double rho = (d->kappa_s * d->kappa_s * d->sigma * d->sigma) /
                       (d->sigma_s * d->sigma_s * d->kappa * d->kappa);
    std::vector<double> im(Lg);
    HIPCK(hipMemcpyAsync(im.data(), cat->inv_mean.p, (size_t)Lg * 8, hipMemcpyDeviceToHost, s),
          "read group means");
    HIPCK(hipStreamSynchronize(s), "sync");
    for (int32_t g2 = d->L; g2 < Lg; ++g2) im[g2] *= rho;
    HIPCK(hipMemcpyAsync(cat->inv_mean.p, im.data(), (size_t)Lg * 8, hipMemcpyHostToDevice, s),
          "write group means");
    HIPCK(hipStreamSynchronize(s), "sync");
  }
  launch_mean4(cat->hypo0.as<double>(), d->M, cat->mu_c.as<double>(), s);
  HIPCK(cat->rec.alloc((size_t)d->N * sizeof(ObsRec)), "alloc observation records");
  launch_pack_obs(cat->obs.as<Obs>(), d->N, cat->pairs.as<int2>(), cat->w_pair.as<double>(),
                  cat->inv_mean.as<double>(), cat->rec.as<ObsRec>(), s);
  HIPCK(hipGetLastError(), "load kernels");
  HIPCK(hipStreamSynchronize(s), "load");
  cat->obs.release();
  ctx->cats.push_back(std::move(cat));
  *cat_id = (int32_t)ctx->cats.size() - 1;
  return SPIDER_OK;
}

int spider_set_phase_net(spider_ctx* ctx, int32_t cat_id, int32_t net_id) {
  if (!ctx) return SPIDER_E_INVALID;
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat || !get_net(ctx, net_id))
    return fail(ctx, SPIDER_E_INVALID, "unknown catalog or network id");
  cat->net_s = net_id;
  return SPIDER_OK;
}

int spider_load_net(spider_ctx* ctx, const spider_net_desc* d, int32_t* net_id) {
  if (!ctx || !d || !net_id) return fail(ctx, SPIDER_E_INVALID, "null argument");
  DeviceGuard g(ctx->device);
  const int D = d->D, H = d->H;
  if (D < 1 || D > SPIDER_MAX_LAYERS || H < 16 || H > 256 || H % 16 != 0)
    return fail(ctx, SPIDER_E_INVALID, "need 1 <= D <= 16 and H a multiple of 16 in [16, 256]");
  if (!(d->v0 > 0)) return fail(ctx, SPIDER_E_INVALID, "v0 must be positive");
  for (int a = 0; a < 3; ++a)
    if (!(d->half_extent[a] > 0) || !std::isfinite(d->center[a]))
      return fail(ctx, SPIDER_E_INVALID, "half extents must be positive, centre finite");
  for (int l = 0; l <= D; ++l)
    if (!d->W[l] || !d->b[l]) return fail(ctx, SPIDER_E_INVALID, "null weight or bias");
  hipStream_t s = ctx->stream;
  std::vector<std::vector<float>> W(D + 1), B(D + 1);
  for (int l = 0; l <= D; ++l) {
    const size_t wn = l == 0 ? (size_t)H * 6 : (l == D ? (size_t)H : (size_t)H * H);
    const size_t bn = l == D ? 1 : (size_t)H;
    HIPCK(fetch(W[l], d->W[l], wn, d->mem, s), "read weights");
    HIPCK(fetch(B[l], d->b[l], bn, d->mem, s), "read biases");
    for (float x : W[l])
      if (!std::isfinite(x)) return fail(ctx, SPIDER_E_INVALID, "non-finite weight");
    for (float x : B[l])
      if (!std::isfinite(x)) return fail(ctx, SPIDER_E_INVALID, "non-finite bias");
  }
  auto net = std::make_unique<Net>();
  net->D = D;
  net->H = H;
  net->v0 = d->v0;
  for (int a = 0; a < 3; ++a) {
    net->center[a] = d->center[a];
    net->half[a] = d->half_extent[a];
  }
  net->bout = B[D][0];
  std::vector<float> bias((size_t)D * H), wt((size_t)std::max(D - 1, 1) * H * H, 0.0f);
  for (int l = 0; l < D; ++l) std::memcpy(&bias[(size_t)l * H], B[l].data(), H * 4);
  for (int l = 1; l < D; ++l)
    for (int n = 0; n < H; ++n)
      for (int k = 0; k < H; ++k) wt[((size_t)(l - 1) * H + k) * H + n] = W[l][(size_t)n * H + k];
  HIPCK(upload(net->W0, W[0].data(), (size_t)H * 6 * 4, SPIDER_MEM_HOST, s), "upload W0");
  HIPCK(upload(net->bias, bias.data(), bias.size() * 4, SPIDER_MEM_HOST, s), "upload biases");
  std::vector<float> w0s(W[0].size()), bias_s(bias.size());
  for (size_t i = 0; i < w0s.size(); ++i) w0s[i] = (float)(kTanhScale * (double)W[0][i]);
  for (size_t i = 0; i < bias_s.size(); ++i) bias_s[i] = (float)(kTanhScale * (double)bias[i]);
  HIPCK(upload(net->W0s, w0s.data(), w0s.size() * 4, SPIDER_MEM_HOST, s), "upload W0");
  HIPCK(upload(net->bias_s, bias_s.data(), bias_s.size() * 4, SPIDER_MEM_HOST, s), "upload biases");
  HIPCK(upload(net->Wt, wt.data(), wt.size() * 4, SPIDER_MEM_HOST, s), "upload hidden weights");
  HIPCK(upload(net->wout, W[D].data(), (size_t)H * 4, SPIDER_MEM_HOST, s), "upload output row");
  for (int prec = 0; prec < 2; ++prec) {
    if (!mlp_mfma_supported(prec, H, D)) continue;
    const size_t lb = mfma_pack_bytes(prec, H);
    const size_t layers = (size_t)std::max(D - 1, 1);
    std::vector<unsigned char> fwd(lb * layers), bwd(lb * layers);
    for (int l = 1; l < D; ++l)
      mfma_pack_layer(prec, H, W[l].data(), fwd.data() + lb * (l - 1), bwd.data() + lb * (l - 1));
    HIPCK(upload(net->pack_fwd[prec], fwd.data(), fwd.size(), SPIDER_MEM_HOST, s), "upload pack");
    HIPCK(upload(net->pack_bwd[prec], bwd.data(), bwd.size(), SPIDER_MEM_HOST, s), "upload pack");
  }
  HIPCK(hipStreamSynchronize(s), "load net");
  ctx->nets.push_back(std::move(net));
  *net_id = (int32_t)ctx->nets.size() - 1;
  return SPIDER_OK;
}

int spider_travel_time(spider_ctx* ctx, int32_t net_id, int32_t precision, const double* x_src,
                       const double* s, int64_t rows, double* T, double* gradT) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Net* net;
  bool skip;
  int rc = travel_time_args(ctx, net_id, precision, rows, &net, &skip);
  if (rc != SPIDER_OK || skip) return rc;
  if (!x_src || !s || !T) return fail(ctx, SPIDER_E_INVALID, "null array");
  HIPCK(ctx->ws.net_out.reserve((size_t)rows * sizeof(RowOut)), "workspace");
  return travel_time_rows(ctx, *net, precision, x_src, s, rows, ctx->ws.net_out.as<RowOut>(), true,
                          T, gradT, nullptr);
}

int spider_tt_forward(spider_ctx* ctx, int32_t net_id, int32_t precision, const double* x_src,
                      const double* s, int64_t rows, double* T) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Net* net;
  bool skip;
  int rc = travel_time_args(ctx, net_id, precision, rows, &net, &skip);
  if (rc != SPIDER_OK || skip) return rc;
  if (!x_src || !s || !T) return fail(ctx, SPIDER_E_INVALID, "null array");
  HIPCK(ctx->ws.net_out.reserve((size_t)rows * sizeof(RowOut)), "workspace");
  return travel_time_rows(ctx, *net, precision, x_src, s, rows, ctx->ws.net_out.as<RowOut>(), true,
                          T, nullptr, nullptr);
}

int spider_tt_backward(spider_ctx* ctx, int32_t net_id, int32_t precision, const double* x_src,
                       const double* s, const double* grad_T, int64_t rows, double* grad_x) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Net* net;
  bool skip;
  int rc = travel_time_args(ctx, net_id, precision, rows, &net, &skip);
  if (rc != SPIDER_OK || skip) return rc;
  if (!x_src || !s || !grad_T || !grad_x) return fail(ctx, SPIDER_E_INVALID, "null array");
  HIPCK(ctx->ws.net_out.reserve((size_t)rows * sizeof(RowOut)), "workspace");
  return travel_time_rows(ctx, *net, precision, x_src, s, rows, ctx->ws.net_out.as<RowOut>(), true,
                          nullptr, grad_x, grad_T);
}

int spider_travel_time_noalloc(spider_ctx* ctx, int32_t net_id, int32_t precision,
                               const double* x_src, const double* s, int64_t rows, double* T,
                               double* gradT) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Net* net;
  bool skip;
  int rc = travel_time_args(ctx, net_id, precision, rows, &net, &skip);
  if (rc != SPIDER_OK || skip) return rc;
  if (rows > SPIDER_NOALLOC_MAX_ROWS)
    return fail(ctx, SPIDER_E_INVALID,
                "rows exceeds SPIDER_NOALLOC_MAX_ROWS (1048576), the allocation-free scratch");
  if (!x_src || !s || !T) return fail(ctx, SPIDER_E_INVALID, "null array");
  if (!ctx->noalloc_scratch) return fail(ctx, SPIDER_E_STATE, "no scratch array on this device");
  // every row of the scratch that the assembly reads is written by the
  // network kernel first: nothing has to start at zero
  return travel_time_rows(ctx, *net, precision, x_src, s, rows, ctx->noalloc_scratch, false, T,
                          gradT, nullptr);
}

static int grad_common(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                       const double* theta, const int64_t* batch_idx, int64_t n, uint64_t seed,
                       int32_t chain, int64_t step, bool grad, Catalog** cat_out, Net** net_out,
                       bool l1 = false) {
  Catalog* cat = get_cat(ctx, cat_id);
  Net* net = get_net(ctx, net_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (!net) return fail(ctx, SPIDER_E_INVALID, "unknown network id");
  if (precision != SPIDER_FP32 && precision != SPIDER_BF16)
    return fail(ctx, SPIDER_E_INVALID, "unknown precision");
  if (!theta) return fail(ctx, SPIDER_E_INVALID, "null theta");
  if (n < 1) return fail(ctx, SPIDER_E_INVALID, "n must be >= 1");
  if (!batch_idx && n > cat->N) return fail(ctx, SPIDER_E_INVALID, "n > N");
  if (!entries_fit(1, n))
    return fail(ctx, SPIDER_E_UNSUPPORTED, "minibatch above 2^30 - 1 observations");
  if (chain < 0 || step < 0) return fail(ctx, SPIDER_E_INVALID, "chain and step must be >= 0");
  int rc = reset_err_flag(ctx);
  if (rc) return rc;
  rc = run_batch(ctx, *cat, *net, precision, 1, n, theta, (int64_t)cat->M * 4, batch_idx, seed,
                 nullptr, step, chain, grad, l1 ? 1.0 / (double)n : (double)cat->N / (double)n, l1);
  if (rc) return rc;
  *cat_out = cat;
  *net_out = net;
  return SPIDER_OK;
}

int spider_grad(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                const double* theta, const int64_t* batch_idx, int64_t n, uint64_t seed,
                int32_t chain, int64_t step, uint32_t flags, double* grad_out,
                double* logpost_out) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!grad_out) return fail(ctx, SPIDER_E_INVALID, "null grad_out");
  Catalog* cat;
  Net* net;
  if (flags & ~(uint32_t)(SPIDER_GRAD_PRIOR | SPIDER_GRAD_CENTROID | SPIDER_GRAD_L1))
    return fail(ctx, SPIDER_E_INVALID, "unknown gradient flags");
  const bool l1 = (flags & SPIDER_GRAD_L1) != 0;
  int rc = grad_common(ctx, cat_id, net_id, precision, theta, batch_idx, n, seed, chain, step,
                       true, &cat, &net, l1);
  if (rc) return rc;
  Workspace& ws = ctx->ws;
  const CatView cv = cat->view();
  launch_centroid(theta, 1, cat->M, ws.partial.as<double>(), ws.thetabar.as<double>(), ctx->stream);
  launch_grad_finish(cv, theta, ws.G.as<double>(), ws.thetabar.as<double>(), flags, grad_out,
                     ctx->stream);
  // L1: -(1/n) sum |r| = -(scale/2) r.z with z = sign(r) and scale = 2/n
  if (logpost_out) launch_obs_z(n, ws.batch(), ctx->stream);
  if (logpost_out)
    launch_logpost(cv, n, l1 ? 2.0 / (double)n : (double)cat->N / (double)n, ws.r.as<double>(),
                   ws.z.as<double>(), theta, ws.thetabar.as<double>(), flags,
                   ws.lp_tmp.as<double>(), logpost_out, ctx->stream);
  HIPCK(hipGetLastError(), "gradient kernels");
  return check_select_flag(ctx);
}

int spider_batch_terms(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                       const double* theta, const int64_t* batch_idx, int64_t n, uint64_t seed,
                       int32_t chain, int64_t step, double* T_i, double* T_j, double* gT_i,
                       double* gT_j, double* r, double* z) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat;
  Net* net;
  int rc = grad_common(ctx, cat_id, net_id, precision, theta, batch_idx, n, seed, chain, step,
                       false, &cat, &net);
  if (rc) return rc;
  launch_batch_terms_out(n, ctx->ws.batch(), theta, T_i, T_j, gT_i, gT_j, r, z, ctx->stream);
  HIPCK(hipGetLastError(), "batch terms");
  return check_select_flag(ctx);
}

int spider_batch_indices(spider_ctx* ctx, int32_t cat_id, uint64_t seed, int32_t chain,
                         int64_t step, int64_t n, int64_t* idx_out) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (n < 1 || n > cat->N) return fail(ctx, SPIDER_E_INVALID, "need 1 <= n <= N");
  if (!idx_out || chain < 0 || step < 0) return fail(ctx, SPIDER_E_INVALID, "bad argument");
  if (!entries_fit(1, n))
    return fail(ctx, SPIDER_E_UNSUPPORTED, "minibatch above 2^30 - 1 observations");
  int rc = reset_err_flag(ctx);
  if (rc) return rc;
  HIPCK(ctx->ws.reserve(1, n, (int64_t)cat->M + 1, 1, cat->M, 1), "workspace");
  BatchBufs b = ctx->ws.batch();
  b.start = nullptr;  // indices only: no (chain, event) counts
  launch_select(cat->view(), 1, n, nullptr, seed, nullptr, step, chain, b, ctx->ws.err.as<int>(),
                ctx->stream);
  HIPCK(hipMemcpyAsync(idx_out, b.obs, (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->stream),
        "copy indices");
  return check_select_flag(ctx);
}

int spider_noise(spider_ctx* ctx, int32_t cat_id, uint64_t seed, int32_t chain, int64_t step,
                 double* eta_out) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (!eta_out || chain < 0 || step < 0) return fail(ctx, SPIDER_E_INVALID, "bad argument");
  launch_noise(cat->view(), seed, chain, step, eta_out, ctx->stream);
  HIPCK(hipGetLastError(), "noise");
  return SPIDER_OK;
}

int spider_reset_chains(spider_ctx* ctx, int32_t cat_id, int32_t n_chains) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (n_chains < 1 || n_chains > 4096) return fail(ctx, SPIDER_E_INVALID, "need 1 <= n_chains <= 4096");
  const size_t per = (size_t)cat->M * 4;
  const int C = n_chains;
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  HIPCK(cat->theta.alloc(per * C * 8), "alloc chains");
  HIPCK(cat->v.alloc(per * C * 8), "alloc chains");
  HIPCK(cat->mean.alloc(per * C * 8), "alloc chains");
  HIPCK(cat->m2.alloc((size_t)cat->M * 10 * C * 8), "alloc chains");
  HIPCK(cat->steps.alloc((size_t)C * 8), "alloc chains");
  HIPCK(cat->mcount.alloc((size_t)C * 8), "alloc chains");
  for (int c = 0; c < C; ++c)
    HIPCK(hipMemcpyAsync(cat->theta.as<double>() + per * c, cat->hypo0.p, per * 8,
                         hipMemcpyDeviceToDevice, ctx->stream),
          "init chains");
  launch_fill(cat->v.as<double>(), 0.0, (int64_t)per * C, ctx->stream);
  launch_fill(cat->mean.as<double>(), 0.0, (int64_t)per * C, ctx->stream);
  launch_fill(cat->m2.as<double>(), 0.0, (int64_t)cat->M * 10 * C, ctx->stream);
  HIPCK(hipMemsetAsync(cat->steps.p, 0, (size_t)C * 8, ctx->stream), "init chains");
  HIPCK(hipMemsetAsync(cat->mcount.p, 0, (size_t)C * 8, ctx->stream), "init chains");
  HIPCK(hipGetLastError(), "init chains");
  cat->C = C;
  cat->adam_zeroed = false;
  cat->samples = nullptr;  // its layout was sized for the previous chains
  cat->sample_cap = 0;
  return SPIDER_OK;
}

// Numeric check of every chain state of the sets (waits for the stream).
static int check_finite_states(spider_ctx* ctx, const spider_chainset* sets, int n_sets) {
  for (int k = 0; k < n_sets; ++k) {
    const spider_chainset& st = sets[k];
    Catalog& cat = *get_cat(ctx, st.cat_id);
    DevBuf bad;
    HIPCK(bad.alloc(16), "alloc");
    const int big = INT_MAX;
    HIPCK(hipMemcpyAsync(bad.p, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream), "flag");
    launch_finite(cat.theta.as<double>(), (int64_t)cat.M * 4 * st.n_chains, (int64_t)cat.M * 4,
                  bad.as<int>(), ctx->stream);
    int first = INT_MAX;
    HIPCK(hipMemcpyAsync(&first, bad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "flag");
    HIPCK(hipStreamSynchronize(ctx->stream), "sync");
    if (first != INT_MAX) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "non-finite state in catalog %d chain %d", st.cat_id, first);
      return fail(ctx, SPIDER_E_NUMERIC, msg);
    }
  }
  return SPIDER_OK;
}

// Noise amplitude of step k of a call (constant, or the linear ramp).
static double noise_at(const spider_sgld_cfg& cfg, int64_t k) {
  if (cfg.noise_ramp == 0) return cfg.noise_scale;
  return cfg.noise_scale + (cfg.noise_scale_end - cfg.noise_scale) * ((double)k / (double)cfg.n_steps);
}

int spider_sgld_steps(spider_ctx* ctx, const spider_chainset* sets, int32_t n_sets,
                      const spider_sgld_cfg* cfg) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!sets || n_sets < 1 || !cfg) return fail(ctx, SPIDER_E_INVALID, "null or empty arguments");
  if (!(cfg->step > 0) || !(cfg->beta2 >= 0 && cfg->beta2 <= 1) || !(cfg->eps_p > 0) ||
      !std::isfinite(cfg->noise_scale) || cfg->noise_scale < 0 || cfg->n_steps < 0 ||
      cfg->burn_in < 0 || cfg->thin < 1 || (cfg->precond != 0 && cfg->precond != 1) ||
      (cfg->noise_ramp != 0 && cfg->noise_ramp != 1) ||
      (cfg->noise_ramp == 1 && !(std::isfinite(cfg->noise_scale_end) && cfg->noise_scale_end >= 0)))
    return fail(ctx, SPIDER_E_INVALID, "invalid sampler configuration");
  for (int k = 0; k < n_sets; ++k) {
    const spider_chainset& st = sets[k];
    Catalog* cat = get_cat(ctx, st.cat_id);
    Net* net = get_net(ctx, st.net_id);
    if (!cat || !net) return fail(ctx, SPIDER_E_INVALID, "unknown catalog or network id");
    if (st.n_chains < 1 || st.batch < 1 || st.batch > cat->N)
      return fail(ctx, SPIDER_E_INVALID, "need n_chains >= 1 and 1 <= batch <= N");
    if (st.precision != SPIDER_FP32 && st.precision != SPIDER_BF16)
      return fail(ctx, SPIDER_E_INVALID, "unknown precision");
    if (!entries_fit(st.n_chains, st.batch))
      return fail(ctx, SPIDER_E_UNSUPPORTED,
                  "a chain set holds more than 2^31 - 1 minibatch entries (2 n_chains batch)");
    if (cat->C < st.n_chains) {
      int rc = spider_reset_chains(ctx, st.cat_id, st.n_chains);
      if (rc) return rc;
    }
  }
  {
    int64_t total = 0;  // entries of all sets (one fused step holds them all)
    for (int k = 0; k < n_sets; ++k) {
      total += 2 * (int64_t)sets[k].n_chains * sets[k].batch;
      if (total > kMaxEntries)
        return fail(ctx, SPIDER_E_UNSUPPORTED,
                    "the chain sets hold more than 2^31 - 1 minibatch entries in total");
    }
  }
  int rc = reset_err_flag(ctx);
  if (rc) return rc;
  UpdateArgs ua{};
  ua.step = cfg->step;
  ua.beta2 = cfg->beta2;
  ua.eps_p = cfg->eps_p;
  ua.noise_scale = cfg->noise_scale;
  ua.precond = cfg->precond;
  ua.seed = cfg->seed;
  ua.burn = cfg->burn_in;
  ua.thin = cfg->thin;
  // sets sharing one network and precision (and no catalog twice, no
  // two-phase catalog) advance in fused steps
  bool fuse = true;
  for (int k = 1; k < n_sets && fuse; ++k)
    fuse = sets[k].net_id == sets[0].net_id && sets[k].precision == sets[0].precision;
  for (int k = 0; k < n_sets && fuse; ++k) {
    const Catalog* c = get_cat(ctx, sets[k].cat_id);
    fuse = c && c->L_p == c->L;
  }
  for (int k = 0; k < n_sets && fuse; ++k)
    for (int j = 0; j < k && fuse; ++j) fuse = sets[j].cat_id != sets[k].cat_id;
  if (fuse && cfg->n_steps > 0) {
    FusedSets f;
    rc = prepare_fused(ctx, sets, n_sets, f);
    if (rc) return rc;
    // a constant noise amplitude makes every step the same launches: the
    // first runs eagerly (it tunes the network kernel), the rest replay a
    // graph of one step
    const bool graph = ctx->graphs && !ctx->profiling && cfg->noise_ramp == 0 && cfg->n_steps > 1;
    for (int64_t t = 0; t < (graph ? 1 : cfg->n_steps); ++t) {
      ua.noise_scale = noise_at(*cfg, t);
      rc = fused_step(ctx, sets, n_sets, f, ua);
      if (rc) return rc;
    }
    if (graph) {
      rc = graph_steps(ctx, sets, n_sets, f, ua, cfg->n_steps - 1);
      if (rc) return rc;
    }
  }
  for (int64_t t = 0; t < (fuse ? 0 : cfg->n_steps); ++t) {
    ua.noise_scale = noise_at(*cfg, t);
    for (int k = 0; k < n_sets; ++k) {
      const spider_chainset& st = sets[k];
      Catalog& cat = *get_cat(ctx, st.cat_id);
      Net& net = *get_net(ctx, st.net_id);
      const int C = st.n_chains;
      rc = run_batch(ctx, cat, net, st.precision, C, st.batch, cat.theta.as<double>(),
                     (int64_t)cat.M * 4, nullptr, cfg->seed, cat.steps.as<int64_t>(), 0, 0, true,
                     (double)cat.N / (double)st.batch);
      if (rc) return rc;
      Workspace& ws = ctx->ws;
      launch_centroid(cat.theta.as<double>(), C, cat.M, ws.partial.as<double>(),
                      ws.thetabar.as<double>(), ctx->stream);
      launch_update(cat.view(), C, cat.theta.as<double>(), cat.v.as<double>(), ws.G.as<double>(),
                    ws.thetabar.as<double>(), cat.steps.as<int64_t>(), cat.mcount.as<int64_t>(),
                    with_samples(ua, cat), cat.mean.as<double>(), cat.m2.as<double>(),
                    ctx->stream);
      HIPCK(hipGetLastError(), "update");
    }
  }
  rc = check_finite_states(ctx, sets, n_sets);
  if (rc) return rc;
  return check_select_flag(ctx);
}

int spider_map_steps(spider_ctx* ctx, const spider_chainset* sets, int32_t n_sets,
                     const spider_map_cfg* cfg) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!sets || n_sets < 1 || !cfg) return fail(ctx, SPIDER_E_INVALID, "null or empty arguments");
  if (!(cfg->lr > 0) || !std::isfinite(cfg->lr) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) ||
      !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0) || cfg->n_steps < 0)
    return fail(ctx, SPIDER_E_INVALID, "invalid optimiser configuration");
  for (int k = 0; k < n_sets; ++k) {
    const spider_chainset& st = sets[k];
    Catalog* cat = get_cat(ctx, st.cat_id);
    Net* net = get_net(ctx, st.net_id);
    if (!cat || !net) return fail(ctx, SPIDER_E_INVALID, "unknown catalog or network id");
    if (st.n_chains < 1 || st.batch < 1 || st.batch > cat->N)
      return fail(ctx, SPIDER_E_INVALID, "need n_chains >= 1 and 1 <= batch <= N");
    if (st.precision != SPIDER_FP32 && st.precision != SPIDER_BF16)
      return fail(ctx, SPIDER_E_INVALID, "unknown precision");
    if (!entries_fit(st.n_chains, st.batch))
      return fail(ctx, SPIDER_E_UNSUPPORTED,
                  "a chain set holds more than 2^31 - 1 minibatch entries (2 n_chains batch)");
    if (cat->C < st.n_chains) {
      int rc = spider_reset_chains(ctx, st.cat_id, st.n_chains);
      if (rc) return rc;
    }
    const size_t bytes = (size_t)cat->M * 4 * cat->C * 8;
    if (!cat->adam_m.p || cat->adam_m.bytes < bytes || cat->adam_v.bytes < bytes) {
      HIPCK(hipStreamSynchronize(ctx->stream), "sync");
      HIPCK(cat->adam_m.alloc(bytes), "alloc optimiser state");
      HIPCK(cat->adam_v.alloc(bytes), "alloc optimiser state");
      cat->adam_zeroed = false;
    }
    if (!cat->adam_zeroed) {
      launch_fill(cat->adam_m.as<double>(), 0.0, (int64_t)cat->M * 4 * cat->C, ctx->stream);
      launch_fill(cat->adam_v.as<double>(), 0.0, (int64_t)cat->M * 4 * cat->C, ctx->stream);
      cat->adam_zeroed = true;
    }
  }
  int rc = reset_err_flag(ctx);
  if (rc) return rc;
  AdamArgs aa;
  aa.lr = cfg->lr;
  aa.beta1 = cfg->beta1;
  aa.beta2 = cfg->beta2;
  aa.eps = cfg->eps;
  for (int64_t t = 0; t < cfg->n_steps; ++t) {
    for (int k = 0; k < n_sets; ++k) {
      const spider_chainset& st = sets[k];
      Catalog& cat = *get_cat(ctx, st.cat_id);
      Net& net = *get_net(ctx, st.net_id);
      const int C = st.n_chains;
      // G = (1/n) sum_batch sign(r) dtau^/dtheta = -grad of the batch L1 loss
      rc = run_batch(ctx, cat, net, st.precision, C, st.batch, cat.theta.as<double>(),
                     (int64_t)cat.M * 4, nullptr, cfg->seed, cat.steps.as<int64_t>(), 0, 0, true,
                     1.0 / (double)st.batch, true);
      if (rc) return rc;
      launch_adam(C, cat.M, cat.theta.as<double>(), cat.adam_m.as<double>(),
                  cat.adam_v.as<double>(), ctx->ws.G.as<double>(), cat.steps.as<int64_t>(), aa,
                  ctx->stream);
      HIPCK(hipGetLastError(), "optimiser step");
    }
  }
  rc = check_finite_states(ctx, sets, n_sets);
  if (rc) return rc;
  return check_select_flag(ctx);
}

// Median of n ascending doubles on the device (mean of the middle two when n is even).
static hipError_t device_median(const double* sorted, int64_t n, hipStream_t s, double* med) {
  double mid[2] = {0, 0};
  const int64_t lo = (n - 1) / 2;
  hipError_t e = hipMemcpyAsync(mid, sorted + lo, (n % 2 ? 1 : 2) * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *med = n % 2 ? mid[0] : 0.5 * (mid[0] + mid[1]);
  return e;
}

extern "C++" {
// Runs the network and residual kernels over all N observations of a
// catalog at one chain's state, in chunks of at most 2^22 observations, and
// calls chunk(start, len) after each (the batch buffers then hold the chunk).
template <class F>
static int over_all_observations(spider_ctx* ctx, Catalog& cat, Net& net, int prec, int chain,
                                 DevBuf& idx, F chunk) {
  const int64_t N = cat.N;
  const int64_t CH = std::min<int64_t>(N, (int64_t)1 << 22);
  HIPCK(idx.alloc((size_t)std::max<int64_t>(CH, 1) * 8), "alloc indices");
  const double* theta = cat.theta.as<double>() + (size_t)cat.M * 4 * chain;
  for (int64_t start = 0; start < N; start += CH) {
    const int64_t len = std::min(CH, N - start);
    launch_iota(idx.as<int64_t>(), start, len, ctx->stream);
    int rc = run_batch(ctx, cat, net, prec, 1, len, theta, (int64_t)cat.M * 4,
                       idx.as<int64_t>(), 0, nullptr, 0, 0, false, 1.0, true);
    if (rc) return rc;
    rc = chunk(start, len, theta);
    if (rc) return rc;
  }
  return SPIDER_OK;
}

}  // extern "C++"

static int screening_args(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                          int32_t chain, Catalog*& cat, Net*& net) {
  cat = get_cat(ctx, cat_id);
  net = get_net(ctx, net_id);
  if (!cat || !net) return fail(ctx, SPIDER_E_INVALID, "unknown catalog or network id");
  if (precision != SPIDER_FP32 && precision != SPIDER_BF16)
    return fail(ctx, SPIDER_E_INVALID, "unknown precision");
  if (chain < 0 || chain >= cat->C) return fail(ctx, SPIDER_E_INVALID, "bad chain index");
  return SPIDER_OK;
}

int spider_outliers(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                    int32_t chain, double k_mad, uint8_t* keep, int64_t* n_keep, double* median,
                    double* mad) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat;
  Net* net;
  int rc = screening_args(ctx, cat_id, net_id, precision, chain, cat, net);
  if (rc) return rc;
  if (!(k_mad > 0) || !std::isfinite(k_mad) || !keep)
    return fail(ctx, SPIDER_E_INVALID, "need k_mad > 0 and a keep array");
  const int64_t N = cat->N;
  DevBuf r, d, srt, idx, temp, cnt;
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  HIPCK(r.alloc((size_t)N * 8), "alloc residuals");
  HIPCK(d.alloc((size_t)N * 8), "alloc residuals");
  HIPCK(srt.alloc((size_t)N * 8), "alloc residuals");
  HIPCK(cnt.alloc(16), "alloc count");
  rc = reset_err_flag(ctx);
  if (rc) return rc;
  // residuals of every observation at the chain's state
  rc = over_all_observations(ctx, *cat, *net, precision, chain, idx,
                             [&](int64_t start, int64_t len, const double*) -> int {
                               HIPCK(hipMemcpyAsync(r.as<double>() + start, ctx->ws.r.p,
                                                    (size_t)len * 8, hipMemcpyDeviceToDevice,
                                                    ctx->stream),
                                     "copy residuals");
                               return SPIDER_OK;
                             });
  if (rc) return rc;
  size_t tb = 0;
  HIPCK(sort_doubles(nullptr, nullptr, N, nullptr, &tb, ctx->stream), "sort size");
  HIPCK(temp.alloc(tb), "alloc sort scratch");
  double med = 0, md = 0;
  HIPCK(sort_doubles(r.as<double>(), srt.as<double>(), N, temp.p, &tb, ctx->stream), "sort");
  HIPCK(device_median(srt.as<double>(), N, ctx->stream, &med), "median");
  launch_absdev(r.as<double>(), N, med, d.as<double>(), ctx->stream);
  HIPCK(sort_doubles(d.as<double>(), srt.as<double>(), N, temp.p, &tb, ctx->stream), "sort");
  HIPCK(device_median(srt.as<double>(), N, ctx->stream, &md), "median");
  HIPCK(hipMemsetAsync(cnt.p, 0, 8, ctx->stream), "count");
  launch_keep(r.as<double>(), N, med, k_mad * md, keep, (unsigned long long*)cnt.p, ctx->stream);
  HIPCK(hipGetLastError(), "screening kernels");
  unsigned long long kept = 0;
  HIPCK(hipMemcpyAsync(&kept, cnt.p, 8, hipMemcpyDeviceToHost, ctx->stream), "count");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  if (n_keep) *n_keep = (int64_t)kept;
  if (median) *median = med;
  if (mad) *mad = md;
  return check_select_flag(ctx);
}

int spider_linearity(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                     int32_t chain, double max_rel_err, uint8_t* keep, int64_t* n_keep) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat;
  Net* net;
  int rc = screening_args(ctx, cat_id, net_id, precision, chain, cat, net);
  if (rc) return rc;
  if (!(max_rel_err >= 0) || !std::isfinite(max_rel_err) || !keep)
    return fail(ctx, SPIDER_E_INVALID, "need max_rel_err >= 0 and a keep array");
  DevBuf idx, cnt;
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  HIPCK(cnt.alloc(16), "alloc count");
  rc = reset_err_flag(ctx);
  if (rc) return rc;
  HIPCK(hipMemsetAsync(cnt.p, 0, 8, ctx->stream), "count");
  rc = over_all_observations(ctx, *cat, *net, precision, chain, idx,
                             [&](int64_t start, int64_t len, const double* theta) -> int {
                               launch_linear_keep(ctx->ws.batch(), theta, len, max_rel_err,
                                                  keep + start, (unsigned long long*)cnt.p,
                                                  ctx->stream);
                               HIPCK(hipGetLastError(), "linearity kernel");
                               return SPIDER_OK;
                             });
  if (rc) return rc;
  unsigned long long kept = 0;
  HIPCK(hipMemcpyAsync(&kept, cnt.p, 8, hipMemcpyDeviceToHost, ctx->stream), "count");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  if (n_keep) *n_keep = (int64_t)kept;
  return check_select_flag(ctx);
}

int spider_set_sample_buffer(spider_ctx* ctx, int32_t cat_id, double* samples,
                             int64_t capacity) {
  if (!ctx) return SPIDER_E_INVALID;
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (samples && capacity < 1) return fail(ctx, SPIDER_E_INVALID, "need capacity >= 1");
  if (samples && cat->C < 1)
    return fail(ctx, SPIDER_E_STATE, "reset the chains before attaching a sample buffer");
  cat->samples = samples;
  cat->sample_cap = samples ? capacity : 0;
  return SPIDER_OK;
}

int spider_quantiles(spider_ctx* ctx, const double* samples, int64_t n_samples, int64_t n_params,
                     const double* probs, int32_t n_probs, double* out) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!samples || !probs || !out) return fail(ctx, SPIDER_E_INVALID, "null argument");
  if (n_samples < 1 || n_params < 1 || n_params > INT32_MAX || n_probs < 1)
    return fail(ctx, SPIDER_E_INVALID, "need n_samples, n_params, n_probs >= 1");
  if (n_samples > kMaxQuantileSamples)
    return fail(ctx, SPIDER_E_UNSUPPORTED, "at most 8192 samples per parameter");
  for (int32_t q = 0; q < n_probs; ++q)
    if (!(probs[q] >= 0.0 && probs[q] <= 1.0))
      return fail(ctx, SPIDER_E_INVALID, "probabilities must lie in [0, 1]");
  DevBuf pd;
  HIPCK(upload(pd, probs, (size_t)n_probs * 8, SPIDER_MEM_HOST, ctx->stream), "upload probs");
  HIPCK(launch_quantiles(samples, n_samples, n_params, pd.as<double>(), n_probs, out,
                         ctx->stream),
        "quantile kernel");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  return SPIDER_OK;
}

int spider_sample_ranks(spider_ctx* ctx, const double* samples, int64_t n_samples,
                        int64_t n_params, const double* values, double* frac) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!samples || !values || !frac) return fail(ctx, SPIDER_E_INVALID, "null argument");
  if (n_samples < 1 || n_params < 1)
    return fail(ctx, SPIDER_E_INVALID, "need n_samples, n_params >= 1");
  HIPCK(launch_ranks(samples, n_samples, n_params, values, frac, ctx->stream), "rank kernel");
  return SPIDER_OK;
}

int spider_ess(spider_ctx* ctx, const double* samples, int64_t n_draws, int32_t n_chains,
               int64_t n_params, double* ess) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  if (!samples || !ess) return fail(ctx, SPIDER_E_INVALID, "null argument");
  if (n_draws < 4 || n_chains < 1 || n_params < 1)
    return fail(ctx, SPIDER_E_INVALID, "need n_draws >= 4, n_chains >= 1, n_params >= 1");
  if (n_chains > kMaxEssChains) return fail(ctx, SPIDER_E_UNSUPPORTED, "at most 64 chains");
  HIPCK(launch_ess(samples, n_draws, n_chains, n_params, ess, ctx->stream), "ess kernel");
  return SPIDER_OK;
}

int spider_noise_ratio(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                       int32_t chain, int64_t batch, int32_t n_batches, const spider_sgld_cfg* cfg,
                       double* ratio, double* mean_ratio) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat;
  Net* net;
  int rc = screening_args(ctx, cat_id, net_id, precision, chain, cat, net);
  if (rc) return rc;
  if (!cfg || !ratio) return fail(ctx, SPIDER_E_INVALID, "null argument");
  if (batch < 1 || batch > cat->N || n_batches < 2)
    return fail(ctx, SPIDER_E_INVALID, "need 1 <= batch <= N and n_batches >= 2");
  if (!entries_fit(1, batch))
    return fail(ctx, SPIDER_E_UNSUPPORTED, "minibatch above 2^30 - 1 observations");
  if (!(cfg->step > 0) || !(cfg->noise_scale > 0) || !(cfg->eps_p > 0))
    return fail(ctx, SPIDER_E_INVALID, "need step, noise_scale, eps_p > 0");
  const int64_t n4 = (int64_t)cat->M * 4;
  int64_t t0 = 0;
  HIPCK(hipMemcpyAsync(&t0, cat->steps.as<int64_t>() + chain, 8, hipMemcpyDeviceToHost,
                       ctx->stream),
        "read step");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  DevBuf mean, m2, part;
  const int64_t nb = noise_ratio_blocks(n4);
  HIPCK(mean.alloc((size_t)n4 * 8), "alloc");
  HIPCK(m2.alloc((size_t)n4 * 8), "alloc");
  HIPCK(part.alloc((size_t)nb * 8), "alloc");
  rc = reset_err_flag(ctx);
  if (rc) return rc;
  const double* theta = cat->theta.as<double>() + (size_t)n4 * chain;
  // the likelihood gradients of the chain's next n_batches minibatches at its
  // current state (the priors add the same vector to each)
  for (int32_t k = 0; k < n_batches; ++k) {
    rc = run_batch(ctx, *cat, *net, precision, 1, batch, theta, n4, nullptr, cfg->seed, nullptr,
                   t0 + k, chain, true, (double)cat->N / (double)batch);
    if (rc) return rc;
    launch_welford(ctx->ws.G.as<double>(), n4, k, mean.as<double>(), m2.as<double>(),
                   ctx->stream);
  }
  launch_noise_ratio(m2.as<double>(), n4, n_batches, cat->v.as<double>() + (size_t)n4 * chain,
                     cfg->precond, cfg->eps_p, cfg->step, cfg->noise_scale, ratio, part.as<double>(),
                     ctx->stream);
  HIPCK(hipGetLastError(), "noise ratio kernels");
  std::vector<double> ps(nb);
  HIPCK(hipMemcpyAsync(ps.data(), part.p, (size_t)nb * 8, hipMemcpyDeviceToHost, ctx->stream),
        "read partial sums");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  double tot = 0.0;
  for (double x : ps) tot += x;
  if (mean_ratio) *mean_ratio = tot / (double)n4;
  return check_select_flag(ctx);
}

int spider_moments(spider_ctx* ctx, int32_t cat_id, int32_t chain, double* mean, double* cov,
                   int64_t* count) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (cat->C == 0) return fail(ctx, SPIDER_E_STATE, "catalog has no chains");
  if (chain < -1 || chain >= cat->C) return fail(ctx, SPIDER_E_INVALID, "bad chain index");
  const int c0 = chain < 0 ? 0 : chain;
  const int C = chain < 0 ? cat->C : 1;
  std::vector<int64_t> cnt(cat->C);
  HIPCK(hipMemcpyAsync(cnt.data(), cat->mcount.p, cnt.size() * 8, hipMemcpyDeviceToHost,
                       ctx->stream),
        "read counts");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  int64_t total = 0;
  for (int c = c0; c < c0 + C; ++c) total += cnt[c];
  if (count) *count = total;
  launch_pool_moments(C, cat->M, cat->mean.as<double>() + (size_t)c0 * cat->M * 4,
                      cat->m2.as<double>() + (size_t)c0 * cat->M * 10,
                      cat->mcount.as<int64_t>() + c0, mean, cov, ctx->stream);
  HIPCK(hipGetLastError(), "moments");
  return SPIDER_OK;
}

int spider_get_state(spider_ctx* ctx, int32_t cat_id, int32_t chain, double* theta, double* v,
                     int64_t* step) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (chain < 0 || chain >= cat->C) return fail(ctx, SPIDER_E_INVALID, "bad chain index");
  const size_t per = (size_t)cat->M * 4;
  if (theta)
    HIPCK(hipMemcpyAsync(theta, cat->theta.as<double>() + per * chain, per * 8,
                         hipMemcpyDeviceToDevice, ctx->stream),
          "copy state");
  if (v)
    HIPCK(hipMemcpyAsync(v, cat->v.as<double>() + per * chain, per * 8, hipMemcpyDeviceToDevice,
                         ctx->stream),
          "copy state");
  if (step) {
    HIPCK(hipMemcpyAsync(step, cat->steps.as<int64_t>() + chain, 8, hipMemcpyDeviceToHost,
                         ctx->stream),
          "copy step");
    HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  }
  return SPIDER_OK;
}

int spider_set_state(spider_ctx* ctx, int32_t cat_id, int32_t chain, const double* theta,
                     const double* v, int64_t step) {
  if (!ctx) return SPIDER_E_INVALID;
  DeviceGuard g(ctx->device);
  Catalog* cat = get_cat(ctx, cat_id);
  if (!cat) return fail(ctx, SPIDER_E_INVALID, "unknown catalog id");
  if (chain < 0 || chain >= cat->C) return fail(ctx, SPIDER_E_INVALID, "bad chain index");
  if (!theta || step < 0) return fail(ctx, SPIDER_E_INVALID, "null theta or negative step");
  const size_t per = (size_t)cat->M * 4;
  HIPCK(hipMemcpyAsync(cat->theta.as<double>() + per * chain, theta, per * 8,
                       hipMemcpyDeviceToDevice, ctx->stream),
        "copy state");
  if (v)
    HIPCK(hipMemcpyAsync(cat->v.as<double>() + per * chain, v, per * 8, hipMemcpyDeviceToDevice,
                         ctx->stream),
          "copy state");
  else
    launch_fill(cat->v.as<double>() + per * chain, 0.0, (int64_t)per, ctx->stream);
  HIPCK(hipMemcpyAsync(cat->steps.as<int64_t>() + chain, &step, 8, hipMemcpyHostToDevice,
                       ctx->stream),
        "copy step");
  HIPCK(hipStreamSynchronize(ctx->stream), "sync");
  return SPIDER_OK;
}

}  // extern "C"
