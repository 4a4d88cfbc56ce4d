// C ABI of libdmrg: contexts, superblocks, the product, its adjoint, the
// Lanczos ground state and density-matrix truncation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <unistd.h>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/dmrg.h"
#include "eigen.h"
#include "kernels.h"
#include "plan.h"

using namespace dmrg;

namespace {

thread_local std::string g_err;

// Host threads for the per-sector eigen-solves: OMP_NUM_THREADS when set
// (the machine's share for this process), else the hardware count; at most 32.
// The sum of row[0..cnt) in the order of one wave's row sum on the device
// (lane l adds entries l, l + 64, ... in batches of 16 per lane, then a
// butterfly over the 64 lanes): the same bits as that device sum.
double wave_order_sum(const double* row, int cnt) {
  double s[64];
  for (int l = 0; l < 64; ++l) s[l] = 0.0;
  for (int b0 = 0; b0 < cnt; b0 += 64 * 16)
    for (int l = 0; l < 64; ++l)
      for (int u = 0; u < 16; ++u) {
        const int b = b0 + l + 64 * u;
        s[l] += b < cnt ? row[b] : 0.0;
      }
  for (int off = 32; off > 0; off >>= 1) {
    double t[64];
    for (int l = 0; l < 64; ++l) t[l] = s[l] + s[l ^ off];
    for (int l = 0; l < 64; ++l) s[l] = t[l];
  }
  return s[0];
}

int host_threads() {
  int n = (int)std::max(1u, std::thread::hardware_concurrency());
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v > 0) n = std::min(n, v);
  }
  return std::max(1, std::min(n, 32));
}

// Host worker threads kept for the life of the process, so that the
// density-matrix solves do not start and join threads on every call.
// run(n, f) calls f(0..n-1) once each, f(0) on the calling thread, and
// returns when all have finished; calls from several host threads queue.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool(host_threads() - 1);
    return pool;
  }
  void run(int n, const std::function<void(int)>& f) {
    std::lock_guard<std::mutex> one(run_mu_);
    if (getpid() != pid_) {   // a forked child has no workers: run serially
      for (int t = 0; t < std::max(1, n); ++t) f(t);
      return;
    }
    n = std::max(1, std::min(n, (int)workers_.size() + 1));
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      active_ = n - 1;
      pending_ = n - 1;
      ++gen_;
    }
    cv_.notify_all();
    f(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  explicit HostPool(int nworkers) : pid_(getpid()) {
    for (int i = 0; i < nworkers; ++i) workers_.emplace_back([this, i] { loop(i + 1); });
  }
  void loop(int id) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* job = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        if (id > active_) continue;
        job = job_;
      }
      (*job)(id);
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) done_.notify_one();
    }
  }
  pid_t pid_;
  std::vector<std::thread> workers_;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* job_ = nullptr;
  uint64_t gen_ = 0;
  int active_ = 0, pending_ = 0;
  bool stop_ = false;
};

dmrg_status fail(dmrg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? DMRG_E_NOMEM : DMRG_E_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// Device memory the library holds per device, and the cap set with
// dmrg_ctx_set_mem_cap (0: none).
constexpr int kMaxDevices = 64;
struct MemAccount {
  std::atomic<int64_t> used{0}, cap{0};
};
MemAccount g_mem[kMaxDevices];

// Device allocation owned by the library, counted against its device's cap.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = -1;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (dev >= 0 && dev < kMaxDevices) g_mem[dev].used.fetch_sub((int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
    dev = -1;
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    const size_t want = std::max<size_t>(n, 256);
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    MemAccount* acct = d >= 0 && d < kMaxDevices ? &g_mem[d] : nullptr;
    if (acct) {
      // reserve first, so that concurrent callers cannot pass the cap together
      const int64_t cap = acct->cap.load();
      const int64_t now = acct->used.fetch_add((int64_t)want) + (int64_t)want;
      if (cap > 0 && now > cap) {
        acct->used.fetch_sub((int64_t)want);
        return hipErrorOutOfMemory;
      }
    }
    e = hipMalloc(&p, want);
    if (e == hipSuccess) {
      bytes = want;
      dev = acct ? d : -1;
    } else {
      p = nullptr;
      if (acct) acct->used.fetch_sub((int64_t)want);
    }
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Sets the context's device for the duration of a call and restores the old one.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// A plan and its device copy.
struct Staged {
  Plan plan;
  DevBuf tiles, segs, gsrc, gscale, dense64, dense32;
  DevBuf images;            // one tile image per workgroup slot of the fused kernel
  DevBuf psi32;             // FP32 copy of the input vector (products that read one)
  DevBuf wg_start;          // persistent launch: each workgroup's slots
  DevBuf coef_img, coef_seg;   // where each coefficient sits in images / segs
  int64_t ncoef_img = 0, ncoef_seg = 0;
  // the macro-tile plan (FP32 / BF16 variant 1), staged on first use
  // (dmrg_sb_set_variant(1) or the autotuner) once the FP32 pool is
  bool mac_staged = false;   // staging attempted
  bool has_mac = false;      // staged and non-empty
  int32_t mac_nwg = 0, mac_nshared = 0, mac_nparts = 0;
  DevBuf mtiles, msegs, mggs, mitems, mwg, mshared, mpart, mcoef_seg, mcoef_gg, mdense;
  int64_t mac_ndense = 0;
  int64_t ncoef_mseg = 0, ncoef_mgg = 0;
  int32_t nwg = 0;
  int32_t img_stride = 0;   // words per image
  int32_t nslots = 0;
  bool has32 = false;
  int max_nseg = 0;
  std::vector<std::pair<SegDesc, TileDesc>> plain;  // one entry per (block, term)
};

// Host copy of a superblock's input (needed to build the transposed plan).
struct OpCopy {
  int64_t delta = 0;
  std::vector<int32_t> row, col;
  std::vector<std::vector<double>> data;
  std::vector<const double*> ptrs;
  dmrg_op view{};
};

}  // namespace

struct dmrg_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  DevBuf tr_images, tr_tmp;   // basis-change scratch
  // optional per-launch timing of the product kernels (HIP events on `stream`)
  hipEvent_t chk[2] = {nullptr, nullptr};   // Lanczos check copies
  int timing = 0;          // time every timing-th product launch (0: off)
  int64_t tick = 0;        // product launches since timing was set
  int64_t products[4] = {0, 0, 0, 0};   // launches per precision while timing was on
  struct Mark {
    hipEvent_t a, b;
    int prec;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> spare;
  // Lanczos workspace (grow-only)
  DevBuf V, w, partial, small;
  DevBuf v32;          // FP32 copy of the next product's input (reduced-precision cycles)
  size_t v32_n = 0;    // its padded length (the padding is zero)
  double* host_small = nullptr;   // pinned, for per-iteration scalars
  size_t host_small_n = 0;
  double* host_rho = nullptr;     // pinned, density-matrix blocks on their way to the host
  size_t host_rho_n = 0;
  hipStream_t cap_stream = nullptr;   // non-blocking, default priority: where Lanczos graphs are captured
};

struct dmrg_sb_s {
  dmrg_ctx ctx = nullptr;
  int device = -1;              // copies, so destruction does not need the context
  hipStream_t stream = nullptr;
  dmrg_prec prec = DMRG_FP64;
  std::vector<int64_t> qS, qE;
  std::vector<int32_t> dS, dE;
  int64_t q_target = 0;
  int64_t q_in = 0;             // == q_target for a Hamiltonian superblock
  std::vector<double> coeff;
  std::vector<int32_t> group;
  std::vector<std::unique_ptr<OpCopy>> opA, opB;
  Staged fwd;
  std::unique_ptr<Staged> adj;
  int variant[3] = {0, 0, 0};   // fused-kernel variant per kernel precision (autotuner)
  int reorth = 0;               // Lanczos reorthogonalisation (dmrg_sb_set_reorth)
  // dmrg_sb_set_graphs: the Lanczos steps between two host checks, captured
  // once per position in a restart cycle and replayed.  The graphs bake in
  // the buffers and launch choices of `key`; a call with another key drops
  // them all.
  struct LzGraphs {
    bool on = false;
    struct Key {
      const void* ptr[8];
      int64_t D;
      int32_t nvec, prec, variant, twice;
      bool operator==(const Key& o) const { return std::memcmp(this, &o, sizeof(Key)) == 0; }
    } key;
    std::vector<hipGraphExec_t> seg;   // by position: steps 1..kCheck-1, then kCheck runs of kCheck
    int64_t replays = 0, captures = 0;
    LzGraphs() { std::memset(&key, 0, sizeof(key)); }
    void drop() {
      for (hipGraphExec_t& g : seg)
        if (g) (void)hipGraphExecDestroy(g);
      seg.clear();
    }
    ~LzGraphs() { drop(); }
  } lzg;
  // density-matrix blocks: tile images per side (built on first use), output
  struct RhoPlan {
    bool built = false;
    std::vector<int64_t> off;   // per sector of the side: offset of its block, -1 if none
    int ntiles = 0;
    int32_t stride = 0;
    int64_t total = 0;
    DevBuf images;
  };
  RhoPlan rho_plan[2];
  // per-sector eigen-solve workspaces of the last truncation on each side,
  // kept so that their pages are reused by the next call
  std::vector<SymEig> rho_eig[2];
  DevBuf rho_out;
  std::vector<double> tr_lambda;
  std::vector<int32_t> tr_sec, tr_kps;
  std::vector<double> tr_W;          // the kept vectors of all sectors, back to back
  std::vector<double> spec_W;        // eigenvectors formed ahead of the selection
  std::vector<const double*> tr_Wp;
};

namespace {

dmrg_status upload(DevBuf& b, const void* src, size_t bytes, hipStream_t s) {
  HIP_TRY(b.ensure(bytes));
  if (bytes) HIP_TRY(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
  return DMRG_OK;
}

// Tile images of a staged plan (again after a coefficient change).
dmrg_status stage_images(Staged& st, hipStream_t s) {
  std::vector<uint32_t> img;
  std::vector<CoefRef> coefs;
  std::string err;
  if (!build_images(st.plan.tiles, st.plan.segs, st.plan.order, st.plan.gsrc, st.plan.gscale, img,
                    st.img_stride, err, &coefs))
    return fail(DMRG_E_UNSUPPORTED, err);
  st.nslots = (int32_t)st.plan.order.size();
  dmrg_status r = upload(st.images, img.data(), img.size() * sizeof(uint32_t), s);
  if (r != DMRG_OK) return r;
  st.ncoef_img = (int64_t)coefs.size();
  if (!coefs.empty() && (r = upload(st.coef_img, coefs.data(), coefs.size() * sizeof(CoefRef), s)) != DMRG_OK)
    return r;
  st.nwg = (int32_t)st.plan.wg_start.size() - 1;
  if (st.nwg > 0 &&
      (r = upload(st.wg_start, st.plan.wg_start.data(), st.plan.wg_start.size() * sizeof(int32_t), s)) !=
          DMRG_OK)
    return r;
  HIP_TRY(hipStreamSynchronize(s));   // the host image vector dies here
  return DMRG_OK;
}

// The macro-tile plan of a staged plan: records, work lists and room for
// the partial tiles on the device.
dmrg_status stage_macro(Staged& st, hipStream_t s);

// The macro-tile plan of a staged FP32 pool, the first time it is asked for.
dmrg_status ensure_macro(Staged& st, hipStream_t s) {
  if (!st.has32 || st.mac_staged) return DMRG_OK;
  st.mac_staged = true;
  return stage_macro(st, s);
}

dmrg_status stage_macro(Staged& st, hipStream_t s) {
  MacroPlan mp;
  {
    std::vector<float> pool32;
    dense_f32(st.plan, pool32);
    build_macro(st.plan, pool32, kPersistentWGs * kMacWGsPerCU, 8, mp);
  }
  dmrg_status r;
  if ((r = upload(st.mdense, mp.dense.data(), mp.dense.size() * sizeof(float), s)) != DMRG_OK) return r;
  st.mac_ndense = (int64_t)mp.dense.size();
  if ((r = upload(st.mtiles, mp.tiles.data(), mp.tiles.size() * sizeof(MacTile), s)) != DMRG_OK) return r;
  if ((r = upload(st.msegs, mp.segs.data(), mp.segs.size() * sizeof(MacSeg), s)) != DMRG_OK) return r;
  if ((r = upload(st.mggs, mp.ggs.data(), mp.ggs.size() * sizeof(MacGG), s)) != DMRG_OK) return r;
  if ((r = upload(st.mitems, mp.items.data(), mp.items.size() * sizeof(MacItem), s)) != DMRG_OK) return r;
  if ((r = upload(st.mwg, mp.wg_start.data(), mp.wg_start.size() * sizeof(int32_t), s)) != DMRG_OK) return r;
  if ((r = upload(st.mshared, mp.shared.data(), mp.shared.size() * sizeof(int32_t), s)) != DMRG_OK) return r;
  if ((r = upload(st.mcoef_seg, mp.coef_seg.data(), mp.coef_seg.size() * sizeof(CoefRef), s)) != DMRG_OK)
    return r;
  if ((r = upload(st.mcoef_gg, mp.coef_gg.data(), mp.coef_gg.size() * sizeof(CoefRef), s)) != DMRG_OK)
    return r;
  st.mac_nwg = (int32_t)mp.wg_start.size() - 1;
  st.mac_nshared = (int32_t)mp.shared.size();
  st.mac_nparts = mp.nparts;
  st.ncoef_mseg = (int64_t)mp.coef_seg.size();
  st.ncoef_mgg = (int64_t)mp.coef_gg.size();
  HIP_TRY(st.mpart.ensure((size_t)std::max(1, mp.nparts) * kMac * kMac * sizeof(float)));
  HIP_TRY(hipStreamSynchronize(s));   // the host records die here
  st.has_mac = st.mac_nwg > 0;
  return DMRG_OK;
}

dmrg_status stage(dmrg_ctx ctx, Staged& st, bool want32) {
  const Plan& p = st.plan;
  hipStream_t s = ctx->stream;
  dmrg_status r;
  if ((r = stage_images(st, s)) != DMRG_OK) return r;
  if ((r = upload(st.tiles, p.tiles.data(), p.tiles.size() * sizeof(TileDesc), s)) != DMRG_OK) return r;
  if ((r = upload(st.segs, p.segs.data(), p.segs.size() * sizeof(SegDesc), s)) != DMRG_OK) return r;
  {
    std::vector<CoefRef> refs(p.segs.size());
    for (size_t i = 0; i < p.segs.size(); ++i)
      refs[i] = {(int64_t)(i * sizeof(SegDesc) + offsetof(SegDesc, c)), p.segs[i].term, 0};
    st.ncoef_seg = (int64_t)refs.size();
    if (!refs.empty() && (r = upload(st.coef_seg, refs.data(), refs.size() * sizeof(CoefRef), s)) != DMRG_OK)
      return r;
    HIP_TRY(hipStreamSynchronize(s));   // the host table dies here
  }
  if ((r = upload(st.gsrc, p.gsrc.data(), p.gsrc.size() * sizeof(int32_t), s)) != DMRG_OK) return r;
  if ((r = upload(st.gscale, p.gscale.data(), p.gscale.size() * sizeof(double), s)) != DMRG_OK) return r;
  if ((r = upload(st.dense64, p.dense.data(), p.dense.size() * sizeof(double), s)) != DMRG_OK) return r;
  if (want32) {
    std::vector<float> f;
    dense_f32(p, f);
    if ((r = upload(st.dense32, f.data(), f.size() * sizeof(float), s)) != DMRG_OK) return r;
    HIP_TRY(hipStreamSynchronize(s));   // the host staging vector dies here
    st.has32 = true;
  }
  st.max_nseg = 0;
  st.plain.clear();
  for (size_t q = 0; q < p.pair_s.size(); ++q) {
    st.max_nseg = std::max(st.max_nseg, p.pair_nseg[q]);
    TileDesc t{};
    t.y_off = p.pair_off[q];
    t.a = p.dS[p.pair_s[q]];
    t.b = p.dE[p.pair_e[q]];
    t.ldy = t.b;
    for (int32_t k = 0; k < p.pair_nseg[q]; ++k) st.plain.push_back({p.segs[p.pair_seg0[q] + k], t});
  }
  HIP_TRY(hipStreamSynchronize(s));
  return DMRG_OK;
}

int kernel_prec(dmrg_prec p) {
  return p == DMRG_FP32 ? kPrecF32 : (p == DMRG_BF16X3 ? kPrecBF16X3 : kPrecF64);
}

bool uses32(dmrg_prec p) { return p == DMRG_FP32 || p == DMRG_BF16X3; }

hipError_t take_event(dmrg_ctx c, hipEvent_t* e) {
  if (!c->spare.empty()) {
    *e = c->spare.back();
    c->spare.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// The fused product in kernel precision kp.  The FP32 and BF16 kernels read
// psi as an FP32 copy in the plan's staging buffer (kPoolPad elements of
// room past the end, so that their vector loads stay inside it): psi32, if
// given, already holds it; otherwise psi is converted into it first.  The
// event pair, if any, brackets the product alone.
//
// Variant 1 (FP32 / BF16, when the macro plan is staged) runs the macro-tile
// kernels with their partial tiles in `part` if given, else in the plan's
// own buffer.

dmrg_status launch_fused(Staged& st, int kp, int variant, const void* dense, const double* psi,
                         double* y, double alpha, double beta, hipStream_t s, hipEvent_t t0,
                         hipEvent_t t1, const float* psi32 = nullptr, float* part = nullptr) {
  const int32_t* wgs = st.nwg > 0 ? st.wg_start.as<int32_t>() : nullptr;
  if (kp == kPrecF64) {
    HIP_TRY(launch_hpsi(kp, 0, st.nslots, st.images.as<uint32_t>(), st.img_stride, dense, psi, y,
                        alpha, beta, s, t0, t1, nullptr, 0, 0, wgs, st.nwg));
    return DMRG_OK;
  }
  const bool mac = variant == 1 && st.has_mac;
  const int64_t n = st.plan.D_in + kPoolPad;
  if (!psi32) {
    HIP_TRY(st.psi32.ensure((size_t)n * sizeof(float)));
    HIP_TRY(launch_psi_to_f32(psi, st.psi32.as<float>(), st.plan.D_in, s));
    psi32 = st.psi32.as<float>();
  }
  const int64_t ndense = (int64_t)st.plan.dense.size() + kPoolPad;
  if (mac) {
    HIP_TRY(launch_hpsi_macro(kp == kPrecBF16X3, st.mac_nwg, st.mac_nshared, st.mtiles.as<MacTile>(),
                              st.msegs.as<MacSeg>(), st.mggs.as<MacGG>(), st.mitems.as<MacItem>(),
                              st.mwg.as<int32_t>(), st.mshared.as<int32_t>(), st.mdense.as<float>(),
                              st.mac_ndense, psi32, n, psi, y, alpha, beta, part ? part : st.mpart.as<float>(), s,
                              t0, t1));
    return DMRG_OK;
  }
  HIP_TRY(launch_hpsi(kp, 0, st.nslots, st.images.as<uint32_t>(), st.img_stride, dense, psi, y, alpha, beta,
                      s, t0, t1, psi32, ndense, n, wgs, st.nwg));
  return DMRG_OK;
}

dmrg_status run_product_inner(dmrg_sb sb, Staged& st, dmrg_prec prec, const double* psi, double* y,
                              double alpha, double beta, hipEvent_t t0, hipEvent_t t1,
                              const float* psi32);

// y = alpha H psi + beta y with a given plan and precision (timed if asked).
// psi32, if given, already holds psi in FP32 with the padding the FP32 and
// BF16 products read (used by those precisions only).
dmrg_status run_product(dmrg_sb sb, Staged& st, dmrg_prec prec, const double* psi, double* y,
                        double alpha, double beta, const float* psi32 = nullptr) {
  dmrg_ctx c = sb->ctx;
  if (c->timing <= 0) return run_product_inner(sb, st, prec, psi, y, alpha, beta, nullptr, nullptr, psi32);
  if ((int)prec >= 0 && (int)prec < 4) ++c->products[(int)prec];
  if (c->tick++ % c->timing != 0)
    return run_product_inner(sb, st, prec, psi, y, alpha, beta, nullptr, nullptr, psi32);
  dmrg_ctx_s::Mark mk;
  HIP_TRY(take_event(c, &mk.a));
  HIP_TRY(take_event(c, &mk.b));
  mk.prec = (int)prec;
  dmrg_status st2 = run_product_inner(sb, st, prec, psi, y, alpha, beta, mk.a, mk.b, psi32);
  c->marks.push_back(mk);
  return st2;
}

dmrg_status run_product_inner(dmrg_sb sb, Staged& st, dmrg_prec prec, const double* psi, double* y,
                              double alpha, double beta, hipEvent_t t0, hipEvent_t t1,
                              const float* psi32) {
  hipStream_t s = sb->ctx->stream;
  const Plan& p = st.plan;
  if (prec == DMRG_FP64_PLAIN) {
    if (t0) HIP_TRY(hipEventRecord(t0, s));
    HIP_TRY(launch_plain(st.plain, p.D, st.dense64.as<double>(), st.gsrc.as<int32_t>(),
                         st.gscale.as<double>(), psi, y, alpha, beta, s));
    if (t1) HIP_TRY(hipEventRecord(t1, s));
    return DMRG_OK;
  }
  const void* dense = st.dense64.p;
  if (uses32(prec)) {
    if (!st.has32) return fail(DMRG_E_ARG, "FP32 operators not staged (use dmrg_sb_set_prec)");
    dense = st.dense32.p;
  }
  const int kp = kernel_prec(prec);
  return launch_fused(st, kp, sb->variant[kp], dense, psi, y, alpha, beta, s, t0, t1, psi32);
}

dmrg_status need_device(dmrg_sb sb) {
  if (sb == nullptr) return fail(DMRG_E_ARG, "null superblock");
  if (sb->ctx == nullptr) return fail(DMRG_E_DEVICE, "superblock was built without a device context");
  return DMRG_OK;
}

dmrg_status need_square(dmrg_sb sb) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (sb->q_in != sb->q_target)
    return fail(DMRG_E_ARG, "this call needs a Hamiltonian (input sector == output sector)");
  return DMRG_OK;
}

std::vector<dmrg_term> term_views(dmrg_sb sb) {
  std::vector<dmrg_term> t(sb->coeff.size());
  for (size_t k = 0; k < t.size(); ++k) {
    t[k].c = sb->coeff[k];
    t[k].group = sb->group[k];
    t[k].A = sb->opA[k] ? &sb->opA[k]->view : nullptr;
    t[k].B = sb->opB[k] ? &sb->opB[k]->view : nullptr;
  }
  return t;
}

dmrg_basis basis_view(const std::vector<int64_t>& q, const std::vector<int32_t>& d) {
  dmrg_basis b;
  b.nsec = (int32_t)q.size();
  b.q = q.data();
  b.dim = d.data();
  return b;
}

std::unique_ptr<OpCopy> copy_op(const dmrg_op* op, const dmrg_basis* b) {
  if (op == nullptr) return nullptr;
  auto c = std::make_unique<OpCopy>();
  c->delta = op->delta;
  for (int32_t k = 0; k < op->nblk; ++k) {
    c->row.push_back(op->row_sec[k]);
    c->col.push_back(op->col_sec[k]);
    const size_t n = (size_t)b->dim[op->row_sec[k]] * b->dim[op->col_sec[k]];
    c->data.emplace_back(op->blk[k], op->blk[k] + n);
  }
  for (auto& d : c->data) c->ptrs.push_back(d.data());
  c->view.delta = c->delta;
  c->view.nblk = (int32_t)c->row.size();
  c->view.row_sec = c->row.data();
  c->view.col_sec = c->col.data();
  c->view.blk = c->ptrs.data();
  return c;
}

}  // namespace

extern "C" {

const char* dmrg_last_error(void) { return g_err.c_str(); }

const char* dmrg_version(void) { return "libdmrg 0.1 (gfx950)"; }

dmrg_status dmrg_ctx_create(int device, void* hip_stream, dmrg_ctx* out) {
  if (out == nullptr) return fail(DMRG_E_ARG, "null output pointer");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(DMRG_E_DEVICE, "no HIP device");
  if (device < 0 || device >= n) return fail(DMRG_E_ARG, "device index out of range");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DMRG_E_DEVICE, std::string("libdmrg is built for gfx950, device is ") + prop.gcnArchName);
  {
    // the fixed scratch of dmrg_hpsi_noalloc on this device
    DeviceGuard g(device);
    if (!g.ok) return fail(DMRG_E_DEVICE, "hipSetDevice failed");
    HIP_TRY(scratch_setup(device));
  }
  auto* c = new dmrg_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  return DMRG_OK;
}

void dmrg_ctx_destroy(dmrg_ctx ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& mk : ctx->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  for (auto e : ctx->spare) (void)hipEventDestroy(e);
  for (auto e : ctx->chk)
    if (e) (void)hipEventDestroy(e);
  if (ctx->host_small) (void)hipHostFree(ctx->host_small);
  if (ctx->host_rho) (void)hipHostFree(ctx->host_rho);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

dmrg_status dmrg_ctx_set_timing(dmrg_ctx ctx, int32_t every) {
  if (!ctx) return fail(DMRG_E_ARG, "null context");
  if (every < 0) return fail(DMRG_E_ARG, "timing stride must be >= 0");
  ctx->timing = every;
  ctx->tick = 0;
  return DMRG_OK;
}

dmrg_status dmrg_ctx_timing(dmrg_ctx ctx, int32_t prec, double* ms_total, int64_t* launches,
                            int64_t* products, int32_t reset) {
  if (!ctx || !ms_total || !launches) return fail(DMRG_E_ARG, "null argument");
  DeviceGuard g(ctx->device);
  double tot = 0.0;
  int64_t n = 0;
  if (!ctx->marks.empty()) HIP_TRY(hipEventSynchronize(ctx->marks.back().b));
  for (auto& mk : ctx->marks) {
    if (mk.prec != prec) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, mk.a, mk.b));
    tot += ms;
    ++n;
  }
  *ms_total = tot;
  *launches = n;
  if (products) *products = (prec >= 0 && prec < 4) ? ctx->products[prec] : 0;
  if (reset) {
    for (auto& mk : ctx->marks) {
      ctx->spare.push_back(mk.a);
      ctx->spare.push_back(mk.b);
    }
    ctx->marks.clear();
    for (auto& c : ctx->products) c = 0;
  }
  return DMRG_OK;
}

dmrg_status dmrg_ctx_set_stream(dmrg_ctx ctx, void* hip_stream) {
  if (!ctx) return fail(DMRG_E_ARG, "null context");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return DMRG_OK;
}

dmrg_status dmrg_ctx_set_mem_cap(dmrg_ctx ctx, int64_t bytes) {
  if (!ctx) return fail(DMRG_E_ARG, "null context");
  if (bytes < 0) return fail(DMRG_E_ARG, "memory cap must be >= 0");
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(DMRG_E_DEVICE, "device index out of range");
  g_mem[ctx->device].cap.store(bytes);
  return DMRG_OK;
}

dmrg_status dmrg_ctx_mem(dmrg_ctx ctx, int64_t* used, int64_t* cap) {
  if (!ctx) return fail(DMRG_E_ARG, "null context");
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(DMRG_E_DEVICE, "device index out of range");
  if (used) *used = g_mem[ctx->device].used.load();
  if (cap) *cap = g_mem[ctx->device].cap.load();
  return DMRG_OK;
}

static dmrg_status build_sb(dmrg_ctx ctx, const dmrg_basis* S, const dmrg_basis* E, int64_t q_in,
                            int64_t q_target, int32_t nterms, const dmrg_term* terms,
                            dmrg_prec prec, dmrg_sb* out) {
  if (out == nullptr) return fail(DMRG_E_ARG, "null output pointer");
  if (prec < DMRG_FP64 || prec > DMRG_FP64_PLAIN) return fail(DMRG_E_ARG, "unknown precision");
  auto sb = std::make_unique<dmrg_sb_s>();
  std::string err;
  dmrg_status st = build_plan_between(S, E, q_in, q_target, nterms, terms, false, sb->fwd.plan, err);
  if (st != DMRG_OK) return fail(st, err);
  sb->q_in = q_in;
  sb->ctx = ctx;
  if (ctx) {
    sb->device = ctx->device;
    sb->stream = ctx->stream;
  }
  sb->prec = prec;
  sb->qS.assign(S->q, S->q + S->nsec);
  sb->qE.assign(E->q, E->q + E->nsec);
  sb->dS.assign(S->dim, S->dim + S->nsec);
  sb->dE.assign(E->dim, E->dim + E->nsec);
  sb->q_target = q_target;
  for (int32_t k = 0; k < nterms; ++k) {
    sb->coeff.push_back(terms[k].c);
    sb->group.push_back(terms[k].group);
    sb->opA.push_back(copy_op(terms[k].A, S));
    sb->opB.push_back(copy_op(terms[k].B, E));
  }
  if (ctx) {
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(DMRG_E_DEVICE, "hipSetDevice failed");
    if ((st = stage(ctx, sb->fwd, uses32(prec))) != DMRG_OK) return st;
  }
  *out = sb.release();
  return DMRG_OK;
}

dmrg_status dmrg_build_superblock(dmrg_ctx ctx, const dmrg_basis* S, const dmrg_basis* E,
                                  int64_t q_target, int32_t nterms, const dmrg_term* terms,
                                  dmrg_prec prec, dmrg_sb* out) {
  return build_sb(ctx, S, E, q_target, q_target, nterms, terms, prec, out);
}

dmrg_status dmrg_build_operator(dmrg_ctx ctx, const dmrg_basis* S, const dmrg_basis* E,
                                int64_t q_in, int64_t q_out, int32_t nterms,
                                const dmrg_term* terms, dmrg_prec prec, dmrg_sb* out) {
  return build_sb(ctx, S, E, q_in, q_out, nterms, terms, prec, out);
}

dmrg_status dmrg_sb_dims(dmrg_sb sb, int64_t* D_in, int64_t* D_out) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  if (D_in) *D_in = sb->fwd.plan.D_in;
  if (D_out) *D_out = sb->fwd.plan.D;
  return DMRG_OK;
}

void dmrg_sb_destroy(dmrg_sb sb) {
  if (!sb) return;
  if (sb->device >= 0) {
    DeviceGuard g(sb->device);
    (void)hipStreamSynchronize(sb->stream);
    delete sb;
  } else {
    delete sb;
  }
}

dmrg_status dmrg_sb_layout(dmrg_sb sb, int64_t* D, int32_t* npairs, const int64_t** off,
                           const int32_t** s_sec, const int32_t** e_sec) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  const Plan& p = sb->fwd.plan;
  if (D) *D = p.D;
  if (npairs) *npairs = (int32_t)p.pair_s.size();
  if (off) *off = p.pair_off.data();
  if (s_sec) *s_sec = p.pair_s.data();
  if (e_sec) *e_sec = p.pair_e.data();
  return DMRG_OK;
}

dmrg_status dmrg_sb_stats(dmrg_sb sb, double* flops_alg, double* flops_exec, double* bytes_alg,
                          int32_t* ntiles) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  const Plan& p = sb->fwd.plan;
  const int elem = uses32(sb->prec) ? 4 : 8;
  if (flops_alg) *flops_alg = p.flops_alg;
  if (flops_exec) *flops_exec = p.flops_exec;
  if (bytes_alg) *bytes_alg = plan_bytes_alg(p, elem);
  if (ntiles) *ntiles = (int32_t)p.tiles.size();
  return DMRG_OK;
}

dmrg_status dmrg_sb_set_coeffs(dmrg_sb sb, const double* c_h) {
  if (!sb || !c_h) return fail(DMRG_E_ARG, "null argument");
  for (size_t k = 0; k < sb->coeff.size(); ++k) sb->coeff[k] = c_h[k];
  Staged* plans[2] = {&sb->fwd, sb->adj.get()};
  const int32_t nt = (int32_t)sb->coeff.size();
  for (Staged* st : plans) {
    if (!st) continue;
    // host copies (images rebuilt later, the plain path's launch arguments)
    for (auto& s : st->plan.segs) s.c = c_h[s.term];
    for (auto& w : st->plain) w.first.c = c_h[w.first.term];
    // device copies: written in place, in stream order, by a small kernel
    if (sb->ctx) {
      DeviceGuard g(sb->ctx->device);
      HIP_TRY(launch_patch_coeffs(st->images.p, st->coef_img.as<CoefRef>(), st->ncoef_img,
                                  sb->coeff.data(), nt, sb->ctx->stream));
      HIP_TRY(launch_patch_coeffs(st->segs.p, st->coef_seg.as<CoefRef>(), st->ncoef_seg,
                                  sb->coeff.data(), nt, sb->ctx->stream));
      if (st->has_mac) {
        HIP_TRY(launch_patch_coeffs(st->msegs.p, st->mcoef_seg.as<CoefRef>(), st->ncoef_mseg,
                                    sb->coeff.data(), nt, sb->ctx->stream));
        HIP_TRY(launch_patch_coeffs(st->mggs.p, st->mcoef_gg.as<CoefRef>(), st->ncoef_mgg,
                                    sb->coeff.data(), nt, sb->ctx->stream));
      }
    }
  }
  return DMRG_OK;
}

dmrg_status dmrg_sb_set_prec(dmrg_sb sb, dmrg_prec prec) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  if (prec < DMRG_FP64 || prec > DMRG_FP64_PLAIN) return fail(DMRG_E_ARG, "unknown precision");
  if (uses32(prec) && sb->ctx && !sb->fwd.has32) {
    DeviceGuard g(sb->ctx->device);
    std::vector<float> f;
    dense_f32(sb->fwd.plan, f);
    dmrg_status r = upload(sb->fwd.dense32, f.data(), f.size() * sizeof(float), sb->ctx->stream);
    if (r != DMRG_OK) return r;
    HIP_TRY(hipStreamSynchronize(sb->ctx->stream));
    sb->fwd.has32 = true;
  }
  sb->prec = prec;
  return DMRG_OK;
}

dmrg_status dmrg_sb_autotune(dmrg_sb sb, int32_t reps, int32_t* variant) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (reps < 1) return fail(DMRG_E_ARG, "reps must be >= 1");
  const int kp = kernel_prec(sb->prec);
  if (sb->prec == DMRG_FP64 || sb->prec == DMRG_FP64_PLAIN) {
    if (variant) *variant = 0;
    return DMRG_OK;
  }
  if (!sb->fwd.has32) return fail(DMRG_E_ARG, "FP32 operators not staged (use dmrg_sb_set_prec)");
  DeviceGuard g(sb->ctx->device);
  hipStream_t s = sb->ctx->stream;
  Staged& stg = sb->fwd;
  if ((st = ensure_macro(stg, s)) != DMRG_OK) return st;
  DevBuf x, y;
  HIP_TRY(x.ensure((size_t)std::max<int64_t>(stg.plan.D_in, 1) * sizeof(double)));
  HIP_TRY(y.ensure((size_t)std::max<int64_t>(stg.plan.D, 1) * sizeof(double)));
  HIP_TRY(hipMemsetAsync(x.p, 0, (size_t)stg.plan.D_in * sizeof(double), s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.f;
  hipError_t err = hipSuccess;
  for (int v = 0; v < kVariants && err == hipSuccess; ++v) {
    if (v == 1 && !stg.has_mac) continue;
    auto go = [&]() {
      return launch_fused(sb->fwd, kp, v, stg.dense32.p, x.as<double>(), y.as<double>(), 1.0, 0.0, s,
                          nullptr, nullptr) == DMRG_OK
                 ? hipSuccess
                 : hipErrorUnknown;
    };
    for (int w = 0; w < 2 && err == hipSuccess; ++w) err = go();
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = go();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && (v == 0 || ms < best_ms)) {
      best = v;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(err);
  sb->variant[kp] = best;
  if (variant) *variant = best;
  return DMRG_OK;
}

dmrg_status dmrg_sb_set_variant(dmrg_sb sb, int32_t variant) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  if (variant < 0 || variant >= kVariants) return fail(DMRG_E_ARG, "unknown kernel variant");
  if (variant == 1 && sb->ctx) {
    DeviceGuard g(sb->ctx->device);
    const dmrg_status st = ensure_macro(sb->fwd, sb->ctx->stream);
    if (st != DMRG_OK) return st;
  }
  sb->variant[kernel_prec(sb->prec)] = variant;
  return DMRG_OK;
}

dmrg_status dmrg_sb_set_reorth(dmrg_sb sb, int32_t mode) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  if (mode != 0 && mode != 1) return fail(DMRG_E_ARG, "reorthogonalisation mode must be 0 or 1");
  sb->reorth = mode;
  return DMRG_OK;
}

dmrg_status dmrg_sb_set_graphs(dmrg_sb sb, int32_t enable) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (enable != 0 && enable != 1) return fail(DMRG_E_ARG, "enable must be 0 or 1");
  sb->lzg.on = enable == 1;
  if (!sb->lzg.on) {
    DeviceGuard g(sb->ctx->device);
    HIP_TRY(hipStreamSynchronize(sb->ctx->stream));   // no replay of them is still queued
    sb->lzg.drop();
  }
  return DMRG_OK;
}

dmrg_status dmrg_sb_graph_stats(dmrg_sb sb, int64_t* captures, int64_t* replays) {
  if (!sb) return fail(DMRG_E_ARG, "null superblock");
  if (captures) *captures = sb->lzg.captures;
  if (replays) *replays = sb->lzg.replays;
  return DMRG_OK;
}

dmrg_status dmrg_hpsi(dmrg_sb sb, const double* psi_d, double* y_d, double alpha, double beta) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (!psi_d || !y_d) return fail(DMRG_E_ARG, "null vector");
  if (psi_d == y_d) return fail(DMRG_E_ARG, "psi and y must not overlap");
  DeviceGuard g(sb->ctx->device);
  return run_product(sb, sb->fwd, sb->prec, psi_d, y_d, alpha, beta);
}

dmrg_status dmrg_hpsi_noalloc(dmrg_sb sb, const double* psi_d, double* y_d, double alpha, double beta) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (!psi_d || !y_d) return fail(DMRG_E_ARG, "null vector");
  if (psi_d == y_d) return fail(DMRG_E_ARG, "psi and y must not overlap");
  DeviceGuard g(sb->ctx->device);
  hipStream_t s = sb->ctx->stream;
  Staged& f = sb->fwd;
  const Plan& p = f.plan;
  if (sb->prec == DMRG_FP64_PLAIN) {
    HIP_TRY(launch_plain(f.plain, p.D, f.dense64.as<double>(), f.gsrc.as<int32_t>(), f.gscale.as<double>(),
                         psi_d, y_d, alpha, beta, s));
    return DMRG_OK;
  }
  const int kp = kernel_prec(sb->prec);
  if (kp == kPrecF64)
    return launch_fused(f, kp, sb->variant[kp], f.dense64.p, psi_d, y_d, alpha, beta, s, nullptr, nullptr);
  if (!f.has32) return fail(DMRG_E_ARG, "FP32 operators not staged (use dmrg_sb_set_prec)");
  float* buf = scratch_ptr(sb->ctx->device);
  if (!buf) return fail(DMRG_E_DEVICE, "the fixed scratch was not set up on this device");
  if (p.D_in + kPoolPad > kScratchFloats) {
    std::ostringstream os;
    os << "dmrg_hpsi_noalloc: the input vector (" << p.D_in << " elements, plus " << kPoolPad
       << " of padding) exceeds the fixed scratch of " << kScratchFloats << " floats";
    return fail(DMRG_E_NOMEM, os.str());
  }
  // the macro-tile variant's partial tiles follow psi in the scratch; when
  // they do not fit, the 32 x 32 tile kernel runs instead
  int variant = sb->variant[kp];
  const int64_t psi_room = (p.D_in + kPoolPad + 63) / 64 * 64;
  const int64_t need = psi_room + (int64_t)f.mac_nparts * kMac * kMac;
  if (variant == 1 && (!f.has_mac || need > kScratchFloats)) variant = 0;
  HIP_TRY(launch_psi_to_f32(psi_d, buf, p.D_in, s));
  return launch_fused(f, kp, variant, f.dense32.p, psi_d, y_d, alpha, beta, s, nullptr, nullptr, buf,
                      variant == 1 ? buf + psi_room : nullptr);
}

dmrg_status dmrg_hpsi_adjoint(dmrg_sb sb, const double* psi_d, const double* g_d, double* gpsi_d,
                              double* gc_h) {
  dmrg_status st = need_device(sb);
  if (st != DMRG_OK) return st;
  if (!psi_d || !g_d) return fail(DMRG_E_ARG, "null vector");
  DeviceGuard guard(sb->ctx->device);
  hipStream_t s = sb->ctx->stream;
  if (gpsi_d) {
    if (gpsi_d == g_d) return fail(DMRG_E_ARG, "g and grad_psi must not overlap");
    if (!sb->adj) {
      auto adj = std::make_unique<Staged>();
      std::string err;
      dmrg_basis bS = basis_view(sb->qS, sb->dS), bE = basis_view(sb->qE, sb->dE);
      std::vector<dmrg_term> tv = term_views(sb);
      st = build_plan_between(&bS, &bE, sb->q_in, sb->q_target, (int32_t)tv.size(), tv.data(), true,
                              adj->plan, err);
      if (st != DMRG_OK) return fail(st, "adjoint plan: " + err);
      if ((st = stage(sb->ctx, *adj, sb->fwd.has32)) != DMRG_OK) return st;
      sb->adj = std::move(adj);
    }
    dmrg_prec p = sb->prec;
    if (uses32(p) && !sb->adj->has32) p = DMRG_FP64;
    if ((st = run_product(sb, *sb->adj, p, g_d, gpsi_d, 1.0, 0.0)) != DMRG_OK) return st;
  }
  if (gc_h) {
    Staged& f = sb->fwd;
    const int nt = (int)f.plan.tiles.size();
    const int stride = std::max(1, f.max_nseg);
    DevBuf part;
    HIP_TRY(part.ensure((size_t)nt * stride * sizeof(double)));
    const bool use32 = uses32(sb->prec) && f.has32;
    HIP_TRY(launch_term_dots(use32 ? kPrecF32 : kPrecF64, nt, f.tiles.as<TileDesc>(),
                             f.segs.as<SegDesc>(), use32 ? f.dense32.p : f.dense64.p,
                             f.gsrc.as<int32_t>(), f.gscale.as<double>(), psi_d, g_d,
                             part.as<double>(), stride, s));
    std::vector<double> h((size_t)nt * stride);
    HIP_TRY(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<double> acc(sb->coeff.size(), 0.0);
    for (int t = 0; t < nt; ++t) {
      const TileDesc& td = f.plan.tiles[t];
      for (int q = 0; q < td.nseg; ++q) acc[f.plan.segs[td.seg0 + q].term] += h[(size_t)t * stride + q];
    }
    for (size_t k = 0; k < acc.size(); ++k) gc_h[k] = acc[k];
  }
  return DMRG_OK;
}

dmrg_status dmrg_lanczos_ground(dmrg_sb sb, const double* psi0_d, int32_t max_iter, double tol,
                                double* E0_h, double* psi_d, int32_t* iters_h, double* resid_h) {
  dmrg_status st = need_square(sb);
  if (st != DMRG_OK) return st;
  if (!psi0_d || !psi_d || !E0_h) return fail(DMRG_E_ARG, "null argument");
  if (max_iter < 1 || !(tol >= 0.0)) return fail(DMRG_E_ARG, "max_iter must be >= 1 and tol >= 0");
  dmrg_ctx ctx = sb->ctx;
  DeviceGuard guard(ctx->device);
  hipStream_t s = ctx->stream;
  const int64_t D = sb->fwd.plan.D;
  const bool reduced = sb->prec == DMRG_FP32 || sb->prec == DMRG_BF16X3;
  // vectors per restart cycle; the host looks at alpha/beta every kCheck steps
  const int per_cycle = reduced ? 100 : std::min<int>(max_iter, 400);
  const int nvec = per_cycle + 1;
  constexpr int kCheck = 4;
  const size_t npart = std::max(lz_partial_size(D, nvec), (size_t)vec_blocks(D));
  const size_t nnorm = lz_norm_partials(D);
  HIP_TRY(ctx->V.ensure((size_t)nvec * D * sizeof(double)));
  HIP_TRY(ctx->w.ensure((size_t)D * sizeof(double)));
  HIP_TRY(ctx->partial.ensure((npart + 2 * nnorm) * sizeof(double)));
  // small: h1[nvec], h2[nvec], u[nvec], nrm2[8], ab[2*nvec], scale[8]
  const size_t nsmall = (size_t)5 * nvec + 16;
  HIP_TRY(ctx->small.ensure(nsmall * sizeof(double)));
  HIP_TRY(hipMemsetAsync(ctx->small.p, 0, nsmall * sizeof(double), s));
  // host: the two check buffers of (alpha, beta), the Ritz coefficients and
  // the two buffers of a check's norm partials
  const size_t nhost = nsmall + 2 * nnorm;
  if (ctx->host_small_n < nhost) {
    if (ctx->host_small) (void)hipHostFree(ctx->host_small);
    ctx->host_small = nullptr;
    HIP_TRY(hipHostMalloc((void**)&ctx->host_small, nhost * sizeof(double), hipHostMallocDefault));
    ctx->host_small_n = nhost;
  }
  // reduced precision: the FP32 copy of the next product's input, with the
  // zero padding past its end that the products' masked loads may reach
  float* v32 = nullptr;
  if (reduced) {
    const size_t n32 = (size_t)D + kPoolPad;
    if (ctx->v32_n < n32 || !ctx->v32.p) {
      HIP_TRY(ctx->v32.ensure(n32 * sizeof(float)));
      ctx->v32_n = n32;
    }
    v32 = ctx->v32.as<float>();
    HIP_TRY(hipMemsetAsync(v32 + D, 0, kPoolPad * sizeof(float), s));
  }
  double* V = ctx->V.as<double>();
  double* w = ctx->w.as<double>();
  double* part = ctx->partial.as<double>();
  double* h1 = ctx->small.as<double>();
  double* h2 = h1 + nvec;
  double* ud = h2 + nvec;
  double* nrm2 = ud + nvec;
  double* ab = nrm2 + 8;
  double* scale = ab + 2 * nvec;
  // partial sums of the norm of a single-pass step's (unnormalised) new
  // vector, by step parity: step j writes [j & 1], step j + 1 reads it
  double* npb[2] = {part + npart, part + npart + nnorm};
  double* hs = ctx->host_small;

  // v0 = psi0 / |psi0|
  HIP_TRY(launch_multi_dot(psi0_d, 0, 1, psi0_d, D, part, nrm2, s));
  HIP_TRY(launch_normalise(V, psi0_d, nrm2, D, s));
  int total = 0;
  double E = 0.0, res = INFINITY;
  bool converged = false;
  std::vector<double> alphas, betas, u;
  // The host reads (alpha, beta) every kCheck steps without draining the
  // stream: the copy for a check point goes out behind that step's kernels
  // into one of two pinned buffers, the steps after it are launched, and the
  // check is evaluated one check point later (the first step of a cycle and
  // the last one allowed are evaluated at once).  A cycle that stops at a
  // check leaves at most kCheck further steps queued; their vectors are not
  // used.
  if (!ctx->chk[0]) {
    HIP_TRY(hipEventCreateWithFlags(&ctx->chk[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ctx->chk[1], hipEventDisableTiming));
  }
  double* hbuf[2] = {hs, hs + 2 * nvec};
  double* uh = hs + 4 * nvec;   // Ritz coefficients on their way to the device
  // A single-pass step leaves its beta to the next step.  At a check point
  // the step's norm partials travel with the (alpha, beta) copy and the host
  // adds them in the device's order (the same bits as a device sum, without
  // a launch on the queue); hnp_step[b] is the step whose partials hnp[b]
  // holds, or -1.
  double* hnp[2] = {hs + nsmall, hs + nsmall + nnorm};
  int hnp_step[2] = {-1, -1};
  auto fill_beta = [&](int b) {
    const int jc = hnp_step[b];
    if (jc < 0) return;
    const double t = wave_order_sum(hnp[b], (int)nnorm);
    hbuf[b][2 * jc + 1] = std::sqrt(t > 0.0 ? t : 0.0);
  };
  double prev_ctol = tol;   // tolerance the previous cycle stopped at
  for (int cycle = 0; !converged && total < max_iter; ++cycle) {
    double beta0 = 0.0;
    int nv = 0;      // basis vectors that enter the Ritz vector of this cycle
    u.clear();
    // evaluates the check taken after step jc from h; true: the cycle stops
    double ctol = tol;                   // this cycle's stopping residual
    double est_prev = -1.0, est_last = -1.0;   // the last two evaluated estimates
    // The first step of a cycle orthogonalises by classical Gram-Schmidt
    // twice.  After it, odd steps subtract the local three-term recurrence
    // (alpha_j V_j + beta_{j-1} V_{j-1}) and run one Gram-Schmidt pass on
    // the remainder (two passes over the basis instead of three); even steps
    // subtract the recurrence alone and do not touch the rest of the basis.
    // A pass on every other step keeps the basis semi-orthogonal (periodic
    // reorthogonalisation in the sense of Grcar and of Simon's analysis of
    // semi-orthogonal Lanczos bases): the loss of orthogonality that one
    // recurrence-only step lets grow is removed by the next pass before it
    // is amplified again, so the overlaps stay near 1e-7 with reduced
    // precision products (two recurrence-only steps in a row let them grow
    // geometrically).  Every cycle's result is certified by the FP64
    // residual of the next cycle's first step.  A basis that is not small
    // against the dimension always runs two full passes: the Krylov space may
    // be exhausted (or confined to a small invariant subspace) within the
    // cycle, and only they leave the vanishing beta that ends the recursion
    // there.
    constexpr int64_t kOncePassMinRatio = 32;   // D >= 32 * vectors per cycle
    const bool twice = sb->reorth == 1 || D < kOncePassMinRatio * nvec;
    auto evaluate = [&](int jc, const double* h) {
      alphas.clear();
      betas.clear();
      // the recursion is valid up to the first vanishing beta
      for (int m = 0; m <= jc; ++m) {
        alphas.push_back(h[2 * m]);
        const double b = h[2 * m + 1];
        betas.push_back(b);
        if (b <= 1e-13 * std::max(1.0, std::fabs(h[2 * m]))) break;
      }
      const int steps = (int)alphas.size();
      if (jc == 0) {
        E = alphas[0];
        res = betas[0];
        beta0 = betas[0];
        // a reduced-precision cycle stops at a fraction of its starting
        // (FP64) residual that its products can still resolve: FP32 products
        // carry about 1e-7 relative error, the BF16 split about 1e-5
        // (measured: 1e-5 for FP32 takes 81 products to the headline ground
        // state where 1e-4 takes 85 and 1e-6 85)
        ctol = reduced ? std::max(tol, (sb->prec == DMRG_FP32 ? 1e-5 : 1e-4) * beta0) : tol;
        if (res <= tol) {
          converged = true;
          nv = 1;
          return true;
        }
      }
      double theta;
      u.assign(steps, 0.0);
      tridiag_lowest(steps, alphas.data(), betas.data(), &theta, u.data());
      nv = steps;
      const double bl = betas[steps - 1];
      const double est = bl * std::fabs(u[steps - 1]);
      if (jc > 0) {
        est_prev = est_last;
        est_last = est;
      }
      const bool breakdown = bl <= 1e-13 * std::max(1.0, std::fabs(theta)) || steps < jc + 1;
      return jc > 0 && (est <= ctol || breakdown);
    };
    // The launches of step j (product, then the orthogonalisation of its
    // kind); at a check point also the norm record the check reads.  Under
    // capture the product takes no timing events.
    auto issue_step = [&](int j, bool check, bool capture, hipStream_t s) -> dmrg_status {
      double* vj = V + (size_t)j * D;
      const dmrg_prec p = (j == 0 && reduced) ? DMRG_FP64 : sb->prec;
      const bool two = j == 0 || twice;
      const bool recurrence = !two && !(j & 1);
      // a reduced-precision product reads the FP32 copy of its input that the
      // previous step wrote beside it (no conversion pass)
      const float* in32 = p == sb->prec ? v32 : nullptr;
      dmrg_status r = capture ? run_product_inner(sb, sb->fwd, p, vj, w, 1.0, 0.0, nullptr, nullptr, in32)
                              : run_product(sb, sb->fwd, p, vj, w, 1.0, 0.0, in32);
      if (r != DMRG_OK) return r;
      double* vnext = j + 1 < nvec ? V + (size_t)(j + 1) * D : nullptr;
      if (two) {
        HIP_TRY(launch_lz_step(w, V, D, j + 1, D, h1, h2, part, ab + 2 * j, vnext, s, v32));
      } else if (!recurrence) {
        // the recurrence and one pass against the basis; the new vector
        // stays unnormalised until the next step, which normalises it in
        // place (no separate finishing launch)
        HIP_TRY(launch_lz_step_onepass(w, V, D, j + 1, D, h1, part, j >= 2 ? npb[(j - 1) & 1] : nullptr,
                                       j >= 2 ? nullptr : ab + 2 * (j - 1) + 1, npb[j & 1], scale,
                                       ab + 2 * j, vnext, s, v32));
      } else {
        // the recurrence alone
        HIP_TRY(launch_lz_step_recurrence(w, V, D, j + 1, D, part, npb[(j - 1) & 1], npb[j & 1],
                                          ab + 2 * j, vnext, s, v32));
      }
      (void)check;   // a single-pass step's beta_j is formed by the next step, or
                     // by the host from the partials copied at a check point
      return DMRG_OK;
    };
    // Steps j0 .. j1 (no check point before j1, none of them the last step
    // allowed) from the graph of their position, captured on first use.
    auto replay = [&](int j0, int j1) -> dmrg_status {
      dmrg_sb_s::LzGraphs& G = sb->lzg;
      dmrg_sb_s::LzGraphs::Key k;
      std::memset(&k, 0, sizeof(k));
      const Staged& f = sb->fwd;
      const void* ptrs[8] = {V, w, part, h1, v32, f.images.p, f.dense32.p, f.mtiles.p};
      std::copy(ptrs, ptrs + 8, k.ptr);
      k.D = D;
      k.nvec = nvec;
      k.prec = (int32_t)sb->prec;
      k.variant = sb->variant[kernel_prec(sb->prec)];
      k.twice = twice;
      if (!(k == G.key)) {
        G.drop();
        G.key = k;
      }
      const size_t pos = (size_t)(j0 / kCheck);
      if (G.seg.size() <= pos) G.seg.resize(pos + 1, nullptr);
      if (!G.seg[pos]) {
        // captured on the context's own side stream (the caller's stream may
        // be the default one, which cannot be captured); nothing runs
        // during the capture, and the graph is launched on the caller's
        // stream
        if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->cap_stream;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        ctx->stream = cs;   // the products queue on the context's stream
        dmrg_status r = DMRG_OK;
        for (int j = j0; j <= j1 && r == DMRG_OK; ++j) r = issue_step(j, j == j1, true, cs);
        ctx->stream = s;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (r != DMRG_OK || e != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          if (r != DMRG_OK) return r;
          HIP_TRY(e);
        }
        const hipError_t ei = hipGraphInstantiate(&G.seg[pos], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) G.seg[pos] = nullptr;
        HIP_TRY(ei);
        ++G.captures;
      }
      HIP_TRY(hipGraphLaunch(G.seg[pos], s));
      ++G.replays;
      if (ctx->timing > 0) ctx->products[(int)sb->prec] += j1 - j0 + 1;
      return DMRG_OK;
    };
    int pend = -1, pbuf = 0, nbuf = 0;   // check in flight: its step and buffer
    for (int j = 0;; ++j) {
      int j1 = j;   // last step of a captured run starting at j (== j: none)
      if (sb->lzg.on && j >= 1) {   // a run up to the next check point
        while ((j1 + 1) % kCheck != 0) ++j1;
        if (!(j1 + 2 < nvec && total + (j1 - j + 1) < max_iter) || j1 == j) j1 = j;
      }
      if (j1 > j) {
        if ((st = replay(j, j1)) != DMRG_OK) return st;
        total += j1 - j + 1;
        j = j1;
      } else {
        const bool check = j == 0 || (j + 1) % kCheck == 0 || j + 2 >= nvec || total + 1 >= max_iter;
        if ((st = issue_step(j, check, false, s)) != DMRG_OK) return st;
        ++total;
      }
      const bool last = j + 2 >= nvec || total >= max_iter;
      if (!(j == 0 || (j + 1) % kCheck == 0 || last)) continue;
      HIP_TRY(hipMemcpyAsync(hbuf[nbuf], ab, 2 * (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      hnp_step[nbuf] = -1;
      if (j >= 1 && !twice) {   // step j left its beta pending
        HIP_TRY(hipMemcpyAsync(hnp[nbuf], npb[j & 1], nnorm * sizeof(double), hipMemcpyDeviceToHost, s));
        hnp_step[nbuf] = j;
      }
      HIP_TRY(hipEventRecord(ctx->chk[nbuf], s));
      if (pend >= 0) {   // the previous check: its copy is behind older steps only
        HIP_TRY(hipEventSynchronize(ctx->chk[pbuf]));
        fill_beta(pbuf);
        if (evaluate(pend, hbuf[pbuf])) break;
        pend = -1;
      }
      // When the estimates' last rate of decrease says this check point
      // will meet the cycle's tolerance, it is evaluated at once: one wait
      // for the queue to drain instead of kCheck more steps that would be
      // thrown away.
      const bool likely = est_prev > 0.0 && est_last > 0.0 &&
                          est_last * (est_last / est_prev) <= 4.0 * ctol;
      // The first step of a cycle is checked at once when the cycle may end
      // there: always in the first cycle (the start vector may already be an
      // eigenvector), and after a cycle that ran to the final tolerance.
      // After a cycle that stopped at its own looser tolerance the FP64
      // residual cannot be met yet, so its check is pipelined like the rest.
      if ((j == 0 && (cycle == 0 || prev_ctol <= tol)) || last || likely) {
        HIP_TRY(hipEventSynchronize(ctx->chk[nbuf]));
        fill_beta(nbuf);
        if (evaluate(j, hbuf[nbuf]) || last) break;
      } else {
        pend = j;
        pbuf = nbuf;
      }
      nbuf ^= 1;
    }
    if (converged) break;
    prev_ctol = ctol;
    // Ritz vector of the cycle -> start of the next one.  The coefficients
    // go through pinned memory that no later host work touches before the
    // next cycle's first (synchronous) check, so the queue is not drained.
    std::copy(u.begin(), u.begin() + nv, uh);
    HIP_TRY(hipMemcpyAsync(ud, uh, nv * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_combine(w, V, D, nv, ud, D, s));
    HIP_TRY(launch_multi_dot(w, 0, 1, w, D, part, nrm2, s));
    HIP_TRY(launch_normalise(V, w, nrm2, D, s));
  }
  if (!converged) {
    // the product cap ended the solve inside a cycle: V[0] now holds that
    // cycle's Ritz vector, whose energy and residual the checks never saw
    // (they belong to the cycle's start); one FP64 product gives them
    if ((st = run_product(sb, sb->fwd, DMRG_FP64, V, w, 1.0, 0.0)) != DMRG_OK) return st;
    HIP_TRY(launch_multi_dot(V, 0, 1, w, D, part, nrm2, s));
    HIP_TRY(launch_multi_dot(w, 0, 1, w, D, part, nrm2 + 1, s));
    HIP_TRY(hipMemcpyAsync(hs, nrm2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    E = hs[0];
    res = std::sqrt(std::max(0.0, hs[1] - hs[0] * hs[0]));
  }
  HIP_TRY(hipMemcpyAsync(psi_d, V, (size_t)D * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  *E0_h = E;
  if (iters_h) *iters_h = total;
  if (resid_h) *resid_h = res;
  if (!converged) {
    std::ostringstream os;
    os << "Lanczos did not reach residual " << tol << " in " << max_iter << " products (last " << res << ")";
    return fail(DMRG_E_NOCONV, os.str());
  }
  return DMRG_OK;
}

dmrg_status dmrg_rho_truncate(dmrg_sb sb, const double* psi_d, int32_t side, int32_t m,
                              int32_t no_split, dmrg_trunc* out) {
  dmrg_status st = need_square(sb);
  if (st != DMRG_OK) return st;
  if (!psi_d || !out) return fail(DMRG_E_ARG, "null argument");
  if (side != 0 && side != 1) return fail(DMRG_E_ARG, "side must be 0 (S') or 1 (E')");
  if (m < 0) return fail(DMRG_E_ARG, "m must be >= 0");
  DeviceGuard guard(sb->ctx->device);
  hipStream_t s = sb->ctx->stream;
  const Plan& p = sb->fwd.plan;
  const std::vector<int64_t>& qs = side == 0 ? sb->qS : sb->qE;
  const std::vector<int32_t>& ds = side == 0 ? sb->dS : sb->dE;
  const int nsec = (int)qs.size();
  // rho blocks of the sectors that appear in a target pair, on the matrix
  // cores; the tile images depend only on the plan and are kept per side
  dmrg_sb_s::RhoPlan& rp = sb->rho_plan[side];
  if (!rp.built) {
    rp.off.assign(nsec, -1);
    std::vector<TileDesc> tiles;
    std::vector<SegDesc> segs;
    int64_t total = 0;
    for (size_t q = 0; q < p.pair_s.size(); ++q) {
      const int32_t a = p.dS[p.pair_s[q]], b = p.dE[p.pair_e[q]];
      const int32_t sec = side == 0 ? p.pair_s[q] : p.pair_e[q];
      const int32_t n = side == 0 ? a : b;
      rp.off[sec] = total;
      SegDesc sg{};
      sg.c = 1.0;
      sg.term = 0;
      sg.psi_off = p.pair_off[q];
      sg.psi_ld = b;
      sg.psi_rows = a;
      sg.op_off = p.pair_off[q];
      sg.op_ld = b;
      sg.gA = -1;
      sg.gB = -1;
      if (side == 0) {          // rho[m][n] = sum_k Psi[m][k] Psi[n][k]
        sg.kind = SEG_MK;
        sg.K = b;
      } else {                  // rho[m][n] = sum_k Psi[k][m] Psi[k][n]
        sg.kind = SEG_KN;
        sg.K = a;
      }
      sg.ch0 = 0;
      const int32_t s0 = (int32_t)segs.size();
      segs.push_back(sg);
      for (int32_t m0 = 0; m0 < n; m0 += kTile)
        for (int32_t n0 = 0; n0 < n; n0 += kTile) {
          TileDesc t{};
          t.y_off = total;
          t.a = n;
          t.b = n;
          t.m0 = m0;
          t.n0 = n0;
          t.seg0 = s0;
          t.nseg = 1;
          t.nchunk = (sg.K + kChunk - 1) / kChunk;
          t.ngemm = 1;
          t.ldy = n;
          tiles.push_back(t);
        }
      total += (int64_t)n * n;
    }
    std::vector<uint32_t> img;
    std::string err;
    if (!build_images(tiles, segs, {}, {}, {}, img, rp.stride, err)) return fail(DMRG_E_UNSUPPORTED, err);
    if ((st = upload(rp.images, img.data(), img.size() * sizeof(uint32_t), s)) != DMRG_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));   // the host image vector dies here
    rp.ntiles = (int)tiles.size();
    rp.total = total;
    rp.built = true;
  }
  const std::vector<int64_t>& rho_off = rp.off;
  const int64_t total = rp.total;
  HIP_TRY(sb->rho_out.ensure((size_t)std::max<int64_t>(total, 1) * sizeof(double)));
  HIP_TRY(launch_hpsi(kPrecF64, 0, rp.ntiles, rp.images.as<uint32_t>(), rp.stride, psi_d, psi_d,
                      sb->rho_out.as<double>(), 1.0, 0.0, s));
  dmrg_ctx ctx = sb->ctx;
  if (ctx->host_rho_n < (size_t)std::max<int64_t>(total, 1)) {
    if (ctx->host_rho) (void)hipHostFree(ctx->host_rho);
    ctx->host_rho = nullptr;
    ctx->host_rho_n = 0;
    const size_t want = (size_t)std::max<int64_t>(total, 1);
    HIP_TRY(hipHostMalloc((void**)&ctx->host_rho, want * sizeof(double), hipHostMallocDefault));
    ctx->host_rho_n = want;
  }
  const double* rho = ctx->host_rho;
  if (total > 0)
    HIP_TRY(hipMemcpyAsync(ctx->host_rho, sb->rho_out.p, (size_t)total * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));

  // per-sector FP64 eigen; zero blocks for sectors without a target pair
  struct Ent {
    double lam;      // clamped
    double raw;
    int64_t q;
    int32_t idx;     // position in the sector's decreasing order
    int32_t sec;
  };
  std::vector<Ent> ents;
  std::vector<SymEig>& eig = sb->rho_eig[side];
  eig.resize(nsec);
  const double floor_ = 1e-13, rel_tie = 1e-6;
  // Sectors are independent: all eigenvalues (and the data for the
  // eigenvectors) on host threads, largest sector first; the eigenvectors
  // are formed below for the kept states only.
  std::vector<int> work(nsec);
  for (int i = 0; i < nsec; ++i) work[i] = i;
  std::stable_sort(work.begin(), work.end(), [&](int x, int y) { return ds[x] > ds[y]; });
  std::atomic<int> next(0), bad(0);
  std::string bad_what;
  const int hw = host_threads();
  // While the last sector is still being reduced, the idle threads form the
  // eigenvectors of the leading m entries of the finished sectors (the only
  // ones of theirs that can be kept); the selection below takes those it
  // keeps from there and forms only the rest.  Every vector is formed by the
  // same routine either way, so the result does not depend on the timing.
  struct SpecItem {
    int sec, p0, np;   // positions p0 .. p0 + np - 1 in decreasing order
  };
  std::vector<SpecItem> spec;
  std::vector<int> kspec(nsec, 0), spec_first(nsec, 0);
  std::vector<int64_t> spec_off(nsec, 0);
  std::vector<std::vector<int>> spec_cols(nsec);
  std::unique_ptr<std::atomic<char>[]> spec_done;
  std::unique_ptr<std::atomic<char>[]> finished(new std::atomic<char>[std::max(nsec, 1)]);
  std::unique_ptr<std::atomic<char>[]> failed(new std::atomic<char>[std::max(nsec, 1)]);
  for (int i = 0; i < nsec; ++i) {
    finished[i].store(0, std::memory_order_relaxed);
    failed[i].store(0, std::memory_order_relaxed);
  }
  std::atomic<int> done(0), spec_next(0), spec_ready(0);
  // threads with nothing to do wait here (blocked, not spinning: the host
  // CPUs are shared hardware threads, and a spinning sibling slows the
  // thread still reducing the largest sector)
  std::mutex wait_mu;
  std::condition_variable wait_cv;
  auto wake = [&]() {
    { std::lock_guard<std::mutex> lk(wait_mu); }
    wait_cv.notify_all();
  };
  auto publish = [&]() {
    struct FE {
      double lam;
      int64_t q;
      int sec, pos;
    };
    std::vector<FE> fe;
    for (int s = 0; s < nsec; ++s) {
      if (!finished[s].load(std::memory_order_acquire) || failed[s].load(std::memory_order_relaxed))
        continue;
      const int n = ds[s];
      for (int c = 0; c < n; ++c) {
        const double raw = eig[s].w[n - 1 - c];
        fe.push_back({raw >= floor_ ? raw : 0.0, qs[s], s, c});
      }
    }
    const int top = std::min<int>(std::max(m, 0), (int)fe.size());
    std::nth_element(fe.begin(), fe.begin() + std::max(top - 1, 0), fe.end(),
                     [](const FE& x, const FE& y) {
                       if (x.lam != y.lam) return x.lam > y.lam;
                       if (x.q != y.q) return x.q < y.q;
                       return x.pos < y.pos;
                     });
    for (int i = 0; i < top; ++i) kspec[fe[i].sec] = std::max(kspec[fe[i].sec], fe[i].pos + 1);
    int64_t tot = 0;
    for (int s = 0; s < nsec; ++s) {
      spec_off[s] = tot;
      tot += (int64_t)ds[s] * kspec[s];
      spec_cols[s].resize(kspec[s]);
      for (int c = 0; c < kspec[s]; ++c) spec_cols[s][c] = ds[s] - 1 - c;
    }
    sb->spec_W.resize((size_t)tot);
    for (int w = 0; w < nsec; ++w) {   // largest sectors first
      const int s = work[w];
      spec_first[s] = (int)spec.size();
      for (int p0 = 0; p0 < kspec[s]; p0 += 4) spec.push_back({s, p0, std::min(4, kspec[s] - p0)});
    }
    spec_done.reset(new std::atomic<char>[std::max<size_t>(spec.size(), 1)]);
    for (size_t i = 0; i < spec.size(); ++i) spec_done[i].store(0, std::memory_order_relaxed);
    spec_ready.store(1, std::memory_order_release);
    wake();
  };
  auto solve = [&](int) {
    for (;;) {
      const int w = next.fetch_add(1);
      if (w >= nsec) break;
      const int sec = work[w];
      const int n = ds[sec];
      // the symmetrised block, in a buffer each host thread keeps
      thread_local std::vector<double> A;
      A.assign((size_t)n * n, 0.0);
      if (rho_off[sec] >= 0)
        std::copy(rho + rho_off[sec], rho + rho_off[sec] + (size_t)n * n, A.begin());
      // symmetrise the computed block, in 16 x 16 tiles so that the
      // transposed reads stay in cache
      constexpr int kSym = 16;
      for (int i0 = 0; i0 < n; i0 += kSym)
        for (int j0 = i0; j0 < n; j0 += kSym)
          for (int i = i0; i < std::min(n, i0 + kSym); ++i)
            for (int j = std::max(i + 1, j0); j < std::min(n, j0 + kSym); ++j) {
              const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
              A[(size_t)i * n + j] = A[(size_t)j * n + i] = v;
            }
      if (!sym_eigen_reduce(n, A.data(), eig[sec], 1)) {
        if (bad.fetch_add(1) == 0) {
          int nonfinite = 0;
          double amax = 0.0;
          for (int64_t x = 0; x < (int64_t)n * n; ++x) {
            const double v = rho_off[sec] >= 0 ? rho[rho_off[sec] + x] : 0.0;
            if (!std::isfinite(v)) ++nonfinite;
            else amax = std::max(amax, std::fabs(v));
          }
          std::ostringstream os;
          os << "sector " << sec << " (dimension " << n << ", " << nonfinite
             << " non-finite entries, max |rho| " << amax << ")";
          bad_what = os.str();
        }
        failed[sec].store(1, std::memory_order_relaxed);
      }
      finished[sec].store(1, std::memory_order_release);
      const int d = done.fetch_add(1, std::memory_order_acq_rel) + 1;
      if (d == nsec - 1) publish();
      if (d == nsec) wake();
    }
    // speculative eigenvectors until the last sector is done
    for (;;) {
      if (done.load(std::memory_order_acquire) >= nsec) return;
      if (!spec_ready.load(std::memory_order_acquire)) {
        std::unique_lock<std::mutex> lk(wait_mu);
        wait_cv.wait(lk, [&] {
          return spec_ready.load(std::memory_order_acquire) || done.load(std::memory_order_acquire) >= nsec;
        });
        continue;
      }
      const int i = spec_next.fetch_add(1);
      if (i >= (int)spec.size()) return;
      const SpecItem& it = spec[i];
      sym_eigen_vectors(eig[it.sec], it.np, spec_cols[it.sec].data() + it.p0,
                        sb->spec_W.data() + spec_off[it.sec] + it.p0, kspec[it.sec], 1);
      spec_done[i].store(1, std::memory_order_release);
    }
  };
  HostPool::get().run(std::min(hw, nsec), solve);
  if (bad.load() > 0)
    return fail(DMRG_E_NOCONV, "density-matrix eigen-solve did not converge in " + bad_what);
  // within a sector, position c in decreasing order is ascending index n - 1 - c
  auto val = [&](int sec, int c) { return eig[sec].w[ds[sec] - 1 - c]; };
  for (int sec = 0; sec < nsec; ++sec)
    for (int c = 0; c < ds[sec]; ++c) {
      const double raw = val(sec, c);
      ents.push_back({raw >= floor_ ? raw : 0.0, raw, qs[sec], c, sec});
    }
  const int ntot = (int)ents.size();
  std::vector<int> ord(ntot);
  for (int i = 0; i < ntot; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (ents[x].lam != ents[y].lam) return ents[x].lam > ents[y].lam;
    if (ents[x].q != ents[y].q) return ents[x].q < ents[y].q;
    return ents[x].idx < ents[y].idx;
  });
  std::vector<int> cluster(ntot, 0);
  for (int i = 1; i < ntot; ++i) {
    const double a = ents[ord[i - 1]].lam, b = ents[ord[i]].lam;
    const bool tied = (a == 0.0 && b == 0.0) || std::fabs(a - b) <= rel_tie * std::max(a, b);
    cluster[i] = cluster[i - 1] + (tied ? 0 : 1);
  }
  for (int i = 0; i < ntot;) {
    int e = i;
    while (e < ntot && cluster[e] == cluster[i]) ++e;
    std::stable_sort(ord.begin() + i, ord.begin() + e, [&](int x, int y) {
      if (ents[x].q != ents[y].q) return ents[x].q < ents[y].q;
      return ents[x].idx < ents[y].idx;
    });
    i = e;
  }
  int keep = m >= ntot ? ntot : m;
  int straddle = 0;
  if (keep < ntot && keep > 0) {
    straddle = cluster[keep - 1] == cluster[keep] && ents[ord[keep]].lam > 0.0;
    if (no_split && straddle)
      while (keep < ntot && cluster[keep] == cluster[keep - 1]) ++keep;
  }
  double eps = 0.0;
  for (int i = keep; i < ntot; ++i) eps += ents[ord[i]].lam;
  sb->tr_lambda.clear();
  sb->tr_sec.clear();
  std::vector<std::vector<int>> per(nsec);
  for (int i = 0; i < keep; ++i) {
    const Ent& e = ents[ord[i]];
    sb->tr_lambda.push_back(e.raw);
    sb->tr_sec.push_back(e.sec);
    per[e.sec].push_back(e.idx);
  }
  sb->tr_kps.assign(nsec, 0);
  sb->tr_Wp.assign(nsec, nullptr);
  std::vector<int64_t> woff(nsec, 0);
  // eigenvectors of the kept states: work items of up to four vectors of one
  // sector, shared by the host threads
  std::vector<std::vector<int>> cols(nsec);
  std::vector<std::pair<int, int>> items;
  int64_t wtot = 0;
  for (int sec = 0; sec < nsec; ++sec) {
    std::vector<int>& idx = per[sec];
    std::sort(idx.begin(), idx.end());
    const int n = ds[sec], k = (int)idx.size();
    sb->tr_kps[sec] = k;
    woff[sec] = wtot;
    wtot += (int64_t)n * k;
  }
  sb->tr_W.resize((size_t)wtot);   // every entry is written below
  const bool have_spec = spec_ready.load(std::memory_order_acquire) != 0;
  for (int sec = 0; sec < nsec; ++sec) {
    const int n = ds[sec], k = sb->tr_kps[sec];
    if (k == 0) continue;
    const std::vector<int>& idx = per[sec];
    sb->tr_Wp[sec] = sb->tr_W.data() + woff[sec];
    cols[sec].resize(k);
    for (int c = 0; c < k; ++c) cols[sec][c] = n - 1 - idx[c];
    // the leading kept columns formed while the last sector was reduced
    // (kept positions are 0..k-1 of the sector's decreasing order; the
    // formed ones a prefix of them)
    int avail = 0;
    if (have_spec && kspec[sec] > 0) {
      bool prefix = true;
      for (int c = 0; c < k; ++c) prefix = prefix && idx[c] == c;
      while (prefix && avail < std::min(k, kspec[sec]) &&
             spec_done[spec_first[sec] + avail / 4].load(std::memory_order_acquire))
        avail = std::min(std::min(k, kspec[sec]), avail / 4 * 4 + 4);
      double* dst = sb->tr_W.data() + woff[sec];
      const double* src = sb->spec_W.data() + spec_off[sec];
      for (int r = 0; r < n; ++r)
        std::copy(src + (size_t)r * kspec[sec], src + (size_t)r * kspec[sec] + avail, dst + (size_t)r * k);
    }
    // the rest in work items (two vectors each in large sectors, whose items
    // are the longest)
    const int per_item = n >= 128 ? 2 : 4;
    for (int q0 = avail; q0 < k; q0 += per_item) items.push_back({sec, q0});
  }
  // largest sectors first, so that their (longest) items do not start last
  std::stable_sort(items.begin(), items.end(), [&](const std::pair<int, int>& x,
                                                   const std::pair<int, int>& y) {
    return ds[x.first] > ds[y.first];
  });
  {
    std::atomic<int> it(0);
    auto vecs = [&](int) {
      for (;;) {
        const int w = it.fetch_add(1);
        if (w >= (int)items.size()) return;
        const int sec = items[w].first, q0 = items[w].second;
        const int k = (int)cols[sec].size();
        const int per_item = ds[sec] >= 128 ? 2 : 4;
        sym_eigen_vectors(eig[sec], std::min(per_item, k - q0), cols[sec].data() + q0,
                          sb->tr_W.data() + woff[sec] + q0, k, 1);
      }
    };
    HostPool::get().run(std::min(hw, (int)items.size()), vecs);
  }
  out->trunc_err = eps;
  out->kept = keep;
  out->straddle = straddle;
  out->lambda = sb->tr_lambda.data();
  out->lambda_sec = sb->tr_sec.data();
  out->nsec = nsec;
  out->kept_per_sec = sb->tr_kps.data();
  out->W = sb->tr_Wp.data();
  out->W_all = sb->tr_W.data();
  out->W_total = wtot;
  return DMRG_OK;
}

dmrg_status dmrg_transform_blocks(dmrg_ctx ctx, int32_t nblk, const dmrg_tblock* blocks,
                                  const double* O_d, const double* W_d, double* out_d) {
  if (!ctx) return fail(DMRG_E_ARG, "null context");
  if (nblk < 0 || (nblk > 0 && (!blocks || !O_d || !W_d || !out_d))) return fail(DMRG_E_ARG, "bad argument");
  if (nblk == 0) return DMRG_OK;
  DeviceGuard guard(ctx->device);
  hipStream_t s = ctx->stream;
  // stage 1: U_b = O_b^T Wr_b (cols x kr) in scratch; stage 2: out_b = U_b^T Wc_b
  std::vector<TileDesc> tiles1, tiles2;
  std::vector<SegDesc> segs;
  std::vector<int64_t> uoff(nblk);
  int64_t utot = 0;
  for (int32_t b = 0; b < nblk; ++b) {
    const dmrg_tblock& B = blocks[b];
    if (B.rows < 0 || B.cols < 0 || B.kr < 0 || B.kc < 0) return fail(DMRG_E_ARG, "negative block size");
    if ((B.o_ld > 0 && B.o_ld < B.cols) || (B.out_ld > 0 && B.out_ld < B.kc))
      return fail(DMRG_E_ARG, "leading dimension smaller than the block width");
    uoff[b] = utot;
    utot += (int64_t)B.cols * B.kr;
  }
  for (int32_t b = 0; b < nblk; ++b) {
    const dmrg_tblock& B = blocks[b];
    if (B.rows == 0 || B.cols == 0 || B.kr == 0 || B.kc == 0) continue;
    for (int stage = 0; stage < 2; ++stage) {
      SegDesc sg{};
      sg.kind = SEG_KN;
      sg.c = 1.0;
      sg.gA = -1;
      sg.gB = -1;
      sg.ch0 = 0;
      TileDesc t{};
      if (stage == 0) {   // U[m][n] = sum_k O[k][m] Wr[k][n]
        sg.K = B.rows;
        sg.op_off = B.o_off;
        sg.op_ld = B.o_ld > 0 ? B.o_ld : B.cols;
        sg.psi_off = B.wr_off;
        sg.psi_ld = B.kr;
        sg.psi_rows = B.rows;
        t.y_off = uoff[b];
        t.a = B.cols;
        t.b = B.kr;
        t.ldy = B.kr;
      } else {            // out[m][n] = sum_k U[k][m] Wc[k][n]
        sg.K = B.cols;
        sg.op_off = uoff[b];
        sg.op_ld = B.kr;
        sg.psi_off = B.wc_off;
        sg.psi_ld = B.kc;
        sg.psi_rows = B.cols;
        t.y_off = B.out_off;
        t.a = B.kr;
        t.b = B.kc;
        t.ldy = B.out_ld > 0 ? B.out_ld : B.kc;
      }
      t.seg0 = (int32_t)segs.size();
      t.nseg = 1;
      t.ngemm = 1;
      t.nchunk = (sg.K + kChunk - 1) / kChunk;
      segs.push_back(sg);
      std::vector<TileDesc>& tl = stage == 0 ? tiles1 : tiles2;
      for (int32_t m0 = 0; m0 < t.a; m0 += kTile)
        for (int32_t n0 = 0; n0 < t.b; n0 += kTile) {
          TileDesc tt = t;
          tt.m0 = m0;
          tt.n0 = n0;
          tl.push_back(tt);
        }
    }
  }
  const size_t n1 = tiles1.size(), n2 = tiles2.size();
  std::vector<uint32_t> img1, img2;
  int32_t stride1 = 0, stride2 = 0;
  {
    std::string err;
    if (!build_images(tiles1, segs, {}, {}, {}, img1, stride1, err) ||
        !build_images(tiles2, segs, {}, {}, {}, img2, stride2, err))
      return fail(DMRG_E_UNSUPPORTED, err);
  }
  const size_t w1 = img1.size();
  img1.insert(img1.end(), img2.begin(), img2.end());
  dmrg_status st;
  if ((st = upload(ctx->tr_images, img1.data(), img1.size() * sizeof(uint32_t), s)) != DMRG_OK) return st;
  HIP_TRY(ctx->tr_tmp.ensure((size_t)std::max<int64_t>(utot, 1) * sizeof(double)));
  const uint32_t* di = ctx->tr_images.as<uint32_t>();
  HIP_TRY(launch_hpsi(kPrecF64, 0, (int)n1, di, stride1, O_d, W_d, ctx->tr_tmp.as<double>(), 1.0, 0.0, s));
  HIP_TRY(launch_hpsi(kPrecF64, 0, (int)n2, di + w1, stride2, ctx->tr_tmp.as<double>(), W_d, out_d, 1.0,
                      0.0, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host tile lists die here
  return DMRG_OK;
}

dmrg_status dmrg_lanczos_tridiag(dmrg_sb sb, const double* v0_d, int32_t nsteps, double* alpha_h,
                                 double* beta_h, int32_t* steps_h, double* norm0_h) {
  dmrg_status st = need_square(sb);
  if (st != DMRG_OK) return st;
  if (!v0_d || !alpha_h || !beta_h || !steps_h || nsteps < 1) return fail(DMRG_E_ARG, "bad argument");
  dmrg_ctx ctx = sb->ctx;
  DeviceGuard guard(ctx->device);
  hipStream_t s = ctx->stream;
  const int64_t D = sb->fwd.plan.D;
  const int nvec = nsteps + 1;
  const size_t npart = std::max(lz_partial_size(D, nvec), (size_t)vec_blocks(D));
  HIP_TRY(ctx->V.ensure((size_t)nvec * D * sizeof(double)));
  HIP_TRY(ctx->w.ensure((size_t)D * sizeof(double)));
  HIP_TRY(ctx->partial.ensure(npart * sizeof(double)));
  // small: h1[nvec], h2[nvec], (unused)[nvec], nrm2[8], ab[2*nvec]
  const size_t nsmall = (size_t)5 * nvec + 8;
  HIP_TRY(ctx->small.ensure(nsmall * sizeof(double)));
  HIP_TRY(hipMemsetAsync(ctx->small.p, 0, nsmall * sizeof(double), s));
  double* V = ctx->V.as<double>();
  double* w = ctx->w.as<double>();
  double* part = ctx->partial.as<double>();
  double* h1 = ctx->small.as<double>();
  double* h2 = h1 + nvec;
  double* nrm2 = h2 + 2 * nvec;
  double* ab = nrm2 + 8;
  HIP_TRY(launch_multi_dot(v0_d, 0, 1, v0_d, D, part, nrm2, s));
  HIP_TRY(launch_normalise(V, v0_d, nrm2, D, s));
  for (int j = 0; j < nsteps; ++j) {
    if ((st = run_product(sb, sb->fwd, sb->prec, V + (size_t)j * D, w, 1.0, 0.0)) != DMRG_OK) return st;
    HIP_TRY(launch_lz_step(w, V, D, j + 1, D, h1, h2, part, ab + 2 * j, V + (size_t)(j + 1) * D, s));
  }
  std::vector<double> hs(2 * nsteps + 1);
  HIP_TRY(hipMemcpyAsync(hs.data(), ab, 2 * nsteps * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hs.data() + 2 * nsteps, nrm2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int steps = 0;
  for (; steps < nsteps; ++steps) {
    alpha_h[steps] = hs[2 * steps];
    beta_h[steps] = hs[2 * steps + 1];
    if (hs[2 * steps + 1] <= 1e-13 * std::max(1.0, std::fabs(hs[2 * steps]))) {
      ++steps;
      break;
    }
  }
  *steps_h = steps;
  if (norm0_h) *norm0_h = std::sqrt(std::max(0.0, hs[2 * nsteps]));
  return DMRG_OK;
}

dmrg_status dmrg_host_ldos(int32_t n, const double* alpha, const double* beta, double weight,
                           double e0, int32_t nomega, const double* omega, double eta, double* out) {
  if (n < 1 || !alpha || !beta || nomega < 0 || (nomega > 0 && (!omega || !out)) || !(eta > 0.0))
    return fail(DMRG_E_ARG, "bad argument");
  for (int32_t k = 0; k < nomega; ++k) {
    const double zr = e0 - omega[k], zi = -eta;   // zeta = E0 - omega - i eta
    // continued fraction from the bottom: f = 1 / (zeta - a_j - b_j^2 f_next)
    double fr = 0.0, fi = 0.0;
    for (int32_t j = n - 1; j >= 0; --j) {
      const double b2 = j + 1 < n ? beta[j] * beta[j] : 0.0;
      const double dr = zr - alpha[j] - b2 * fr, di = zi - b2 * fi;
      const double den = dr * dr + di * di;
      fr = dr / den;
      fi = -di / den;
    }
    out[k] = 2.0 * weight * fi;
  }
  return DMRG_OK;
}

dmrg_status dmrg_host_sym_eigen(int32_t n, double* a, double* w) {
  if (n < 0 || (n > 0 && (!a || !w))) return fail(DMRG_E_ARG, "bad argument");
  if (!sym_eigen(n, a, w)) return fail(DMRG_E_NOCONV, "QR sweeps did not converge");
  return DMRG_OK;
}

dmrg_status dmrg_host_tridiag_lowest(int32_t n, const double* alpha, const double* beta,
                                     double* theta, double* u) {
  if (n < 1 || !alpha || !theta || !u || (n > 1 && !beta)) return fail(DMRG_E_ARG, "bad argument");
  tridiag_lowest(n, alpha, beta, theta, u);
  return DMRG_OK;
}

}  // extern "C"
