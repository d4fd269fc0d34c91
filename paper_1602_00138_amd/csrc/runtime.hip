// Host runtime: operator and basis handles, Algorithm 2 (recycling and global basis
// construction, Sec. 4.3) in CG form, the reduced matrices of eq. (newreduced), and
// the C ABI of include/rom.h.  All arithmetic runs in the kernels of this library;
// the host only sequences launches and takes the decisions of Algorithm 2 (skip
// test, convergence, truncation) from scalars read back at its sync points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <string>
#include <thread>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "kernels.h"

struct rom_operator {
  rom_grid grid;
  int64_t n;
  bool var;
  double Dc;
  double* diag_star;
  double* fx;
  double* fy;
  double* fz;
  double* Dfield = nullptr;   // per-node D (copy), when var
  rom::Stencil S{};
};

struct rom_basis {
  const rom_operator* op;
  int64_t n, ld;
  int m, cap;
  double* Q;
  double* Gstar;
  int64_t ldg;
  int n_src, n_det;
  const int64_t* idx_dev;   // n_src + n_det node indices (sources first)
  const double* scale_dev;  // n_src + n_det scales
};

namespace rom {

namespace {

thread_local std::string g_err;

constexpr size_t ALIGN = 256;
// restarts of one solve from its true residual (each a full CG solve)
constexpr int MAX_SWEEPS = 64;
// smallest residual reduction asked of one FP32 sweep (about 16 FP32 unit roundoffs:
// below it the FP32 true residual no longer follows the recursive one)
constexpr double FP32_GOAL_MIN = 1e-6;
// CG steps per captured graph (even: a chunk of one-launch steps then ends on the parity
// it started from)
constexpr int GRAPH_STEPS = 8;
static_assert(GRAPH_STEPS % 2 == 0, "one-launch graph chunks alternate the parity");
// The next convergence poll is placed past the extrapolated stop by this factor and pad:
// a launch after the stop returns at once (a few microseconds), while a poll that comes too
// early idles the GPU for a host round trip and costs another one.
constexpr double POLL_MARGIN = 1.15;
constexpr int POLL_PAD = 2;

struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int REC_MAX = 16;        // learned recycle vectors per point
constexpr double REC_KEEP = 1e-6;  // share of a recycle vector's norm outside V to keep it

// Small control block read back by the host at every decision point.
struct Ctrl {
  double sc[16];
  int status[4];
  int pad[4];
  double rn[G_MAX];        // squared residual norms of a batch
  double gs[3 * G_MAX];    // initial-guess step per member: d^T r, d^T A d, ||r1||^2
  CGState cg[G_MAX];
};
// Host copy of the control block: Ctrl, then the publish flag on its own cache line.
constexpr size_t CTRL_FLAG_OFFSET = (sizeof(Ctrl) + 127) / 128 * 128;
constexpr size_t CTRL_HOST_BYTES = CTRL_FLAG_OFFSET + 128;
// How long the host spins on the publish flag before it blocks on the stream.
constexpr int CTRL_SPIN_MS = 5;
static_assert(offsetof(Ctrl, cg) % 8 == 0 && sizeof(CGState) % 8 == 0,
              "the control block is published in 8-byte words");
static_assert(sizeof(Ctrl) <= 16384, "the publish kernel copies at most 16 KiB");


int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Per-class kernel accounting; launches of the classes in `mask` are bracketed by
// HIP events on the launch stream and harvested at the host sync points.
class Timer {
 public:
  explicit Timer(int mask) : mask_(mask) {
    for (int k = 0; k < ROM_NK; ++k) ms[k] = bytes[k] = flops[k] = 0.0, launches[k] = 0;
  }
  ~Timer() {
    for (auto& e : pool_) (void)hipEventDestroy(e);
  }
  // the next ROM_LAUNCH of class cls records (a, b) in its own dispatch
  void begin(int cls) {
    if (!(mask_ >> cls & 1)) return;
    hipEvent_t a = get(), b = get();
    pending_events().a = a;
    pending_events().b = b;
    open_.push_back({cls, a, b});
  }
  void end(int cls, double by, double fl = 0.0) {
    add(cls, by, fl);
    if (!(mask_ >> cls & 1) || open_.empty() || open_.back().cls != cls) return;
    if (pending_events().a) {
      // nothing was launched: the events were never recorded
      pending_events().a = pending_events().b = nullptr;
      free_.push_back(open_.back().a);
      free_.push_back(open_.back().b);
    } else {
      pending_.push_back(open_.back());
    }
    open_.pop_back();
  }
  // account a launch without events
  void add(int cls, double by, double fl = 0.0) {
    bytes[cls] += by;
    flops[cls] += fl;
    launches[cls] += 1;
  }
  // correct the byte / flop count of class cls
  void adjust(int cls, double dby, double dfl) {
    bytes[cls] += dby;
    flops[cls] += dfl;
  }
  // Undo the accounting of the last `count` launches of class cls (launches that
  // returned at once because the iteration had already stopped).
  void discard(int cls, int count, double by, double fl) {
    if (count <= 0) return;
    bytes[cls] -= by * count;
    flops[cls] -= fl * count;
    launches[cls] -= count;
    if (!(mask_ >> cls & 1)) return;
    for (int k = (int)pending_.size() - 1; k >= 0 && count > 0; --k) {
      if (pending_[k].cls != cls) continue;
      free_.push_back(pending_[k].a);
      free_.push_back(pending_[k].b);
      pending_.erase(pending_.begin() + k);
      --count;
    }
  }
  // call after a stream synchronisation
  void harvest() {
    for (auto& p : pending_) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) ms[p.cls] += t;
      free_.push_back(p.a);
      free_.push_back(p.b);
    }
    pending_.clear();
  }
  double ms[ROM_NK], bytes[ROM_NK], flops[ROM_NK];
  long long launches[ROM_NK];

 private:
  struct Pair {
    int cls;
    hipEvent_t a, b;
  };
  hipEvent_t get() {
    if (!free_.empty()) {
      hipEvent_t e = free_.back();
      free_.pop_back();
      return e;
    }
    hipEvent_t e;
    ROM_HIP(hipEventCreate(&e));
    pool_.push_back(e);
    return e;
  }
  int mask_;
  std::vector<hipEvent_t> pool_, free_;
  std::vector<Pair> open_, pending_;
};

Stencil make_stencil(const rom_operator& op) { return op.S; }

Bumps make_bumps(const rom_mu& mu, int dim) {
  Bumps b;
  std::memset(&b, 0, sizeof(b));
  b.nb = mu.nb;
  b.dim = dim;
  b.mu0 = mu.mu0;
  for (int k = 0; k < mu.nb; ++k) {
    double* p = b.p + k * (dim + 2);
    for (int a = 0; a < dim; ++a) p[a] = mu.centers[k * dim + a];
    p[dim] = mu.radii[k];
    p[dim + 1] = mu.amps[k];
  }
  return b;
}

void check_mu(const rom_mu* mu, int dim) {
  if (!mu) throw Error(ROM_EINVAL, "null parameter point");
  if (mu->nb < 0 || mu->nb > ROM_MAX_BUMPS) throw Error(ROM_EINVAL, "bump count out of range");
  if (mu->nb > 0 && (!mu->centers || !mu->radii || !mu->amps))
    throw Error(ROM_EINVAL, "null bump arrays");
  if (!std::isfinite(mu->mu0) || mu->mu0 < 0) throw Error(ROM_EINVAL, "mu0 must be >= 0");
  for (int k = 0; k < mu->nb; ++k) {
    if (!(mu->radii[k] > 0) || !std::isfinite(mu->radii[k]))
      throw Error(ROM_EINVAL, "bump radius must be > 0");
    if (!std::isfinite(mu->amps[k])) throw Error(ROM_EINVAL, "bump amplitude not finite");
    for (int a = 0; a < dim; ++a)
      if (!std::isfinite(mu->centers[k * dim + a])) throw Error(ROM_EINVAL, "bump centre not finite");
  }
}

void check_grid(const rom_grid* g) {
  if (!g) throw Error(ROM_EINVAL, "null grid");
  if (g->dim != 2 && g->dim != 3) throw Error(ROM_EINVAL, "dim must be 2 or 3");
  for (int a = 0; a < 3; ++a)
    if (g->n[a] < 1) throw Error(ROM_EINVAL, "grid sizes must be >= 1");
  if (g->dim == 2 && g->n[2] != 1) throw Error(ROM_EINVAL, "2D grids need n[2] == 1");
  for (int f = 0; f < 6; ++f)
    if (g->bc[f] != 0 && g->bc[f] != 1) throw Error(ROM_EINVAL, "bc must be 0 or 1");
  if (!(g->robin_A >= 0) || !std::isfinite(g->robin_A)) throw Error(ROM_EINVAL, "robin_A must be >= 0");
  const double n = (double)g->n[0] * g->n[1] * g->n[2];
  if (n > 2.0e9) throw Error(ROM_EINVAL, "grid too large");
}

size_t operator_layout(const rom_grid& g, bool var, Arena& a, rom_operator* op) {
  const int64_t n = (int64_t)g.n[0] * g.n[1] * g.n[2];
  double* diag = a.take<double>(n);
  double *fx = nullptr, *fy = nullptr, *fz = nullptr, *Dcopy = nullptr;
  if (var) {
    fx = a.take<double>(n);
    fy = a.take<double>(n);
    fz = g.dim == 3 ? a.take<double>(n) : nullptr;
    Dcopy = a.take<double>(n);
  }
  if (op) {
    op->Dfield = Dcopy;
    op->diag_star = diag;
    op->fx = fx;
    op->fy = fy;
    op->fz = fz;
  }
  return a.off;
}

// Launch shapes chosen by the CG autotuner, per process: (device, value size, batch
// size, U_j width class, grid size) -> blocks per member.
using TuneKey = std::tuple<int, int, int, int, int64_t, int>;
std::map<TuneKey, int>& tune_map() {
  static std::map<TuneKey, int> m;
  return m;
}
std::mutex& tune_mu() {
  static std::mutex mu;
  return mu;
}

// ------------------------------------------------------------------------------------
// Algorithm 2, CG form.

class Sequencer {
 public:
  Sequencer(rom_operator* op, int n_src, int n_det, int k_u, int K, const rom_opts& o)
      : op_(op), S_(op->S), n_(op->n), ld_(round_up(op->n, 64)), n_src_(n_src), n_det_(n_det),
        n_rhs_(n_src + n_det), K_(K), ku_in_(k_u), o_(o) {
    const int64_t full = (int64_t)k_u + (int64_t)n_rhs_ * K;
    cap_ = o.cap > 0 ? (int)std::min<int64_t>(o.cap, full) : (int)std::min<int64_t>(full, 4096);
    cap_ = (int)std::min<int64_t>(cap_, n_);
    if (cap_ < 1) cap_ = 1;
    ldg_ = round_up(cap_, 2);   // even: the projections read 16-byte column pairs
    pool_cap_ = n_rhs_ + std::max(0, cap_);
    tol_ = o.tol;
    trunc_ = o.trunc;
    maxit_ = o.maxit > 0 ? o.maxit : (int)std::min<int64_t>(n_, 1 << 30);
    chunk_ = o.check_every > 0 ? o.check_every : 16;
    mixed_ = o.precision == ROM_PREC_MIXED;
    tune_ = o.tune != 0;
    graph_ = o.graph != 0;
    guess_ = o.guess;
    recycle_ = o.recycle;
    n_rec_ = o.recycle ? o.n_recycle : 0;
    inner_tol_ = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    G_ = std::max(1, std::min(o.group, std::min(G_MAX, n_rhs_)));
  }

  int cap() const { return cap_; }

  ~Sequencer() {
    if (!graphs_.empty()) {
      // an error may have left replays queued: let them drain first
      (void)hipStreamSynchronize(st_);
      for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    }
    if (cap_st_) (void)hipStreamDestroy(cap_st_);
    if (h_) (void)hipHostFree(h_);
  }

  size_t layout(void* base) {
    Arena a(base);
    const int G = G_;
    const int64_t wsz = ld_ * NJ_MAX;   // one member's recycle space
    Q_ = a.take<double>(ld_ * cap_);
    pool_ = a.take<double>(ld_ * pool_cap_);
    Wp_ = a.take<double>(wsz * G);
    AWp_ = a.take<double>(wsz * G);
    x0_ = a.take<double>(ld_ * G);
    r_ = a.take<double>(ld_ * G);
    g_ = a.take<double>(ld_ * G);
    // s, q (p_) and w of the CG in two buffers each (the one-launch step alternates them)
    s_ = a.take<double>(2 * ld_ * G);
    p_ = a.take<double>(2 * ld_ * G);
    w_ = a.take<double>(2 * ld_ * G);
    d_ = a.take<double>(ld_ * G);
    xt_ = a.take<double>(ld_ * G);
    r2_ = a.take<double>(ld_ * G);
    vAB_ = a.take<double>(3 * ld_);   // u, A_* u, A_i u of an append
    fa_ = a.take<double>(ld_);
    fw_ = a.take<double>(ld_);
    xg_ = a.take<double>(ld_ * G);
    blk_ = G > 1 ? a.take<double>(ld_ * 2 * G) : nullptr;
    bblk_ = G > 1 ? a.take<double>((size_t)(cap_ + 8) * 2 * G) : nullptr;
    diag_i_ = a.take<double>(ld_);
    dmu_ = a.take<double>(ld_);
    // the rows of bump support (at most a quarter of the grid) and V on them
    nzcap_ = std::min<int64_t>(n_, std::max<int64_t>(1024, n_ / 4));
    ldb_ = round_up(nzcap_, 64);
    Vb_ = a.take<double>((size_t)ldb_ * cap_);
    bidx_ = a.take<int64_t>(nzcap_);
    dmub_ = a.take<double>(nzcap_);
    zb_ = a.take<double>(nzcap_);
    nzwork_ = a.take<int>(ceil_div(n_, 256) + 1);
    Gs_ = a.take<double>((size_t)ldg_ * cap_);
    Gi_ = a.take<double>((size_t)ldg_ * cap_);
    Lc_ = a.take<double>((size_t)ldg_ * cap_);
    Lr_ = a.take<double>((size_t)ldg_ * cap_);
    const size_t gp = std::max(gram_partials_max(cap_, cap_, n_, true),
                               gram_partials_max(NJ_MAX, NJ_MAX, n_, false));
    gram_part_ = a.take<double>(std::max<size_t>(gp, 1));
    const StencilShape sh = stencil_shape(S_, 1024);
    const StencilShape sh5 = stencil_shape(S_, 512);
    red_part_ = a.take<double>(std::max<size_t>(2 * 1024, (size_t)std::max(sh5.blocks, 256) * G));
    // CG partials per member: the operator step's (dcg_iter_values(NJ_MAX) rows of at most
    // sh.blocks, twice: the one-launch step alternates halves), the start's (NJ_MAX + 1
    // rows) and the update's (one row)
    pos_ = (int64_t)std::max(dcg_op_values(NJ_MAX), dcg_iter_values(NJ_MAX)) *
           std::max(sh.blocks, 1);
    part_o_ = a.take<double>((size_t)pos_ * G * 2);
    p2s_ = (int64_t)(NJ_MAX + 1) * dcg_blocks(n_);
    part2_ = a.take<double>((size_t)p2s_ * G);
    pus_ = dcg_blocks(n_);
    part_u_ = a.take<double>((size_t)pus_ * G);
    cgv_ = a.take<CGVec>(G_MAX);
    size_t gt = std::max(gemvt_partials_max(n_, std::max(cap_ + 1, NJ_MAX), 3),
                         gemvt_partials_max(cap_, cap_, 2));
    gt = std::max(gt, proj_partials_max(std::max(cap_, NJ_MAX), G_MAX, n_));
    gt_part_ = a.take<double>(std::max<size_t>(gt, 1));
    tbuf_ = a.take<double>((size_t)(std::max(cap_, NJ_MAX) + 8) * std::max(G, 2));
    ubuf_ = a.take<double>((size_t)(cap_ + 8) * G);
    cbuf_ = a.take<double>((size_t)(cap_ + 8) * G);
    tmpl_ = a.take<double>(std::max(cap_, REC_MAX) + 8);
    tmpr_ = a.take<double>(2 * (cap_ + 8));
    bvals_ = a.take<double>(4 * (cap_ + 8));   // [t | h | h_i | b row] of an append
    fcw_ = a.take<double>(2 * (cap_ + 8));     // [w | y]
    ftmp_ = a.take<double>(2 * (cap_ + 8));
    GWs_ = a.take<double>((size_t)NJ_MAX * NJ_MAX * G);
    if (n_rec_ > 0) {
      rec_ = a.take<double>(ld_ * REC_MAX);
      rAW_ = a.take<double>(ld_ * REC_MAX);
      rtb_ = a.take<double>((size_t)(cap_ + 8) * REC_MAX);
      rub_ = a.take<double>((size_t)(cap_ + 8) * REC_MAX);
    }
    lwork_ = a.take<double>(linv_rebuild_work(cap_));
    LWinv_ = a.take<double>(NJ_MAX * NJ_MAX * G);
    GWinv_ = a.take<double>(NJ_MAX * NJ_MAX * G);
    if (mixed_) {
      W32_ = a.take<float>(wsz * G);
      AW32_ = a.take<float>(wsz * G);
      s32_ = a.take<float>(2 * ld_ * G);
      p32_ = a.take<float>(2 * ld_ * G);
      w32_ = a.take<float>(2 * ld_ * G);
      d32_ = a.take<float>(ld_ * G);
      diag32_ = a.take<float>(ld_);
      if (S_.var) {
        fx32_ = a.take<float>(ld_);
        fy32_ = a.take<float>(ld_);
        fz32_ = S_.dim == 3 ? a.take<float>(ld_) : nullptr;
      }
    }
    ctrl_ = a.take<Ctrl>(1);
    idx_dev_ = a.take<int64_t>(n_rhs_);
    scale_dev_ = a.take<double>(n_rhs_);
    return a.off + ALIGN;
  }

  // Streaming form of Algorithm 2: begin() takes the right-hand sides and U_0, each
  // point() runs one parameter point, finish() reports.  run() is the three in a row.
  void begin(const int64_t* src_idx, const double* src_scale, const int64_t* det_idx,
             const double* det_scale, const double* U0, hipStream_t st) {
    t0_ = std::chrono::steady_clock::now();
    st_ = st;
    timer_.reset(new Timer(o_.timing));
    tm_ = timer_.get();
    // the control block's host copy and, after it, the publish flag: coherent pinned memory
    // that the publish kernel writes directly
    ROM_HIP(hipHostMalloc((void**)&h_, CTRL_HOST_BYTES, hipHostMallocMapped | hipHostMallocCoherent));
    hflag_ = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(h_) + CTRL_FLAG_OFFSET);
    *hflag_ = 0;
    seq_ = 0;
    void* dh = nullptr;
    ROM_HIP(hipHostGetDevicePointer(&dh, h_, 0));
    dh_ = dh;
    dflag_ = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(dh) + CTRL_FLAG_OFFSET);
    U0_ = U0;
    idx_.assign(src_idx, src_idx + n_src_);
    idx_.insert(idx_.end(), det_idx, det_idx + n_det_);
    scale_.assign(src_scale, src_scale + n_src_);
    scale_.insert(scale_.end(), det_scale, det_scale + n_det_);
    ROM_HIP(hipMemcpyAsync(idx_dev_, idx_.data(), n_rhs_ * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ROM_HIP(hipMemcpyAsync(scale_dev_, scale_.data(), n_rhs_ * sizeof(double), hipMemcpyHostToDevice, st));
    ROM_HIP(hipMemsetAsync(ctrl_, 0, sizeof(Ctrl), st));
    ROM_HIP(hipMemsetAsync(Gs_, 0, sizeof(double) * ldg_ * cap_, st));
    ROM_HIP(hipMemsetAsync(Gi_, 0, sizeof(double) * ldg_ * cap_, st));
    ROM_HIP(hipMemsetAsync(Lc_, 0, sizeof(double) * ldg_ * cap_, st));
    ROM_HIP(hipMemsetAsync(Lr_, 0, sizeof(double) * ldg_ * cap_, st));
    if (mixed_ && S_.var) {
      // FP32 face coefficients for the FP32 stencil of the mixed form
      launch_cast_f32(n_, op_->fx, fx32_, st);
      launch_cast_f32(n_, op_->fy, fy32_, st);
      if (S_.dim == 3) launch_cast_f32(n_, op_->fz, fz32_, st);
      S_.fx32 = fx32_;
      S_.fy32 = fy32_;
      S_.fz32 = fz32_;
    }
    sync();

    m_ = 0;
    extra_.assign(n_rhs_, {});
    next_slot_ = n_rhs_;
    next_point_ = 0;
    status_ = ROM_OK;
    recs_.clear();
    recs_.reserve((size_t)K_ * n_rhs_);
    total_its_ = 0;
    n_solved_ = n_kept_ = n_drop_trunc_ = n_drop_cap_ = n_nonconv_ = n_uj_capped_ = 0;
  }

  // The next parameter point of the sequence; Xi (device, N x n_rhs, ld N) receives its
  // solutions when not NULL, records (host, n_rhs) its records.  Returns ROM_OK, or
  // ROM_ENOCONV if a solve of this point reached maxit.
  rom_status point(const rom_mu& p, double* Xi, rom_record* records) {
    if (next_point_ >= K_)
      throw Error(ROM_EINVAL, "the sequence was sized for " + std::to_string(K_) + " points");
    const size_t first = recs_.size();
    const int nonconv = n_nonconv_;
    const int i = next_point_++;
    sweep_point(i, p, Xi);
    sync();
    tm_->harvest();
    if (records) std::memcpy(records, recs_.data() + first, (size_t)n_rhs_ * sizeof(rom_record));
    return n_nonconv_ > nonconv ? ROM_ENOCONV : ROM_OK;
  }

  // The basis as it stands (a view into the workspace, refreshed by every call).
  const rom_basis* basis_view() {
    view_.op = op_;
    view_.n = n_;
    view_.ld = ld_;
    view_.m = m_;
    view_.cap = cap_;
    view_.Q = Q_;
    view_.Gstar = Gs_;
    view_.ldg = ldg_;
    view_.n_src = n_src_;
    view_.n_det = n_det_;
    view_.idx_dev = idx_dev_;
    view_.scale_dev = scale_dev_;
    return &view_;
  }

  void report(rom_record* records, rom_stats* stats) {
    if (records) std::memcpy(records, recs_.data(), recs_.size() * sizeof(rom_record));
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->m = m_;
      stats->k_u = ku_;
      stats->n_solved = n_solved_;
      stats->n_kept = n_kept_;
      stats->n_dropped_trunc = n_drop_trunc_;
      stats->n_dropped_cap = n_drop_cap_;
      stats->n_nonconv = n_nonconv_;
      stats->n_uj_capped = n_uj_capped_;
      stats->total_its = total_its_;
      stats->seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
      for (int k = 0; k < ROM_NK; ++k) {
        stats->kernel_ms[k] = tm_->ms[k];
        stats->kernel_bytes[k] = tm_->bytes[k];
        stats->kernel_flops[k] = tm_->flops[k];
        stats->kernel_launches[k] = tm_->launches[k];
      }
    }
  }

  rom_basis* make_basis() {
    rom_basis* V = new rom_basis;
    *V = *basis_view();
    return V;
  }

  int points_done() const { return next_point_; }
  int points_max() const { return K_; }
  int grid_dim() const { return S_.dim; }
  int n_rhs() const { return n_rhs_; }
  hipStream_t stream() const { return st_; }

  rom_status run(const rom_mu* params, const int64_t* src_idx, const double* src_scale,
                 const int64_t* det_idx, const double* det_scale, const double* U0,
                 double* X_out, rom_record* records, rom_stats* stats, hipStream_t st,
                 rom_basis** out_basis) {
    begin(src_idx, src_scale, det_idx, det_scale, U0, st);
    try {
      for (int i = 0; i < K_; ++i)
        point(params[i], X_out ? X_out + (int64_t)i * n_rhs_ * n_ : nullptr, nullptr);
    } catch (...) {
      // the records of the right-hand sides completed before the error
      if (records) {
        std::memset(records, 0, (size_t)K_ * n_rhs_ * sizeof(rom_record));
        std::memcpy(records, recs_.data(), recs_.size() * sizeof(rom_record));
      }
      throw;
    }
    report(records, stats);
    *out_basis = make_basis();
    return status_;
  }

 private:
  // The first `bytes` of the control block into h_, once the stream has reached this
  // point: a one-wave kernel writes them into the coherent host copy and then a sequence
  // number, on which the host spins (a blocking stream wait, which took tens of
  // microseconds to return after the GPU finished, only after CTRL_SPIN_MS).
  void pull(size_t bytes) {
    const unsigned s = ++seq_;
    launch_publish(ctrl_, dh_, bytes, dflag_, s, st_);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 1;; ++spin) {
      if (__atomic_load_n(hflag_, __ATOMIC_ACQUIRE) == s) return;
      if ((spin & 255) == 0 &&
          std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(CTRL_SPIN_MS))
        break;
      __builtin_ia32_pause();
    }
    ROM_HIP(hipStreamSynchronize(st_));
    if (__atomic_load_n(hflag_, __ATOMIC_ACQUIRE) != s)
      throw Error(ROM_EHIP, "control block not published after the stream completed");
  }
  // the scalars and flags (everything before the CG states)
  void pull_head() { pull(offsetof(Ctrl, cg)); }
  // and the CG states of nb members
  void pull_cg(int nb) { pull(offsetof(Ctrl, cg) + sizeof(CGState) * nb); }

  void sync() {
    pull_head();
    tm_->harvest();
    check_status();
  }

  void check_status() {
    const std::string where = " (point " + std::to_string(cur_point_) + ", basis size " +
                              std::to_string(m_) + ")";
    if (h_->status[0]) {
      std::string info;
      if (h_->sc[12] > 0 || h_->sc[13] != 0)
        info = "; border of column " + std::to_string((long)h_->sc[12]) + ": diagonal " +
               std::to_string(h_->sc[13]) + ", projected part " + std::to_string(h_->sc[14]);
      throw Error(ROM_ENOTSPD, "outer Gram matrix V^T A V not positive definite" + where + info);
    }
    if (h_->status[1])
      throw Error(ROM_ENOTSPD, "recycle Gram matrix U_j^T A U_j not positive definite" + where);
  }

  void account_spmv(int cls) {
    const double by = 8.0 * n_ * (3 + (S_.var ? S_.dim : 0));
    tm_->add(cls, by, 13.0 * n_);
  }

  // In-place classical Gram-Schmidt of v against the first `cols` columns of M
  // (orthonormal, ld_), with the second pass taken only when the first one removed more
  // than half of ||v||^2 (Kahan-Parlett "twice is enough"; the second-pass kernels
  // test this on the device).  Returns ||v_out|| / ||v_in||; ctrl sc[4] = ||v_out||^2.
  double cgs2_inplace(double* v, const double* M, int cols) {
    launch_axpby(n_, 1.0, v, 0.0, nullptr, v, &ctrl_->sc[5], red_part_, st_);
    if (cols > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        Skip skip;
        if (pass == 1) {
          skip.v = &ctrl_->sc[4];
          skip.thr = 0.5;
        }
        tm_->begin(ROM_K_GEMVT);
        launch_gemvt(M, ld_, n_, cols, v, 0, 1, tbuf_, gt_part_, st_, skip);
        tm_->end(ROM_K_GEMVT, 8.0 * n_ * (cols + 1), 2.0 * n_ * cols);
        tm_->begin(ROM_K_GEMVN);
        launch_gemvn(M, ld_, n_, cols, tbuf_, 1.0, v, -1.0, v, &ctrl_->sc[4], red_part_, st_,
                     skip);
        tm_->end(ROM_K_GEMVN, 8.0 * n_ * (cols + 2), 2.0 * n_ * cols);
      }
    } else {
      ROM_HIP(hipMemcpyAsync(&ctrl_->sc[4], &ctrl_->sc[5], sizeof(double),
                             hipMemcpyDeviceToDevice, st_));
    }
    pull_head();
    const double a = h_->sc[4], b = h_->sc[5];
    if (cols > 0 && a > 0.5 * b) {
      // the second pass returned at once: drop it from the accounting
      tm_->discard(ROM_K_GEMVT, 1, 8.0 * n_ * (cols + 1), 2.0 * n_ * cols);
      tm_->discard(ROM_K_GEMVN, 1, 8.0 * n_ * (cols + 2), 2.0 * n_ * cols);
    }
    tm_->harvest();
    check_status();
    if (!(b > 0.0) || !std::isfinite(a) || !std::isfinite(b)) return 0.0;
    return std::sqrt(a / b);
  }

  // Append v to V if its normalised part outside range(V) exceeds trunc; border the
  // Gram matrices V^T A_* V and V^T A_i V and the inverse Cholesky factor.  Each
  // Gram-Schmidt pass also projects A_* of its input: with the pass input u, its
  // coefficients t = V^T u and h = V^T A_* u, the new column q = (u - V t)/rho has
  // V^T A_* q = (h - G_* t)/rho, so the border needs no further pass over V.  The border
  // is taken from the last pass run: after the second pass ||t|| / rho is of the order
  // of the rounding error, and a single pass is only kept when rho >= ||u|| / sqrt(2)
  // (||t|| <= rho), so errors already in G_* are not amplified from one column to the
  // next.  V^T A_i q adds V^T (dmu o q), which only reads the row chunks inside the
  // absorption bumps.
  bool append_q(const double* v, double* rho_out) {
    *rho_out = -1.0;
    if (m_ >= cap_) return false;
    const int m = m_;
    double* slot = Q_ + (int64_t)m * ld_;
    double* u = vAB_;               // pass input, then A_* of it at vAB_ + ld_
    launch_axpby(n_, 1.0, v, 0.0, nullptr, u, &ctrl_->sc[5], red_part_, st_);
    bool pass2 = false;
    // the next right-hand side of this point takes its start from this pass (see
    // fused_start): V y and V w are formed with the old V while it is read for u - V t
    const bool fuse = fuse_next_.on && m > 0 && gemvn_fused_ok(Q_, ld_, m);
    if (m > 0) {
      launch_spmv(S_, op_->diag_star, u, vAB_ + ld_, st_);
      account_spmv(ROM_K_OTHER);
      if (fuse) {
        launch_spmv(S_, diag_i_, u, vAB_ + 2 * ld_, st_);
        account_spmv(ROM_K_OTHER);
      }
      tm_->begin(ROM_K_GEMVT);
      launch_gemvt(Q_, ld_, n_, m, u, ld_, fuse ? 3 : 2, bvals_, gt_part_, st_);   // [t1 | h1 (| h1i)]
      tm_->end(ROM_K_GEMVT, 8.0 * n_ * (m + (fuse ? 3 : 2)), (fuse ? 6.0 : 4.0) * n_ * m);
      if (fuse) {
        // [w | y] = G_i^{-1} [V^T A_i u | V^T b_next] in one pair of triangular products
        launch_gather_row(Q_, ld_, m, fuse_next_.idx, fuse_next_.sc, bvals_ + 3 * m, st_);
        launch_linv_solve_multi(Lc_, Lr_, ldg_, m, bvals_ + 2 * m, m, 2, ftmp_, fcw_, gt_part_,
                                st_);
        tm_->begin(ROM_K_OUTER);
        launch_gemvn_fused(Q_, ld_, n_, m, bvals_, fcw_ + m, fcw_, u, slot, fa_, fw_,
                           &ctrl_->sc[4], red_part_, st_);
        tm_->end(ROM_K_OUTER, 8.0 * n_ * (m + 4), 6.0 * n_ * m);
      } else {
        tm_->begin(ROM_K_GEMVN);
        launch_gemvn(Q_, ld_, n_, m, bvals_, 1.0, u, -1.0, slot, &ctrl_->sc[4], red_part_, st_);
        tm_->end(ROM_K_GEMVN, 8.0 * n_ * (m + 2), 2.0 * n_ * m);
      }
      // second pass (the kernels return at once when the first kept more than half
      // of ||v||^2): input slot, [t2 | h2] = V^T [slot, A_* slot]
      Skip skip{&ctrl_->sc[4], 0.5};
      ROM_HIP(hipMemcpyAsync(u, slot, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
      launch_spmv(S_, op_->diag_star, u, vAB_ + ld_, st_);
      account_spmv(ROM_K_OTHER);
      tm_->begin(ROM_K_GEMVT);
      launch_gemvt(Q_, ld_, n_, m, u, ld_, 2, tbuf_, gt_part_, st_, skip);
      tm_->end(ROM_K_GEMVT, 8.0 * n_ * (m + 2), 4.0 * n_ * m);
      tm_->begin(ROM_K_GEMVN);
      launch_gemvn(Q_, ld_, n_, m, tbuf_, 1.0, slot, -1.0, slot, &ctrl_->sc[4], red_part_, st_,
                   skip);
      tm_->end(ROM_K_GEMVN, 8.0 * n_ * (m + 2), 2.0 * n_ * m);
      pull_head();
      pass2 = !(h_->sc[4] > 0.5 * h_->sc[5]);
      if (!pass2) {
        tm_->discard(ROM_K_GEMVT, 1, 8.0 * n_ * (m + 2), 4.0 * n_ * m);
        tm_->discard(ROM_K_GEMVN, 1, 8.0 * n_ * (m + 2), 2.0 * n_ * m);
      }
      tm_->harvest();
      check_status();
    } else {
      ROM_HIP(hipMemcpyAsync(slot, u, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
      ROM_HIP(hipMemcpyAsync(&ctrl_->sc[4], &ctrl_->sc[5], sizeof(double),
                             hipMemcpyDeviceToDevice, st_));
      sync();
    }
    const double a = h_->sc[4], b = h_->sc[5];
    const double rho = (b > 0.0 && std::isfinite(a) && std::isfinite(b)) ? std::sqrt(a / b) : 0.0;
    *rho_out = rho;
    if (fuse) {
      fused_ready_ = true;
      fused_kept_ = false;
      fused_rho_ = std::sqrt(a);   // ||u - V t||, the norm q is divided by
    }
    if (!(rho > trunc_)) return false;
    const double* th = pass2 ? tbuf_ : bvals_;   // [t | h] of the last pass
    if (m > 0) launch_gemvt(Gs_, ldg_, m, m, th, 0, 1, cbuf_, gt_part_, st_);   // G_* t
    launch_normalize(n_, slot, &ctrl_->sc[4], st_);
    border_new(m, slot, th + m);
    ++m_;
    if (fuse) fused_kept_ = true;
    return true;
  }

  // Border of G_*, G_i and Linv for the new (normalised) column k = q: h = V^T A_* u of
  // the last Gram-Schmidt pass, G_* t in cbuf_, ||q_unnormalised||^2 in sc[4].
  void border_new(int k, const double* q, const double* h) {
    launch_spmv(S_, op_->diag_star, q, vAB_, st_);
    account_spmv(ROM_K_OTHER);
    launch_spmv(S_, diag_i_, q, vAB_ + ld_, st_);
    account_spmv(ROM_K_OTHER);
    // d2 = [q^T A_* q, q^T A_i q]; z = dmu o q; w = V^T z (bump rows only: on the
    // gathered rows when the point has them, else the row chunks with a non-zero)
    if (compact_) {
      launch_dot2_scale(n_, q, vAB_, vAB_ + ld_, dmu_, nullptr, &ctrl_->sc[8], red_part_, st_);
      launch_gather_scale(q, bidx_, dmub_, nzr_, Vb_ + (int64_t)k * ldb_, zb_, st_);
      if (k > 0) {
        tm_->begin(ROM_K_GEMVT);
        launch_gemvt(Vb_, ldb_, nzr_, k, zb_, 0, 1, tmpl_, gt_part_, st_);
        tm_->end(ROM_K_GEMVT, 8.0 * nzr_ * (k + 1), 2.0 * nzr_ * k);
      }
    } else {
      launch_dot2_scale(n_, q, vAB_, vAB_ + ld_, dmu_, r2_, &ctrl_->sc[8], red_part_, st_);
      if (k > 0) {
        tm_->begin(ROM_K_GEMVT);
        launch_gemvt(Q_, ld_, n_, k, r2_, 0, 1, tmpl_, gt_part_, st_);
        tm_->end(ROM_K_GEMVT, 8.0 * n_ * (k + 1), 2.0 * n_ * k);
      }
    }
    launch_border_from_proj(h, cbuf_, tmpl_, &ctrl_->sc[4], &ctrl_->sc[8], k, tmpr_, st_);
    launch_border_fill(tmpr_, k, Gs_, Gi_, ldg_, st_);
    launch_linv_border(Lc_, Lr_, ldg_, k, Gi_ + (int64_t)k * ldg_, tmpl_, tmpr_,
                       &ctrl_->status[0], gt_part_, st_, &ctrl_->sc[12]);
  }

  // G_i = V^T A_* V + mu0 I + V^T diag(mu_i - mu0) V, then its inverse Cholesky factor.
  void rebuild_gi() {
    if (m_ == 0) return;
    tm_->begin(ROM_K_GRAM);
    if (compact_)
      launch_gram(Vb_, ldb_, m_, Vb_, ldb_, m_, nzr_, dmub_, true, Gs_, ldg_, mu0_, Gi_, ldg_,
                  gram_part_, st_);
    else
      launch_gram(Q_, ld_, m_, Q_, ld_, m_, n_, dmu_, true, Gs_, ldg_, mu0_, Gi_, ldg_,
                  gram_part_, st_);
    tm_->end(ROM_K_GRAM, 8.0 * n_ * (m_ + 1), 2.0 * n_ * m_ * m_);
    launch_linv_rebuild(Gi_, ldg_, m_, Lc_, Lr_, lwork_, &ctrl_->status[0], st_);
  }

  // Pack U_j = [U_0 part of V, extra columns of RHS j] into member slot y and form
  // A_i U_j, its Gram matrix and the inverse (FP64; FP32 copies of U_j and A_i U_j in the
  // mixed form).  At point 0 every U_j is U_0 (slot 0, built once per point).
  // src (groups after the first point): the group's slot that holds the first ku_ columns
  // of A_i U_j (and their FP32 copies), the same for every member; -1 before the group's
  // first member is built, which then builds them in full and becomes the source.  Later
  // members form A_i only on their own columns (the CG kernels read the shared ones from
  // the source slot) and take the U_0 block of their Gram matrix from the source's.  They
  // pack only their own columns of U_j too: U_0's are V's first ku_ columns, read from Q_
  // for U^T r and the Gram border, and packed into the slot only before a Gram-Schmidt
  // pass against U_j (update_Uj).
  int make_W(int i, int j, int y, int* src = nullptr) {
    const int key = i == 0 ? -1 : j;
    ColPtrs cp;
    int nj = 0;
    for (int c = 0; c < ku_; ++c) cp.p[nj++] = Q_ + (int64_t)c * ld_;
    if (i > 0)
      for (int sl : extra_[j])
        if (nj < NJ_MAX) cp.p[nj++] = pool_ + (int64_t)sl * ld_;
    for (int c = 0; c < n_rec_kept_ && nj < NJ_MAX; ++c) cp.p[nj++] = rec_ + (int64_t)c * ld_;
    const bool part = src && *src >= 0 && *src != y && i > 0 && ku_ > 0 && nj >= ku_;
    const int from = part ? *src : y;   // the slot holding the first ku_ columns of A_i U_j
    if (key == w_key_[y] && nj == w_nj_[y] && from == w_src_[y]) {
      if (src && *src < 0) *src = y;
      return nj;
    }
    w_key_[y] = key;
    w_nj_[y] = nj;
    w_src_[y] = from;
    if (nj == 0) return 0;
    const int64_t off = (int64_t)y * ld_ * NJ_MAX;
    double* W = Wp_ + off;
    double* AW = AWp_ + off;
    double* GW = GWs_ + (int64_t)y * NJ_MAX * NJ_MAX;
    const int k0 = part ? ku_ : 0;   // first column formed here
    const int ne = nj - k0;
    if (part) {
      ColPtrs co;
      for (int c = 0; c < ne; ++c) co.p[c] = cp.p[k0 + c];
      if (ne > 0) launch_pack_cols(n_, co, ne, W + k0 * ld_, ld_, st_);
    } else {
      launch_pack_cols(n_, cp, nj, W, ld_, st_);
    }
    w_full_[y] = !part;
    if (ne > 0) launch_spmm(S_, diag_i_, W + k0 * ld_, ld_, ne, AW + k0 * ld_, st_);
    tm_->begin(ROM_K_GRAM);
    if (!part) {
      // up to 16 columns the MFMA projection W^T (A W) in one pass over W (the factorisation
      // below symmetrises it); wider, the tile Gram kernel, whose lower triangle
      // W_i^T (A W_j), i >= j, is mirrored
      if (nj <= G_MAX)
        launch_proj(W, ld_, nj, AW, ld_, nj, n_, GW, nj, gt_part_, st_);
      else
        launch_gram(W, ld_, nj, AW, ld_, nj, n_, nullptr, true, nullptr, 0, 0.0, GW, nj,
                    gram_part_, st_);
      tm_->end(ROM_K_GRAM, 16.0 * n_ * nj, 2.0 * n_ * nj * nj);
    } else {
      // columns ku_.. : [U_0, E]^T (A E), U_0 from Q_ and E from the slot (the MFMA
      // projection for up to 16 columns); the U_0 block from the source; the block below
      // it mirrored
      double* Gb = GW + (int64_t)k0 * nj;
      if (ne > 0 && ne <= G_MAX) {
        launch_proj(Q_, ld_, k0, AW + k0 * ld_, ld_, ne, n_, Gb, nj, gt_part_, st_);
        launch_proj(W + k0 * ld_, ld_, ne, AW + k0 * ld_, ld_, ne, n_, Gb + k0, nj, gt_part_,
                    st_);
      } else if (ne > 0) {
        launch_gram(Q_, ld_, k0, AW + k0 * ld_, ld_, ne, n_, nullptr, false, nullptr, 0, 0.0, Gb,
                    nj, gram_part_, st_);
        launch_gram(W + k0 * ld_, ld_, ne, AW + k0 * ld_, ld_, ne, n_, nullptr, false, nullptr,
                    0, 0.0, Gb + k0, nj, gram_part_, st_);
      }
      launch_gram_assemble(GWs_ + (int64_t)from * NJ_MAX * NJ_MAX, w_nj_[from], k0, GW, nj,
                           st_);
      tm_->end(ROM_K_GRAM, 8.0 * n_ * (nj + ne), 2.0 * n_ * nj * ne);
    }
    launch_small_chol_inv(GW, nj, LWinv_ + (int64_t)y * NJ_MAX * NJ_MAX,
                          GWinv_ + (int64_t)y * NJ_MAX * NJ_MAX, &ctrl_->status[1], st_);
    if (mixed_ && ne > 0) {
      launch_cast_cols_f32(n_, ne, W + k0 * ld_, ld_, W32_ + off + k0 * ld_, st_);
      launch_cast_cols_f32(n_, ne, AW + k0 * ld_, ld_, AW32_ + off + k0 * ld_, st_);
    }
    if (src && *src < 0) *src = y;
    return nj;
  }

  // One parameter point of Algorithm 2 (point index i of the sequence).
  void sweep_point(int i, const rom_mu& p, double* Xi) {
    hipStream_t st = st_;
    {
      cur_point_ = i;
      mu0_ = p.mu0;
      launch_mu_eval(S_, make_bumps(p, S_.dim), op_->diag_star, diag_i_, dmu_, st);
      // the rows of bump support of this point, and V gathered on them
      launch_nz_rows(n_, dmu_, bidx_, dmub_, nzcap_, &ctrl_->status[2], nzwork_, st);
      sync();
      nzr_ = h_->status[2];
      compact_ = nzr_ > 0 && nzr_ <= nzcap_;
      if (compact_) launch_gather_idx(Q_, ld_, bidx_, nzr_, 0, m_, Vb_, ldb_, st);
      if (mixed_) launch_cast_f32(n_, diag_i_, diag32_, st);
      if (i == 0) {
        // V <- orth(U_0): CGS2 append of every column (Alg. 2 initialisation)
        for (int c = 0; c < ku_in_; ++c) {
          double rho;
          append_q(U0_ + (int64_t)c * n_, &rho);
        }
        ku_ = m_;
      } else {
        rebuild_gi();
      }
      prepare_recycle(i);
      fused_ready_ = false;
      for (int y = 0; y < G_MAX; ++y) w_key_[y] = -2;
      if (G_ == 1)
        point_sequential(i, Xi);
      else
        point_grouped(i, Xi);
      if (i == 0) {
        // U_j <- [U_0, X_0(:, j)] (Sec. 4.2.2), X_0(:, j) orthonormalised against U_0
        for (int j = 0; j < n_rhs_; ++j) {
          double* slot = pool_ + (int64_t)j * ld_;
          const double rho = cgs2_inplace(slot, Q_, ku_);
          extra_[j].clear();
          if (rho > trunc_ && ku_ < NJ_MAX) {
            launch_normalize(n_, slot, &ctrl_->sc[4], st);
            extra_[j].push_back(j);
          }
        }
      }
    }
  }

  // Learned recycle vectors of point i (FP32, n_rec_ of them), made A_i-orthogonal to V as
  // it stands at the point start (w <- w - V G_i^{-1} V^T A_i w: the part of w that the
  // outer Galerkin projection on V cannot supply, which is where every correction of this
  // point lies) and orthonormal among themselves; a vector keeps its place iff more than
  // REC_KEEP of its norm survives.  They join U_j of every right-hand side solved at this
  // point (not V, and not the U_j of later points).
  void prepare_recycle(int i) {
    n_rec_kept_ = 0;
    if (n_rec_ <= 0) return;
    const int k = n_rec_;
    launch_convert_cols(n_, k, recycle_ + (int64_t)i * k * n_, n_, rec_, ld_, st_);
    launch_col_norms(n_, k, rec_, ld_, ctrl_->rn, red_part_, st_);
    if (m_ > 0) {
      const int64_t mm = round_up(m_, 2);   // even: the projections read column pairs
      launch_spmm(S_, diag_i_, rec_, ld_, k, rAW_, st_);
      launch_proj(Q_, ld_, m_, rAW_, ld_, k, n_, rtb_, mm, gt_part_, st_);    // t = V^T A w
      launch_proj(Lr_, ldg_, m_, rtb_, mm, k, m_, rub_, mm, gt_part_, st_);   // Linv t
      launch_proj(Lc_, ldg_, m_, rub_, mm, k, m_, rtb_, mm, gt_part_, st_);   // G^{-1} t
      launch_gemvn_multi(Q_, ld_, n_, m_, rtb_, mm, k, 1.0, rec_, ld_, -1.0, rec_, ld_, st_);
    }
    sync();
    double gn[REC_MAX];
    for (int c = 0; c < k; ++c) gn[c] = h_->rn[c];
    int kk = 0;
    for (int c = 0; c < k; ++c) {
      double* w = rec_ + (int64_t)c * ld_;
      if (kk > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          launch_gemvt(rec_, ld_, n_, kk, w, 0, 1, tmpl_, gt_part_, st_);
          launch_gemvn(rec_, ld_, n_, kk, tmpl_, 1.0, w, -1.0, w, &ctrl_->sc[4], red_part_, st_);
        }
      } else {
        launch_col_norms(n_, 1, w, ld_, &ctrl_->sc[4], red_part_, st_);
      }
      sync();
      const double a = h_->sc[4], b = gn[c];
      const double rho = (b > 0.0 && std::isfinite(a) && std::isfinite(b)) ? std::sqrt(a / b) : 0.0;
      if (rho > REC_KEEP) {
        double* slot = rec_ + (int64_t)kk * ld_;
        if (slot != w)
          ROM_HIP(hipMemcpyAsync(slot, w, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
        launch_normalize(n_, slot, &ctrl_->sc[4], st_);
        ++kk;
      }
    }
    n_rec_kept_ = kk;
  }

  // Start of the right-hand side after a fused append (V' = [V, q] when the correction u was
  // kept, q = (u - V t) / rho): the Galerkin coefficients c' = G'^{-1} V'^T b split by the
  // border into c'[0:m] = y - G^{-1} g c'_m with g = V^T A_i q, and
  // q - V G^{-1} g = (u - V w) / rho with w = G^{-1} V^T A_i u, so
  // x0 = V' c' = V y + (u - V w) c'_m / rho; c'_m comes from the bordered factor.  Without
  // an append, V is unchanged and x0 = V y.  u is the correction, still in g_.
  void fused_start(int64_t idx, double sc) {
    if (fused_kept_) {
      launch_gather_row(Q_, ld_, m_, idx, sc, tbuf_, st_);
      launch_linv_solve(Lc_, Lr_, ldg_, m_, tbuf_, ubuf_, cbuf_, gt_part_, st_);
      launch_fused_start(n_, fa_, g_, fw_, cbuf_ + (m_ - 1), 1.0 / fused_rho_, x0_, st_);
    } else {
      ROM_HIP(hipMemcpyAsync(x0_, fa_, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
    }
    fused_ready_ = false;
  }

  // Bookkeeping of a solved right-hand side: iterations, final residual, convergence.
  void record_solve(int its, int restarts, double res, int flag, rom_record& rec) {
    if (flag == 1) throw Error(ROM_ENOTSPD, "CG met non-positive curvature (operator not SPD)");
    if (flag == 2) throw Error(ROM_ENONFINITE, "non-finite value in CG");
    total_its_ += its;
    rec.its = its;
    rec.restarts = restarts;
    rec.final_res = res;
    rec.converged = res <= tol_;
    if (!rec.converged) {
      ++n_nonconv_;
      status_ = ROM_ENOCONV;
    }
  }

  // U_j grows by the correction of RHS j orthonormalised against the persistent columns
  // of the recycle space it was solved with (member slot y: U_0, then RHS j's earlier
  // corrections, all orthonormal), when the correction joined V (i > 0).  The point's
  // learned recycle vectors, packed after them, are only A_i-orthogonal to V and are not
  // part of U_j, so the Gram-Schmidt pass leaves them out.  U_j stops growing at NJ_MAX
  // columns (counted in n_uj_capped_).
  void update_Uj(int i, int j, int y, const double* gptr, int nj) {
    if (i == 0 || next_slot_ >= pool_cap_) return;
    const int npers = ku_ + (int)extra_[j].size();
    if (npers >= NJ_MAX) {
      ++n_uj_capped_;
      return;
    }
    double* slot = pool_ + (int64_t)next_slot_ * ld_;
    launch_axpby(n_, 1.0, gptr, 0.0, nullptr, slot, nullptr, red_part_, st_);
    if (!w_full_[y]) {
      ColPtrs cu;
      for (int c = 0; c < ku_; ++c) cu.p[c] = Q_ + (int64_t)c * ld_;
      launch_pack_cols(n_, cu, ku_, Wp_ + (int64_t)y * ld_ * NJ_MAX, ld_, st_);
      w_full_[y] = true;
    }
    const double ru = cgs2_inplace(slot, Wp_ + (int64_t)y * ld_ * NJ_MAX, std::min(npers, nj));
    if (ru > trunc_) {
      launch_normalize(n_, slot, &ctrl_->sc[4], st_);
      extra_[j].push_back(next_slot_++);
    }
  }

  // A solved right-hand side j of the sequential order (correction at gptr, solution
  // at xdst): V grows by the CGS2-orthogonalised correction when it passes the
  // truncation test and the cap, then U_j.
  void finish_solved(int i, int j, int y, const double* gptr, const double* xdst, int nj,
                     int its, int restarts, double res, int flag, rom_record& rec) {
    record_solve(its, restarts, res, flag, rec);
    if (m_ < cap_) {
      double rho = 0.0;
      const bool kept = append_q(gptr, &rho);
      rec.rho = rho;
      rec.kept = kept;
      if (kept) {
        ++n_kept_;
        update_Uj(i, j, y, gptr, nj);
      } else {
        ++n_drop_trunc_;
      }
    } else {
      ++n_drop_cap_;
    }
    if (i == 0)
      ROM_HIP(hipMemcpyAsync(pool_ + (int64_t)j * ld_, xdst, sizeof(double) * n_,
                             hipMemcpyDeviceToDevice, st_));
    rec.m = m_;
  }

  // The corrections of a group's solved members (y with act[y], in order) join V as a
  // block: two block Gram-Schmidt passes against V as it stood at the group start (one
  // MFMA projection and one multi-vector update per pass), then, member by member, two
  // passes against the columns this group already added and the truncation test on the
  // remaining norm relative to ||g||.  The Gram borders of the k new columns come from
  // one projection of [A_* Q_new, A_i Q_new] on the extended basis, then the inverse
  // Cholesky factor is bordered column by column.  Fills rec[y].rho / kept / m.
  void append_block(int nb, const int* act, rom_record* rec) {
    int ys[G_MAX];
    int s = 0;
    for (int y = 0; y < nb; ++y)
      if (act[y]) ys[s++] = y;
    if (s == 0) return;
    const int m0 = m_;
    if (m0 >= cap_) {
      for (int c = 0; c < s; ++c) {
        ++n_drop_cap_;
        rec[ys[c]].m = m_;
      }
      return;
    }
    double* U = d_;   // working copies of the corrections, s columns
    for (int c = 0; c < s; ++c)
      ROM_HIP(hipMemcpyAsync(U + (int64_t)c * ld_, g_ + (int64_t)ys[c] * ld_, sizeof(double) * n_,
                             hipMemcpyDeviceToDevice, st_));
    launch_col_norms(n_, s, U, ld_, ctrl_->rn, red_part_, st_);
    if (m0 > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        tm_->begin(ROM_K_GEMVT);
        launch_proj(Q_, ld_, m0, U, ld_, s, n_, tbuf_, m0, gt_part_, st_);
        tm_->end(ROM_K_GEMVT, 8.0 * n_ * (m0 + s), 2.0 * n_ * m0 * s);
        tm_->begin(ROM_K_GEMVN);
        launch_gemvn_multi(Q_, ld_, n_, m0, tbuf_, m0, s, 1.0, U, ld_, -1.0, U, ld_, st_);
        tm_->end(ROM_K_GEMVN, 8.0 * n_ * (m0 + 2 * s), 2.0 * n_ * m0 * s);
      }
    }
    sync();
    double gn[G_MAX];
    for (int c = 0; c < s; ++c) gn[c] = h_->rn[c];
    int k = 0;
    double* Qnew = Q_ + (int64_t)m0 * ld_;
    for (int c = 0; c < s; ++c) {
      rom_record& r = rec[ys[c]];
      if (m0 + k >= cap_) {
        ++n_drop_cap_;
        r.m = m0 + k;
        continue;
      }
      double* w = U + (int64_t)c * ld_;
      if (k > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          launch_gemvt(Qnew, ld_, n_, k, w, 0, 1, tmpl_, gt_part_, st_);
          launch_gemvn(Qnew, ld_, n_, k, tmpl_, 1.0, w, -1.0, w, &ctrl_->sc[4], red_part_, st_);
        }
      } else {
        launch_col_norms(n_, 1, w, ld_, &ctrl_->sc[4], red_part_, st_);
      }
      sync();
      const double a = h_->sc[4], b = gn[c];
      const double rho = (b > 0.0 && std::isfinite(a) && std::isfinite(b)) ? std::sqrt(a / b) : 0.0;
      r.rho = rho;
      if (rho > trunc_) {
        double* slot = Qnew + (int64_t)k * ld_;
        ROM_HIP(hipMemcpyAsync(slot, w, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
        launch_normalize(n_, slot, &ctrl_->sc[4], st_);
        ++k;
        r.kept = 1;
        ++n_kept_;
      } else {
        ++n_drop_trunc_;
      }
      r.m = m0 + k;
    }
    if (k == 0) return;
    // borders: B = [V^T A_* Q_new | V^T A_i Q_new] over the m0 + k columns
    launch_spmm(S_, op_->diag_star, Qnew, ld_, k, blk_, st_);
    launch_spmm(S_, diag_i_, Qnew, ld_, k, blk_ + (int64_t)k * ld_, st_);
    for (int c = 0; c < 2 * k; ++c) account_spmv(ROM_K_OTHER);
    const int mk = m0 + k;
    for (int h = 0; h < 2 * k; h += 16) {
      const int nv = std::min(16, 2 * k - h);
      tm_->begin(ROM_K_GEMVT);
      launch_proj(Q_, ld_, mk, blk_ + (int64_t)h * ld_, ld_, nv, n_, bblk_ + (int64_t)h * mk, mk,
                  gt_part_, st_);
      tm_->end(ROM_K_GEMVT, 8.0 * n_ * (mk + nv), 2.0 * n_ * mk * nv);
    }
    launch_border_fill_block(bblk_, mk, m0, k, Gs_, Gi_, ldg_, st_);
    if (compact_) launch_gather_idx(Q_, ld_, bidx_, nzr_, m0, mk, Vb_, ldb_, st_);
    for (int c = 0; c < k; ++c)
      launch_linv_border(Lc_, Lr_, ldg_, m0 + c, Gi_ + (int64_t)(m0 + c) * ldg_, tmpl_, tmpr_,
                         &ctrl_->status[0], gt_part_, st_, &ctrl_->sc[12]);
    m_ = mk;
  }

  // The right-hand sides of point i one at a time (the paper's order).
  void point_sequential(int i, double* Xi) {
    hipStream_t st = st_;
    for (int j = 0; j < n_rhs_; ++j) {
      const int64_t idx = idx_[j];
      const double sc = scale_[j];
      const double nb = std::fabs(sc);
      rom_record rec;
      std::memset(&rec, 0, sizeof(rec));
      rec.point = i;
      rec.rhs = j;
      rec.rho = -1.0;
      // ---- outer projection on V (Galerkin in the A(p_i) inner product)
      if (fused_ready_) {
        fused_start(idx, sc);
      } else if (m_ > 0) {
        launch_gather_row(Q_, ld_, m_, idx, sc, tbuf_, st);
        launch_linv_solve(Lc_, Lr_, ldg_, m_, tbuf_, ubuf_, cbuf_, gt_part_, st);
        tm_->begin(ROM_K_OUTER);
        launch_gemvn(Q_, ld_, n_, m_, cbuf_, 0.0, nullptr, 1.0, x0_, nullptr, red_part_, st);
        tm_->end(ROM_K_OUTER, 8.0 * n_ * (m_ + 1), 2.0 * n_ * m_);
      } else {
        ROM_HIP(hipMemsetAsync(x0_, 0, sizeof(double) * n_, st));
      }
      launch_resid_unit(S_, diag_i_, x0_, idx, sc, r_, &ctrl_->sc[0], red_part_, st);
      account_spmv(ROM_K_OTHER);
      sync();
      const double rho0 = std::sqrt(h_->sc[0]) / nb;
      rec.rho0 = rho0;
      double* xdst = Xi ? Xi + (int64_t)j * n_ : xt_;
      if (rho0 <= tol_) {
        ROM_HIP(hipMemcpyAsync(xdst, x0_, sizeof(double) * n_, hipMemcpyDeviceToDevice, st));
        if (i == 0)
          ROM_HIP(hipMemcpyAsync(pool_ + (int64_t)j * ld_, x0_, sizeof(double) * n_,
                                 hipMemcpyDeviceToDevice, st));
        rec.final_res = rho0;
        rec.converged = 1;
        rec.m = m_;
        recs_.push_back(rec);
        continue;
      }
      // ---- inner recycled CG on A g = r with U_j (correction equation, eq. (resi))
      ++n_solved_;
      rec.solved = 1;
      rec.rho_guess = -1.0;
      // a given initial guess moves the start to its A-optimal point on x0 + span(xg - x0)
      // when that lowers the residual (r_ and the base point follow)
      xbase_ = x0_;
      double res = rho0;
      if (guess_) {
        res = guess_step(guess_ + ((int64_t)i * n_rhs_ + j) * n_, nb, rho0);
        rec.rho_guess = res;
      }
      int flag = 0, its = 0, restarts = 0;
      int nj = 0;
      if (res > tol_) {
        nj = make_W(i, j, 0);
        if (!mixed_) {
          its = cg_solve<double>(r_, 1.0, g_, nj, tol_ * nb, maxit_, flag);
          launch_axpby(n_, 1.0, xbase_, 1.0, g_, xdst, &ctrl_->sc[6], red_part_, st);
          res = true_residual(xdst, idx, sc, nb);
          while (res > tol_ && its < maxit_ && flag == 0 && restarts < MAX_SWEEPS) {
            ++restarts;
            its += cg_solve<double>(r2_, 1.0, d_, nj, tol_ * nb, maxit_ - its, flag);
            launch_axpby(n_, 1.0, g_, 1.0, d_, g_, nullptr, red_part_, st);
            launch_axpby(n_, 1.0, xbase_, 1.0, g_, xdst, &ctrl_->sc[6], red_part_, st);
            res = true_residual(xdst, idx, sc, nb);
          }
        } else {
          its = refine(xdst, idx, sc, nb, nj, rec, res, restarts, flag);
        }
      } else {
        ROM_HIP(hipMemcpyAsync(xdst, xbase_, sizeof(double) * n_, hipMemcpyDeviceToDevice, st));
        nj = make_W(i, j, 0);
      }
      // the correction that joins V and U_j is x - x0 (x0 in range(V))
      if (xbase_ != x0_) launch_axpby(n_, 1.0, xdst, -1.0, x0_, g_, nullptr, red_part_, st);
      // the append of this correction also forms the next right-hand side's start
      fuse_next_.on = j + 1 < n_rhs_;
      if (fuse_next_.on) {
        fuse_next_.idx = idx_[j + 1];
        fuse_next_.sc = scale_[j + 1];
      }
      finish_solved(i, j, 0, g_, xdst, nj, its, restarts, res, flag, rec);
      fuse_next_.on = false;
      recs_.push_back(rec);
    }
  }

  // The right-hand sides of point i in groups of G_: one outer projection per group
  // (the basis as it stands at the group start), the group's inner solves together,
  // then the appends in right-hand-side order.
  void point_grouped(int i, double* Xi) {
    hipStream_t st = st_;
    for (int j0 = 0; j0 < n_rhs_; j0 += G_) {
      const int nb = std::min(G_, n_rhs_ - j0);
      double* xdst = Xi ? Xi + (int64_t)j0 * n_ : xt_;
      const int64_t ldx = Xi ? n_ : ld_;
      // ---- outer projection of the group: X0 = V G_i^{-1} V^T [b_j0 ..]
      if (m_ > 0) {
        // t = V^T B (rows of V), u = L^{-1} t = Lr^T t, c = L^{-T} u = Lc^T u
        const int mm = (int)round_up(m_, 2);
        launch_gather_rows(Q_, ld_, m_, idx_dev_ + j0, scale_dev_ + j0, nb, tbuf_, mm, st);
        launch_proj(Lr_, ldg_, m_, tbuf_, mm, nb, m_, ubuf_, mm, gt_part_, st);
        launch_proj(Lc_, ldg_, m_, ubuf_, mm, nb, m_, cbuf_, mm, gt_part_, st);
        tm_->begin(ROM_K_OUTER);
        launch_gemvn_multi(Q_, ld_, n_, m_, cbuf_, mm, nb, 0.0, nullptr, 0, 1.0, x0_, ld_, st);
        tm_->end(ROM_K_OUTER, 8.0 * n_ * (m_ + nb), 2.0 * n_ * m_ * nb);
      } else {
        ROM_HIP(hipMemsetAsync(x0_, 0, sizeof(double) * ld_ * nb, st));
      }
      launch_resid_cols(S_, diag_i_, x0_, ld_, nb, idx_dev_ + j0, scale_dev_ + j0, r_, ld_,
                        ctrl_->rn, 1, red_part_, st);
      for (int y = 0; y < nb; ++y) account_spmv(ROM_K_OTHER);
      sync();
      rom_record rec[G_MAX];
      double nbv[G_MAX], res[G_MAX];
      int act[G_MAX], nj[G_MAX];
      bool any = false;
      for (int y = 0; y < nb; ++y) {
        const int j = j0 + y;
        std::memset(&rec[y], 0, sizeof(rom_record));
        rec[y].point = i;
        rec[y].rhs = j;
        rec[y].rho = -1.0;
        nbv[y] = std::fabs(scale_[j]);
        res[y] = std::sqrt(h_->rn[y]) / nbv[y];
        rec[y].rho0 = res[y];
        act[y] = res[y] > tol_;
        nj[y] = 0;
        if (act[y]) {
          any = true;
          ++n_solved_;
          rec[y].solved = 1;
        } else {
          rec[y].final_res = res[y];
          rec[y].converged = 1;
          rec[y].m = m_;
        }
      }
      // skipped members: x = x0
      launch_axpby_cols(n_, nb, 1.0, x0_, ld_, 0.0, nullptr, 0, xdst, ldx, st);
      if (any) {
        // after the first point, the group's first member builds the shared columns of its
        // recycle space and the others read them from its slot
        int src = -1;
        for (int y = 0; y < nb; ++y)
          if (act[y]) nj[y] = make_W(i, j0 + y, i == 0 ? 0 : y, i == 0 ? nullptr : &src);
        // initial guesses move the members' base points (the Galerkin starts kept in xg_)
        bool moved[G_MAX] = {};
        if (guess_) guess_group(i, j0, nb, act, nbv, res, rec, moved);
        else
          for (int y = 0; y < nb; ++y)
            if (act[y]) rec[y].rho_guess = -1.0;
        int its[G_MAX], restarts[G_MAX], flag[G_MAX];
        solve_group(i == 0, i == 0 ? -1 : src, nb, j0, act, nj, nbv, res, xdst, ldx, its,
                    restarts, flag, rec);
        // the correction that joins V and U_j is x - x0 (x0 the Galerkin start, in range(V))
        for (int y = 0; y < nb; ++y)
          if (moved[y]) {
            launch_axpby(n_, 1.0, xdst + y * ldx, -1.0, xg_ + (int64_t)y * ld_,
                         g_ + (int64_t)y * ld_, nullptr, red_part_, st);
          }
        for (int y = 0; y < nb; ++y)
          if (act[y]) record_solve(its[y], restarts[y], res[y], flag[y], rec[y]);
        // ---- the group's corrections join V (in right-hand-side order), then U_j
        append_block(nb, act, rec);
        for (int y = 0; y < nb; ++y)
          if (act[y] && rec[y].kept)
            update_Uj(i, j0 + y, i == 0 ? 0 : y, g_ + (int64_t)y * ld_, nj[y]);
      }
      for (int y = 0; y < nb; ++y) {
        if (i == 0)
          ROM_HIP(hipMemcpyAsync(pool_ + (int64_t)(j0 + y) * ld_, xdst + y * ldx,
                                 sizeof(double) * n_, hipMemcpyDeviceToDevice, st));
        recs_.push_back(rec[y]);
      }
    }
  }

  // Inner solves of the active members of a group, restarted from the FP64 true
  // residual until each meets tol (plain form: FP64 sweeps; mixed form: FP32 sweeps in
  // FP64 refinement, a stalled member continuing in FP64).  On entry r_ holds the
  // members' residuals b - A x0 and res[] their relative norms; on exit g_ holds the
  // corrections, xdst the solutions and res[] the final relative residuals.
  void solve_group(bool shared, int src, int nb, int j0, const int* act, const int* nj,
                   const double* nbv,
                   double* res, double* xdst, int64_t ldx, int* its, int* restarts, int* flag,
                   rom_record* rec) {
    ROM_HIP(hipMemsetAsync(g_, 0, sizeof(double) * ld_ * nb, st_));
    bool live[G_MAX], fp32[G_MAX];
    for (int y = 0; y < nb; ++y) {
      live[y] = act[y] != 0;
      fp32[y] = mixed_;
      its[y] = restarts[y] = flag[y] = 0;
    }
    const double* rcur = r_;
    for (;;) {
      Batch b32, b64;
      b32.nb = b64.nb = nb;
      b32.shared = b64.shared = shared;
      b32.src = b64.src = src;
      Coefs c32, c64;
      bool any32 = false, any64 = false;
      for (int y = 0; y < nb; ++y) {
        c32.c[y] = c64.c[y] = 0.0;
        b32.nj[y] = b64.nj[y] = nj[y];
        if (!live[y]) continue;
        const double rn = res[y] * nbv[y];
        if (fp32[y]) {
          const double goal =
              std::min(0.5, std::max(std::max(inner_tol_, FP32_GOAL_MIN), 0.5 * tol_ / res[y]));
          b32.active[y] = 1;
          b32.rscale[y] = 1.0 / rn;
          b32.tol_abs[y] = goal;
          b32.maxit[y] = std::min(maxit_ - its[y], std::max(64, (maxit_ - its[y]) / 4));
          c32.c[y] = rn;
          any32 = true;
        } else {
          b64.active[y] = 1;
          b64.rscale[y] = 1.0;
          b64.tol_abs[y] = tol_ * nbv[y];
          b64.maxit[y] = maxit_ - its[y];
          c64.c[y] = 1.0;
          if (mixed_) ++rec[y].fp64_sweeps;
          any64 = true;
        }
      }
      if (any32) {
        cg_batch<float>(b32, rcur, d32_);
        for (int y = 0; y < nb; ++y)
          if (b32.active[y]) {
            its[y] += b32.its[y];
            if (b32.flag[y]) {
              fp32[y] = false;   // FP32 breakdown: keep g, go on in FP64
              c32.c[y] = 0.0;
            }
          }
        launch_refine_cols<float>(n_, nb, c32, d32_, ld_, g_, x0_, ld_, xdst, ldx, st_);
      }
      if (any64) {
        cg_batch<double>(b64, rcur, d_);
        for (int y = 0; y < nb; ++y)
          if (b64.active[y]) {
            its[y] += b64.its[y];
            flag[y] = b64.flag[y];
          }
        launch_refine_cols<double>(n_, nb, c64, d_, ld_, g_, x0_, ld_, xdst, ldx, st_);
      }
      launch_resid_cols(S_, diag_i_, xdst, ldx, nb, idx_dev_ + j0, scale_dev_ + j0, r2_, ld_,
                        ctrl_->rn, 1, red_part_, st_);
      for (int y = 0; y < nb; ++y) account_spmv(ROM_K_OTHER);
      sync();
      bool more = false;
      for (int y = 0; y < nb; ++y) {
        if (!live[y]) continue;
        const double prev = res[y];
        res[y] = std::sqrt(h_->rn[y]) / nbv[y];
        if (res[y] <= tol_ || its[y] >= maxit_ || flag[y] != 0 || restarts[y] >= MAX_SWEEPS) {
          live[y] = false;
          continue;
        }
        ++restarts[y];
        if (fp32[y] && !(res[y] <= 0.5 * prev)) fp32[y] = false;
        more = true;
      }
      if (!more) break;
      rcur = r2_;
    }
  }

  // Initial guess xg (FP32): d = xg - x0, alpha = d^T r / d^T A d (the A-optimal step
  // along d from the Galerkin start), x1 = x0 + alpha d, r1 = r - alpha A d.  Kept, as
  // the base point xg_ with r_ = r1, when ||r1|| < ||r||.  Returns the relative residual
  // of the start taken.
  double guess_step(const float* xg, double nb, double rho0) {
    launch_guess_dir(n_, xg, x0_, d_, st_);
    launch_spmv(S_, diag_i_, d_, w_, st_);
    account_spmv(ROM_K_OTHER);
    launch_dot2_scale(n_, d_, r_, w_, dmu_, r2_, &ctrl_->sc[8], red_part_, st_);
    sync();
    const double dr = h_->sc[8], dad = h_->sc[9];
    if (!(dad > 0.0) || !std::isfinite(dr) || !std::isfinite(dad)) return rho0;
    const double alpha = dr / dad;
    launch_axpby(n_, 1.0, r_, -alpha, w_, r2_, &ctrl_->sc[10], red_part_, st_);
    sync();
    const double rho1 = std::sqrt(h_->sc[10]) / nb;
    if (!(rho1 < rho0)) return rho0;
    launch_axpby(n_, 1.0, x0_, alpha, d_, xg_, nullptr, red_part_, st_);
    ROM_HIP(hipMemcpyAsync(r_, r2_, sizeof(double) * n_, hipMemcpyDeviceToDevice, st_));
    xbase_ = xg_;
    return rho1;
  }

  // The initial-guess step of guess_step for the active members of a group (right-hand
  // sides j0 + y at point i), with two host syncs for the whole group.  A member whose
  // guess lowers its residual takes the moved start as its base point: x0_ column y
  // becomes x0 + alpha d (the Galerkin start is kept in xg_ column y) and r_ column y its
  // residual.  res[y] becomes the relative residual of the start taken, rec[y].rho_guess
  // too; moved[y] says which members moved.
  void guess_group(int i, int j0, int nb, const int* act, const double* nbv, double* res,
                   rom_record* rec, bool* moved) {
    bool any = false;
    for (int y = 0; y < nb; ++y) {
      moved[y] = false;
      if (!act[y]) continue;
      any = true;
      launch_guess_dir(n_, guess_ + ((int64_t)i * n_rhs_ + j0 + y) * n_, x0_ + (int64_t)y * ld_,
                       d_ + (int64_t)y * ld_, st_);
    }
    if (!any) return;
    launch_spmm(S_, diag_i_, d_, ld_, nb, w_, st_);
    for (int y = 0; y < nb; ++y) {
      if (!act[y]) continue;
      account_spmv(ROM_K_OTHER);
      launch_dot2_scale(n_, d_ + (int64_t)y * ld_, r_ + (int64_t)y * ld_, w_ + (int64_t)y * ld_,
                        dmu_, nullptr, &ctrl_->gs[3 * y], red_part_, st_);
    }
    sync();
    double alpha[G_MAX];
    bool step[G_MAX];
    for (int y = 0; y < nb; ++y) {
      step[y] = false;
      if (!act[y]) continue;
      rec[y].rho_guess = res[y];
      const double dr = h_->gs[3 * y], dad = h_->gs[3 * y + 1];
      if (!(dad > 0.0) || !std::isfinite(dr) || !std::isfinite(dad)) continue;
      alpha[y] = dr / dad;
      step[y] = true;
      launch_axpby(n_, 1.0, r_ + (int64_t)y * ld_, -alpha[y], w_ + (int64_t)y * ld_,
                   r2_ + (int64_t)y * ld_, &ctrl_->gs[3 * y + 2], red_part_, st_);
    }
    sync();
    for (int y = 0; y < nb; ++y) {
      if (!step[y]) continue;
      const double rho1 = std::sqrt(h_->gs[3 * y + 2]) / nbv[y];
      if (!(rho1 < res[y])) continue;
      double* x0y = x0_ + (int64_t)y * ld_;
      double* keep = xg_ + (int64_t)y * ld_;
      launch_axpby(n_, 1.0, x0y, 0.0, nullptr, keep, nullptr, red_part_, st_);
      launch_axpby(n_, 1.0, keep, alpha[y], d_ + (int64_t)y * ld_, x0y, nullptr, red_part_, st_);
      ROM_HIP(hipMemcpyAsync(r_ + (int64_t)y * ld_, r2_ + (int64_t)y * ld_, sizeof(double) * n_,
                             hipMemcpyDeviceToDevice, st_));
      res[y] = rho1;
      rec[y].rho_guess = rho1;
      moved[y] = true;
    }
  }

  // r2 = b - A x in FP64 (b = sc e_idx); returns ||r2|| / nb.
  double true_residual(const double* x, int64_t idx, double sc, double nb) {
    launch_resid_unit(S_, diag_i_, x, idx, sc, r2_, &ctrl_->sc[3], red_part_, st_);
    account_spmv(ROM_K_OTHER);
    sync();
    return std::sqrt(h_->sc[3]) / nb;
  }

  // Mixed form: FP64 iterative refinement around FP32 deflated-CG sweeps.  On entry
  // r_ = b - A x0 with relative norm res; on exit x = x0 + g meets tol (or maxit).
  // Each FP32 sweep solves A d = r / ||r|| to the relative tolerance
  // max(inner_tol, tol / (2 res), FP32_GOAL_MIN), with at most a quarter of the
  // remaining iteration budget (at least 64), and is followed by g += ||r|| d and the
  // FP64 residual.  A sweep that breaks down or fails to halve the residual hands the
  // solve to the FP64 solver for its remaining sweeps.
  int refine(double* x, int64_t idx, double sc, double nb, int nj, rom_record& rec, double& res,
             int& restarts, int& flag) {
    ROM_HIP(hipMemsetAsync(g_, 0, sizeof(double) * n_, st_));
    const double* rcur = r_;
    bool fp32 = true;
    int its = 0;
    for (;;) {
      const double rn = res * nb;
      if (fp32) {
        const double goal =
            std::min(0.5, std::max(std::max(inner_tol_, FP32_GOAL_MIN), 0.5 * tol_ / res));
        const int budget = std::min(maxit_ - its, std::max(64, (maxit_ - its) / 4));
        int f32 = 0;
        its += cg_solve<float>(rcur, 1.0 / rn, d32_, nj, goal, budget, f32);
        if (f32 != 0) {
          fp32 = false;   // FP32 breakdown: keep g, go on in FP64
          if (its < maxit_) continue;
          launch_axpby(n_, 1.0, xbase_, 1.0, g_, x, nullptr, red_part_, st_);
          break;
        }
        launch_refine_update(n_, rn, d32_, g_, xbase_, x, st_);
      } else {
        ++rec.fp64_sweeps;
        its += cg_solve<double>(rcur, 1.0, d_, nj, tol_ * nb, maxit_ - its, flag);
        launch_axpby(n_, 1.0, g_, 1.0, d_, g_, nullptr, red_part_, st_);
        launch_axpby(n_, 1.0, xbase_, 1.0, g_, x, &ctrl_->sc[6], red_part_, st_);
      }
      const double prev = res;
      res = true_residual(x, idx, sc, nb);
      if (res <= tol_ || its >= maxit_ || flag != 0 || restarts >= MAX_SWEEPS) break;
      ++restarts;
      if (fp32 && !(res <= 0.5 * prev)) fp32 = false;
      rcur = r2_;
    }
    return its;
  }

  // The CG vectors (q holds the q part of the split direction) and partials of the
  // operator step (po), the start (ps) and the update (pu), as the solve's type; s, q and w
  // of parity 1 at + pstride, the operator step's partials of parity 1 at po + pohalf.
  struct CgBufs32 {
    const float *W, *AW, *diag;
    float *s, *q, *w, *po, *ps, *pu;
    int64_t pstride, pohalf;
  };
  struct CgBufs64 {
    const double *W, *AW, *diag;
    double *s, *q, *w, *po, *ps, *pu;
    int64_t pstride, pohalf;
  };
  void bufs(CgBufs64& b) const {
    b = {Wp_, AWp_, diag_i_, s_, p_, w_, part_o_, part2_, part_u_, ld_ * G_, pos_ * G_};
  }
  void bufs(CgBufs32& b) const {
    b = {W32_, AW32_, diag32_, s32_, p32_, w32_, reinterpret_cast<float*>(part_o_),
         reinterpret_cast<float*>(part2_), reinterpret_cast<float*>(part_u_), ld_ * G_,
         pos_ * G_};
  }

  // One batched deflated-CG solve: member y (active[y]) solves A_i d_y = rscale[y] r_y
  // with the recycle space of slot y (slot 0 for every member when shared) until
  // ||s_y|| <= tol_abs[y] or maxit[y] steps.  r_y at rhs + y*ld_ (FP64), d_y at
  // dvec + y*ld_ (type T).
  struct Batch {
    int nb = 0;
    bool shared = false;
    int src = -1;   // slot of the shared leading columns (see make_W), -1: each its own
    int active[G_MAX] = {};
    int nj[G_MAX] = {};
    int maxit[G_MAX] = {};
    double rscale[G_MAX] = {};
    double tol_abs[G_MAX] = {};
    int its[G_MAX] = {};
    int flag[G_MAX] = {};
  };

  // Launch shape of the CG step kernels, encoded as (P << 5) | (quad << 4) | (narrow << 3) |
  // op: quad for the FP32 operator step's four-node walk (two-launch step only), P blocks
  // per member of the update kernel, narrow for its variant with half the rows per thread,
  // op the operator step's target block count per member (op_target; the fewer blocks, the
  // more z planes per thread and the fewer partial rows to reduce).  Fixed shape: the full
  // grid for one member, split among the members of a batch (narrow for batches), and the
  // four-node walk in FP32 where it applies.  With opts.tune the first batch of each
  // (arithmetic, batch size, U_j width class, grid size) in the process times every
  // power-of-two P with both variants, every operator target and, in FP32, both walks on
  // its own data (three rounds of 8 CG steps each after a warm-up round, from its real
  // start; the solve then restarts) and keeps the fastest (by its best round) for the rest
  // of the process.
  // Bit 2 of op selects the one-launch step (then P and narrow are unused): every block of
  // it sums all partial rows of the previous step, so only the 256 and 64 block targets are
  // candidates for it.
  static int shape_code(int P, int nr, int op, int quad = 0) {
    return (P << 5) | (quad << 4) | (nr << 3) | op;
  }
  static int shape_P(int code) { return code >> 5; }
  static bool shape_quad(int code) { return ((code >> 4) & 1) != 0; }
  static int shape_nr(int code) { return (code >> 3) & 1; }
  static bool shape_one(int code) { return (code & 4) != 0; }
  // op 0: 1024 blocks per member divided among the members (at least 64); 1, 2, 3: 1024,
  // 256, 64 blocks per member
  static int op_target(int code, int nb) {
    const int op = code & 3;
    return op == 0 ? std::max(64, 1024 / nb) : op == 1 ? 1024 : op == 2 ? 256 : 192;
  }
  template <typename T, typename Bufs>
  StencilShape op_shape(const Bufs& b, int code, int nb) const {
    return cg_apply_shape<T>(S_, op_target(code, nb), b.diag, b.q, b.w, ld_, b.AW,
                             shape_quad(code) && !shape_one(code));
  }

  template <typename T, typename Bufs>
  int cg_shape(const Batch& bt, const Bufs& b, const double* rhs, T* dvec, const Slots& sl,
               int64_t gstride, int njmax) {
    const int nb = bt.nb;
    const int Pmax = dcg_blocks(n_);
    const int mode = o_.cg_step;   // 0 either form (tuned) / two launches, 1 two, 2 one
    const int quad = sizeof(T) == 4 ? 1 : 0;
    const int fixed = mode == 2 ? shape_code(Pmax, 0, 4 | 2)
                                : shape_code(std::max(std::min(Pmax, 8), Pmax / nb),
                                             nb > 1 ? 1 : 0, 0, quad);
    if (!tune_) return fixed;
    int dev = 0;
    ROM_HIP(hipGetDevice(&dev));
    const TuneKey key{dev, (int)sizeof(T), nb, njt_of(njmax), (int64_t)n_, mode};
    {
      std::lock_guard<std::mutex> lk(tune_mu());
      auto it = tune_map().find(key);
      if (it != tune_map().end()) return it->second;
    }
    std::vector<int> cand;
    if (mode != 2)
      for (int P = Pmax; P >= 8; P /= 2)
        for (int nr = 0; nr < 2; ++nr)
          for (int op = 1; op <= 3; ++op)
            for (int qd = 0; qd <= quad; ++qd) cand.push_back(shape_code(P, nr, op, qd));
    if (mode != 1)
      for (int op = 2; op <= 3; ++op) cand.push_back(shape_code(Pmax, 0, 4 | op));
    int best = fixed;
    if (cand.size() > 1) {
      CGState* cg = ctrl_->cg;
      CgSetup su;
      std::memset(&su, 0, sizeof(su));
      for (int y = 0; y < nb; ++y) {
        su.tol2[y] = 0.0;
        su.rscale[y] = bt.rscale[y];
        su.maxit[y] = 1 << 30;
        su.nj[y] = bt.nj[y];
        su.active[y] = bt.active[y];
      }
      hipEvent_t e0, e1;
      ROM_HIP(hipEventCreate(&e0));
      ROM_HIP(hipEventCreate(&e1));
      struct Ev {
        hipEvent_t a, b;
        ~Ev() {
          (void)hipEventDestroy(a);
          (void)hipEventDestroy(b);
        }
      } guard{e0, e1};
      // each shape's time is the minimum over 3 rounds of 8 steps (the first round only
      // warms up): single short windows were noisy enough to flip the choice between runs.
      // Every window starts the solve afresh (untimed), so that both forms time the same
      // first 8 steps from the real start.
      std::vector<float> tmin(cand.size(), 1e30f);
      for (int rep = 0; rep < 4; ++rep) {
        for (size_t ci = 0; ci < cand.size(); ++ci) {
          const int shape = cand[ci];
          const int P = shape_P(shape), nr = shape_nr(shape);
          const StencilShape sh = op_shape<T>(b, shape, nb);
          launch_cg_setup(cg, cgv_, su, nb, st_);
          launch_dcg_start<T>(b.W, b.AW, sl, n_, njmax, GWinv_, gstride, rhs, ld_,
                              dvec, b.s, b.q, ld_, cg, b.ps, p2s_, nb, Pmax, st_);
          ROM_HIP(hipEventRecord(e0, st_));
          for (int step = 0; step < 8; ++step) {
            if (shape_one(shape)) {
              launch_dcg_iter<T>(S_, sh, b.diag, b.s, b.q, b.w, b.pstride, ld_, dvec, b.AW,
                                 sl, njmax, GWinv_, GWs_, gstride, cg, cgv_, b.ps,
                                 Pmax, p2s_, b.po, pos_, b.pohalf, sh.blocks, step & 1,
                                 step == 0, nb, st_);
            } else {
              launch_dcg_op<T>(S_, sh, b.diag, b.q, b.s, b.w, ld_, b.AW, sl, njmax,
                               GWinv_, GWs_, gstride, cg, cgv_, b.ps, Pmax, p2s_, b.pu, P,
                               pus_, b.po, pos_, nb, st_);
              launch_dcg_update<T>(b.q, b.w, dvec, b.s, ld_, n_, njmax, cg, cgv_, b.po,
                                   sh.blocks, pos_, b.pu, pus_, nb, P, st_, nr);
            }
          }
          ROM_HIP(hipEventRecord(e1, st_));
          ROM_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          ROM_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) tmin[ci] = std::min(tmin[ci], ms);
        }
      }
      float best_ms = 1e30f;
      for (size_t ci = 0; ci < cand.size(); ++ci)
        if (tmin[ci] < best_ms) {
          best_ms = tmin[ci];
          best = cand[ci];
        }
    }
    std::lock_guard<std::mutex> lk(tune_mu());
    tune_map()[key] = best;
    return best;
  }

  // A captured chunk of GRAPH_STEPS CG steps, replayed instead of individual launches:
  // (operator step, update) pairs, which take the step index from the CG state, or
  // one-launch steps of parities 1, 0, 1, ... (a chunk follows the eager step 0 or another
  // chunk).  One graph per (value type, batch size, shared recycle space, width class,
  // shape, slot and count of the shared leading columns, output vector), kept for the rest
  // of the call.
  template <typename T, typename Bufs>
  hipGraphExec_t chunk_graph(const Bufs& b, int nb, bool shared, int njmax, int shape,
                             const Slots& sl, int64_t gstride, T* dvec, const StencilShape& sh) {
    const GraphKey key{(int)sizeof(T), nb, shared ? 1 : 0, njt_of(njmax), shape, sl.soff, sl.ns,
                       (const void*)dvec};
    const int P = shape_P(shape), nr = shape_nr(shape);
    auto it = graphs_.find(key);
    if (it != graphs_.end()) return it->second;
    CGState* cg = ctrl_->cg;
    // captured on a private stream (the caller's may be the legacy default stream, which
    // cannot capture); the replays run on the caller's stream
    if (!cap_st_) ROM_HIP(hipStreamCreateWithFlags(&cap_st_, hipStreamNonBlocking));
    hipStream_t cs = cap_st_;
    hipGraph_t g = nullptr;
    const int P0 = dcg_blocks(n_);
    ROM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      for (int c = 0; c < GRAPH_STEPS; ++c) {
        if (shape_one(shape)) {
          launch_dcg_iter<T>(S_, sh, b.diag, b.s, b.q, b.w, b.pstride, ld_, dvec, b.AW, sl,
                             njmax, GWinv_, GWs_, gstride, cg, cgv_, b.ps, P0, p2s_, b.po,
                             pos_, b.pohalf, sh.blocks, (c + 1) & 1, 0, nb, cs);
          continue;
        }
        launch_dcg_op<T>(S_, sh, b.diag, b.q, b.s, b.w, ld_, b.AW, sl, njmax, GWinv_,
                         GWs_, gstride, cg, cgv_, b.ps, P0, p2s_, b.pu, P, pus_, b.po, pos_, nb,
                         cs);
        launch_dcg_update<T>(b.q, b.w, dvec, b.s, ld_, n_, njmax, cg, cgv_, b.po, sh.blocks,
                             pos_, b.pu, pus_, nb, P, cs, nr);
      }
    } catch (...) {
      hipGraph_t dummy = nullptr;
      (void)hipStreamEndCapture(cs, &dummy);
      if (dummy) (void)hipGraphDestroy(dummy);
      throw;
    }
    ROM_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Error(ROM_EHIP, "hipGraphInstantiate failed");
    graphs_[key] = ex;
    return ex;
  }

  template <typename T>
  void cg_batch(Batch& bt, const double* rhs, T* dvec) {
    typename std::conditional<std::is_same<T, float>::value, CgBufs32, CgBufs64>::type b;
    bufs(b);
    const int nb = bt.nb;
    CGState* cg = ctrl_->cg;
    const int64_t wstride = bt.shared ? 0 : ld_ * NJ_MAX;
    const int64_t gstride = bt.shared ? 0 : (int64_t)NJ_MAX * NJ_MAX;
    CgSetup su;
    std::memset(&su, 0, sizeof(su));
    int njmax = 0, nact = 0;
    for (int y = 0; y < nb; ++y) {
      bt.its[y] = bt.flag[y] = 0;
      su.tol2[y] = bt.tol_abs[y] * bt.tol_abs[y];
      su.rscale[y] = bt.rscale[y];
      su.maxit[y] = bt.maxit[y];
      su.nj[y] = bt.nj[y];
      su.active[y] = bt.active[y];
      if (bt.active[y]) {
        njmax = std::max(njmax, bt.nj[y]);
        ++nact;
      }
    }
    if (nact == 0) return;
    // after the first point every member's recycle space starts with the same ku_ columns
    // (U_0 and A_i U_0), built in the group's source slot only (make_W): the kernels read
    // them from there for every member
    Slots sl{wstride, ld_, 0, 0};
    if (!bt.shared && bt.src >= 0 && ku_ > 0) {
      sl.soff = bt.src * wstride;
      sl.ns = ku_;
    }
    const int shape = cg_shape<T>(bt, b, rhs, dvec, sl, gstride, njmax);
    const int P = shape_P(shape), nr = shape_nr(shape);
    // the operator step's shape (two x-nodes per thread where the layout allows); its block
    // count is the number of the operator step's partial rows per member
    const StencilShape sh = op_shape<T>(b, shape, nb);
    launch_cg_setup(cg, cgv_, su, nb, st_);
    // U_j^T r_j for the start
    if (njmax > 0) {
      if (bt.shared && nact > 1) {
        tm_->begin(ROM_K_GEMVT);
        launch_proj(Wp_, ld_, njmax, rhs, ld_, nb, n_, cg[0].t, sizeof(CGState) / sizeof(double),
                    gt_part_, st_);
        tm_->end(ROM_K_GEMVT, 8.0 * n_ * (njmax + nb), 2.0 * n_ * njmax * nb);
      } else if (!bt.shared && bt.src >= 0 && ku_ > 0) {
        // U_0's part of every member's U_j^T r from V's first ku_ columns in one projection
        // over the batch's right-hand sides (the values of inactive members are unused),
        // then each active member's own columns
        tm_->begin(ROM_K_GEMVT);
        launch_proj(Q_, ld_, ku_, rhs, ld_, nb, n_, cg[0].t, sizeof(CGState) / sizeof(double),
                    gt_part_, st_);
        tm_->end(ROM_K_GEMVT, 8.0 * n_ * (ku_ + nb), 2.0 * n_ * ku_ * nb);
        for (int y = 0; y < nb; ++y)
          if (bt.active[y] && bt.nj[y] > ku_) {
            const int ne = bt.nj[y] - ku_;
            tm_->begin(ROM_K_GEMVT);
            launch_gemvt(Wp_ + y * wstride + (int64_t)ku_ * ld_, ld_, n_, ne,
                         rhs + (int64_t)y * ld_, 0, 1, cg[y].t + ku_, gt_part_, st_);
            tm_->end(ROM_K_GEMVT, 8.0 * n_ * (ne + 1), 2.0 * n_ * ne);
          }
      } else {
        for (int y = 0; y < nb; ++y)
          if (bt.active[y] && bt.nj[y] > 0) {
            tm_->begin(ROM_K_GEMVT);
            launch_gemvt(Wp_ + y * wstride, ld_, n_, bt.nj[y], rhs + (int64_t)y * ld_, 0, 1,
                         cg[y].t, gt_part_, st_);
            tm_->end(ROM_K_GEMVT, 8.0 * n_ * (bt.nj[y] + 1), 2.0 * n_ * bt.nj[y]);
          }
      }
    }
    const double E = sizeof(T);
    double njavg = 0.0;
    for (int y = 0; y < nb; ++y)
      if (bt.active[y]) njavg += bt.nj[y];
    njavg /= nact;
    // the start runs once per solve on the full grid for every member (its 256-thread
    // blocks would leave the chip idle on the update's grid); the first operator step
    // reduces its partial rows
    const int P0 = dcg_blocks(n_);
    // the shared leading columns of U and AU count once per launch, the rest per member
    const double ns = sl.ns;
    tm_->begin(ROM_K_DCG_ENDS);
    launch_dcg_start<T>(b.W, b.AW, sl, n_, njmax, GWinv_, gstride, rhs, ld_, dvec, b.s,
                        b.q, ld_, cg, b.ps, p2s_, nb, P0, st_);
    tm_->end(ROM_K_DCG_ENDS, nact * (8.0 * n_ + E * n_ * (2 * (njavg - ns) + 3)) + 2 * E * n_ * ns,
             nact * n_ * (2.0 + 4.0 * njavg));
    // algorithmic bytes and flops per member and step: the operator step reads q, s and its
    // own columns of AU and writes w, and per launch reads the diagonal (and face
    // coefficients) and the shared columns of AU once for all its members; the update reads
    // q, w, g, s and writes q, g, s
    const double by_shared = E * n_ * (1 + (S_.var ? S_.dim : 0) + ns);
    const double by_op = E * n_ * (3 + njavg - ns);
    const double fl_op = n_ * (21.0 + 6.0 * njavg);
    const double by_upd = 7.0 * E * n_;
    const double fl_upd = 8.0 * n_;
    // the one-launch step reads s, q, w, g and its own columns of AU and writes s, q, w, g
    // per member (and the diagonal, faces and shared columns of AU once)
    const bool one = shape_one(shape);
    const double by_one = E * n_ * (8 + njavg - ns);
    const double fl_one = fl_op + fl_upd;
    int step = 0;   // one-launch steps launched (the next one's index)
    int next = chunk_;
    int its_before[G_MAX] = {};
    double gam_before[G_MAX];
    for (int y = 0; y < G_MAX; ++y) gam_before[y] = -1.0;
    int nlive = nact;
    int Pu = P;   // blocks of the update whose partials the next operator step sums
    // CG steps as replays of a captured chunk when asked for and no step kernel is timed
    const int cg_classes =
        (1 << ROM_K_DCG_OP) | (1 << ROM_K_DCG_UPDATE) | (1 << ROM_K_DCG_STEP);
    const bool graphs = graph_ && !(o_.timing & cg_classes);
    auto iter = [&](hipStream_t st) {
      launch_dcg_iter<T>(S_, sh, b.diag, b.s, b.q, b.w, b.pstride, ld_, dvec, b.AW, sl,
                         njmax, GWinv_, GWs_, gstride, cg, cgv_, b.ps, P0, p2s_, b.po,
                         pos_, b.pohalf, step == 0 ? P0 : sh.blocks, step & 1, step == 0, nb,
                         st);
      ++step;
    };
    for (;;) {
      if (one) {
        // launches in this chunk; step 0 (no update) runs eagerly before the first replay
        const bool had0 = step == 0;
        int launched = 0;
        if (graphs) {
          if (step == 0) {
            iter(st_);
            ++launched;
          }
          const int reps = std::max(1, (next - launched + GRAPH_STEPS - 1) / GRAPH_STEPS);
          hipGraphExec_t ex =
              chunk_graph<T>(b, nb, bt.shared, njmax, shape, sl, gstride, dvec, sh);
          for (int r = 0; r < reps; ++r) ROM_HIP(hipGraphLaunch(ex, st_));
          step += reps * GRAPH_STEPS;
          launched += reps * GRAPH_STEPS;
          for (int c = 0; c < launched; ++c)
            tm_->add(ROM_K_DCG_STEP, nlive * by_one + by_shared, nlive * fl_one);
        } else {
          for (int c = 0; c < next; ++c) {
            tm_->begin(ROM_K_DCG_STEP);
            iter(st_);
            tm_->end(ROM_K_DCG_STEP, nlive * by_one + by_shared, nlive * fl_one);
          }
          launched = next;
        }
        pull_cg(nb);
        // updates done per member in this chunk; a member's launches that did the whole
        // step are its updates plus step 0, then one more read its stopping test; launches
        // after the last member's stop returned at once
        int maxreal = 0, steps = 0, still = 0;
        for (int y = 0; y < nb; ++y) {
          if (!bt.active[y] || its_before[y] < 0) continue;
          const CGState& c = h_->cg[y];
          const int real = c.its - its_before[y];
          maxreal = std::max(maxreal, real);
          steps += real;
          if (c.done) {
            its_before[y] = -1;
          } else {
            ++still;
            its_before[y] = c.its;
          }
        }
        const bool stop = still == 0;
        // (a stop read by step 0 itself: that one launch)
        const int counted = had0 && maxreal == 0 ? 1 : maxreal + (had0 ? 1 : 0) + 1;
        tm_->discard(ROM_K_DCG_STEP, stop ? launched - counted : 0, by_shared, 0.0);
        const double over = (double)nlive * launched - steps - (had0 ? nlive : 0);
        tm_->adjust(ROM_K_DCG_STEP, -over * by_one, -over * fl_one);
        tm_->harvest();
        if (stop) break;
        int pred = 2;
        for (int y = 0; y < nb; ++y) {
          if (!bt.active[y] || its_before[y] < 0) continue;
          const CGState& c = h_->cg[y];
          const double gam = c.gamma[c.its & 1];
          int py = chunk_;
          if (gam_before[y] > 0.0 && gam > 0.0 && gam < gam_before[y] && launched > 0) {
            const double rate = std::log(gam / gam_before[y]) / launched;   // < 0
            py = (int)std::ceil(POLL_MARGIN * std::log(c.tol2 / gam) / rate) + POLL_PAD;
          }
          pred = std::max(pred, py);
          gam_before[y] = gam;
        }
        nlive = still;
        next = std::min(64, std::max(2, pred));
        continue;
      }
      if (graphs) {
        const int reps = (next + GRAPH_STEPS - 1) / GRAPH_STEPS;
        hipGraphExec_t ex =
            chunk_graph<T>(b, nb, bt.shared, njmax, shape, sl, gstride, dvec, sh);
        for (int r = 0; r < reps; ++r) ROM_HIP(hipGraphLaunch(ex, st_));
        next = reps * GRAPH_STEPS;
        for (int c = 0; c < next; ++c) {
          tm_->add(ROM_K_DCG_OP, nlive * by_op + by_shared, nlive * fl_op);
          tm_->add(ROM_K_DCG_UPDATE, nlive * by_upd, nlive * fl_upd);
        }
      }
      for (int c = 0; c < (graphs ? 0 : next); ++c) {
        tm_->begin(ROM_K_DCG_OP);
        launch_dcg_op<T>(S_, sh, b.diag, b.q, b.s, b.w, ld_, b.AW, sl, njmax, GWinv_,
                         GWs_, gstride, cg, cgv_, b.ps, P0, p2s_, b.pu, Pu, pus_, b.po, pos_, nb,
                         st_);
        tm_->end(ROM_K_DCG_OP, nlive * by_op + by_shared, nlive * fl_op);
        tm_->begin(ROM_K_DCG_UPDATE);
        launch_dcg_update<T>(b.q, b.w, dvec, b.s, ld_, n_, njmax, cg, cgv_, b.po, sh.blocks,
                             pos_, b.pu, pus_, nb, P, st_, nr);
        tm_->end(ROM_K_DCG_UPDATE, nlive * by_upd, nlive * fl_upd);
        Pu = P;
      }
      pull_cg(nb);
      // member-steps (updates) done in this chunk; once the last member stopped, the
      // launches after the operator step that stopped it returned at once
      int maxreal = 0, steps = 0, still = 0;
      for (int y = 0; y < nb; ++y) {
        if (!bt.active[y] || its_before[y] < 0) continue;
        const CGState& c = h_->cg[y];
        const int real = c.its - its_before[y];
        maxreal = std::max(maxreal, real);
        steps += real;
        if (c.done) {
          its_before[y] = -1;
        } else {
          ++still;
          its_before[y] = c.its;
        }
      }
      const bool stop = still == 0;
      tm_->discard(ROM_K_DCG_OP, stop ? next - maxreal - 1 : 0, by_shared, 0.0);
      tm_->discard(ROM_K_DCG_UPDATE, stop ? next - maxreal : 0, 0.0, 0.0);
      const double over = (double)nlive * next - steps;
      tm_->adjust(ROM_K_DCG_OP, -over * by_op, -over * fl_op);
      tm_->adjust(ROM_K_DCG_UPDATE, -over * by_upd, -over * fl_upd);
      tm_->harvest();
      if (stop) break;
      // next poll: extrapolate each live member's contraction of s^T s to its tolerance
      int pred = 2;
      for (int y = 0; y < nb; ++y) {
        if (!bt.active[y] || its_before[y] < 0) continue;
        const CGState& c = h_->cg[y];
        const double gam = c.gamma[c.its & 1];
        int py = chunk_;
        if (gam_before[y] > 0.0 && gam > 0.0 && gam < gam_before[y] && next > 0) {
          const double rate = std::log(gam / gam_before[y]) / next;   // < 0
          py = (int)std::ceil(POLL_MARGIN * std::log(c.tol2 / gam) / rate) + POLL_PAD;
        }
        pred = std::max(pred, py);
        gam_before[y] = gam;
      }
      nlive = still;
      next = std::min(64, std::max(2, pred));
    }
    // the correction: g = g_q - U e
    tm_->begin(ROM_K_DCG_ENDS);
    launch_dcg_finish<T>(b.W, sl, n_, njmax, dvec, ld_, cg, cgv_, nb, st_);
    tm_->end(ROM_K_DCG_ENDS, nact * E * n_ * (2 + njavg - ns) + E * n_ * ns,
             nact * 2.0 * n_ * njavg);
    for (int y = 0; y < nb; ++y) {
      if (!bt.active[y]) continue;
      bt.its[y] = h_->cg[y].its;
      bt.flag[y] = h_->cg[y].flag;
    }
  }

  // Deflated CG on A_i d = rscale * rhs with the recycle space in slot 0, in arithmetic T
  // (the right-hand side is FP64); stops at ||s|| <= tol_abs.  Returns iterations.
  template <typename T>
  int cg_solve(const double* rhs, double rscale, T* dvec, int nj, double tol_abs, int maxit,
               int& flag) {
    Batch bt;
    bt.nb = 1;
    bt.shared = true;
    bt.active[0] = 1;
    bt.nj[0] = nj;
    bt.maxit[0] = maxit;
    bt.rscale[0] = rscale;
    bt.tol_abs[0] = tol_abs;
    cg_batch<T>(bt, rhs, dvec);
    flag = bt.flag[0];
    return bt.its[0];
  }

  rom_operator* op_;
  Stencil S_;
  int64_t n_, ld_;
  int n_src_, n_det_, n_rhs_, K_, ku_in_;
  rom_opts o_;
  int cap_, ldg_, pool_cap_;
  double tol_, trunc_;
  int maxit_, chunk_;
  int G_ = 1;                // right-hand sides per group
  int cur_point_ = 0;
  int64_t pos_ = 0, p2s_ = 0, pus_ = 0;   // per-member strides of the CG partials
  bool mixed_ = false;
  bool tune_ = false;
  bool graph_ = false;
  const float* guess_ = nullptr;   // per (point, RHS) initial guesses (FP32, N each)
  const float* recycle_ = nullptr; // per point learned recycle vectors (FP32, N each)
  int n_rec_ = 0, n_rec_kept_ = 0;
  double* rec_ = nullptr;          // the current point's kept recycle vectors (ld x REC_MAX)
  double* rAW_ = nullptr;          // A_i times them
  double* rtb_ = nullptr;          // V^T A_i w, then G_i^{-1} V^T A_i w
  double* rub_ = nullptr;
  const double* xbase_ = nullptr;  // base point of the current inner solve
  using GraphKey = std::tuple<int, int, int, int, int, int64_t, int, const void*>;
  std::map<GraphKey, hipGraphExec_t> graphs_;
  hipStream_t cap_st_ = nullptr;   // capture stream of the graphs
  double inner_tol_ = 1e-5;
  hipStream_t st_ = nullptr;
  Timer* tm_ = nullptr;
  Ctrl* h_ = nullptr;
  unsigned* hflag_ = nullptr;   // publish flag (host view)
  void* dh_ = nullptr;          // device view of h_
  unsigned* dflag_ = nullptr;   // device view of the flag
  unsigned seq_ = 0;
  double mu0_ = 0.0;
  int m_ = 0, ku_ = 0, next_slot_ = 0;
  int w_key_[G_MAX], w_nj_[G_MAX] = {}, w_src_[G_MAX] = {};
  bool w_full_[G_MAX] = {};   // the slot holds U_0's columns too (see make_W)
  // results
  std::vector<rom_record> recs_;
  rom_status status_ = ROM_OK;
  long long total_its_ = 0;
  int n_solved_ = 0, n_kept_ = 0, n_drop_trunc_ = 0, n_drop_cap_ = 0, n_nonconv_ = 0;
  int n_uj_capped_ = 0;
  int next_point_ = 0;
  const double* U0_ = nullptr;
  std::unique_ptr<Timer> timer_;
  std::chrono::steady_clock::time_point t0_;
  rom_basis view_{};
  std::vector<std::vector<int>> extra_;
  std::vector<int64_t> idx_;
  std::vector<double> scale_;
  // device buffers
  double *Q_, *pool_, *Wp_, *AWp_, *x0_, *r_, *g_, *s_, *p_, *w_, *d_, *xt_, *r2_, *vAB_;
  double *blk_ = nullptr, *bblk_ = nullptr;   // block append: A Q_new, its projections
  double* xg_ = nullptr;                       // start moved by an initial guess
  double *diag_i_, *dmu_, *Gs_, *Gi_, *Lc_, *Lr_, *gram_part_, *red_part_, *gt_part_;
  // bump-row compaction of the current point: V^T (dmu o q) and V^T diag(dmu) V only read
  // the rows where dmu != 0, so V is kept gathered on them (Vb, nzr_ x m, ld ldb_)
  double *Vb_ = nullptr, *dmub_ = nullptr, *zb_ = nullptr;
  int64_t* bidx_ = nullptr;
  int* nzwork_ = nullptr;
  int64_t nzcap_ = 0, ldb_ = 0, nzr_ = 0;
  bool compact_ = false;
  double *tbuf_, *ubuf_, *cbuf_, *tmpl_, *tmpr_, *bvals_, *GWs_, *LWinv_, *GWinv_, *lwork_;
  // the next right-hand side's start fused into an append's first Gram-Schmidt pass:
  // fa_ = V y, fw_ = V w (y = G_i^{-1} V^T b_next, w = G_i^{-1} V^T A_i u)
  double *fa_ = nullptr, *fw_ = nullptr, *fcw_ = nullptr, *ftmp_ = nullptr;
  struct {
    bool on = false;
    int64_t idx = 0;
    double sc = 0.0;
  } fuse_next_;
  bool fused_ready_ = false, fused_kept_ = false;
  double fused_rho_ = 0.0;
  Ctrl* ctrl_;
  double *part_o_, *part2_, *part_u_;
  CGVec* cgv_ = nullptr;
  // mixed form: FP32 copies of U_j, A U_j, the diagonal and the face coefficients, and the
  // FP32 CG vectors
  float *W32_ = nullptr, *AW32_ = nullptr, *s32_ = nullptr, *p32_ = nullptr, *w32_ = nullptr;
  float *d32_ = nullptr, *diag32_ = nullptr, *fx32_ = nullptr, *fy32_ = nullptr, *fz32_ = nullptr;
  int64_t* idx_dev_;
  double* scale_dev_;
};

rom_status fail(const Error& e) {
  g_err = e.what();
  return e.code;
}

void check_opts(const rom_opts* o) {
  if (!o) throw Error(ROM_EINVAL, "null options");
  if (!(o->tol > 0) || !std::isfinite(o->tol)) throw Error(ROM_EINVAL, "tol must be > 0");
  if (!(o->trunc >= 0) || !std::isfinite(o->trunc)) throw Error(ROM_EINVAL, "trunc must be >= 0");
  if (o->cap < 0 || o->cap > 4096) throw Error(ROM_EINVAL, "cap must be in [0, 4096]");
  if (o->maxit < 0 || o->check_every < 0) throw Error(ROM_EINVAL, "maxit/check_every must be >= 0");
  if (o->precision != ROM_PREC_FP64 && o->precision != ROM_PREC_MIXED)
    throw Error(ROM_EINVAL, "precision must be ROM_PREC_FP64 or ROM_PREC_MIXED");
  if (!(o->inner_tol >= 0) || !(o->inner_tol < 1)) throw Error(ROM_EINVAL, "inner_tol must be in [0, 1)");
  if (o->group < 0 || o->group > G_MAX) throw Error(ROM_EINVAL, "group must be in [0, 16]");
  if (o->tune != 0 && o->tune != 1) throw Error(ROM_EINVAL, "tune must be 0 or 1");
  if (o->graph != 0 && o->graph != 1) throw Error(ROM_EINVAL, "graph must be 0 or 1");
  if (o->cg_step < 0 || o->cg_step > 2) throw Error(ROM_EINVAL, "cg_step must be 0, 1 or 2");
  if (o->recycle && (o->n_recycle < 1 || o->n_recycle > REC_MAX))
    throw Error(ROM_EINVAL, "n_recycle must be in [1, 16]");
}

void check_counts(int n_src, int n_det, int k_u, int K) {
  if (n_src < 0 || n_det < 0 || n_src + n_det < 1) throw Error(ROM_EINVAL, "need at least one RHS");
  if (k_u < 0 || k_u >= NJ_MAX) throw Error(ROM_EINVAL, "k_u must be in [0, 63]");
  if (K < 1) throw Error(ROM_EINVAL, "K must be >= 1");
  if ((int64_t)n_src + n_det > 100000) throw Error(ROM_EINVAL, "too many right-hand sides");
}

}  // namespace

rom_status report(const Error& e) { return fail(e); }
void report_message(const std::string& m) { g_err = m; }

namespace {

// The diagonal of A(p) for rom_apply_operator_static.  A file-scope device array exists
// once on every device that loads the library; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in, not a device address).
static __device__ __align__(256) double static_scratch[ROM_STATIC_MAX_N];

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex& static_scratch_mu() {
  static std::mutex m;
  return m;
}
double* static_scratch_ptr[STATIC_MAX_DEVICES] = {};

}  // namespace

// Device address of static_scratch on the current device, looked up once per device.
double* static_scratch_device() {
  int dev = 0;
  ROM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) throw Error(ROM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(static_scratch_mu());
  if (!static_scratch_ptr[dev]) {
    void* p = nullptr;
    ROM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(static_scratch)));
    if (!p) throw Error(ROM_EHIP, "hipGetSymbolAddress returned a null address");
    static_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return static_scratch_ptr[dev];
}

}  // namespace rom

using rom::Error;

extern "C" {

const char* rom_last_error(void) { return rom::g_err.c_str(); }

rom_status rom_operator_bytes(const rom_grid* grid, int variable_D, size_t* bytes) {
  try {
    rom::check_grid(grid);
    if (!bytes) throw Error(ROM_EINVAL, "null bytes");
    rom::Arena a(nullptr);
    *bytes = rom::operator_layout(*grid, variable_D != 0, a, nullptr) + rom::ALIGN;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_assemble_operator(const rom_grid* grid, double D_const, const double* D_field,
                                 void* op_mem, size_t op_bytes, rom_operator** op,
                                 void* stream) {
  try {
    rom::check_grid(grid);
    if (!op || !op_mem) throw Error(ROM_EINVAL, "null operator memory or handle");
    if (!D_field && (!(D_const > 0) || !std::isfinite(D_const)))
      throw Error(ROM_EINVAL, "constant D must be > 0");
    const bool var = D_field != nullptr;
    rom::Arena sizing(nullptr);
    const size_t need = rom::operator_layout(*grid, var, sizing, nullptr);
    if (op_bytes < need) throw Error(ROM_ECAPACITY, "operator memory too small");
    if ((uintptr_t)op_mem % 16) throw Error(ROM_EINVAL, "operator memory must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    rom_operator* o = new rom_operator;
    o->grid = *grid;
    o->n = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    o->var = var;
    o->Dc = D_const;
    rom::Arena a(op_mem);
    rom::operator_layout(*grid, var, a, o);
    try {
      rom::launch_assemble(*grid, D_const, D_field, o->diag_star, o->fx, o->fy, o->fz, st);
      if (var)
        ROM_HIP(hipMemcpyAsync(o->Dfield, D_field, sizeof(double) * o->n, hipMemcpyDeviceToDevice,
                               st));
    } catch (...) {
      delete o;
      throw;
    }
    rom::Stencil& S = o->S;
    S.nx = grid->n[0];
    S.ny = grid->n[1];
    S.nz = grid->n[2];
    S.dim = grid->dim;
    S.n = o->n;
    S.var = var ? 1 : 0;
    const double hx = 1.0 / (S.nx + 1), hy = 1.0 / (S.ny + 1), hz = 1.0 / (S.nz + 1);
    S.cx = var ? 0.0 : D_const / (hx * hx);
    S.cy = var ? 0.0 : D_const / (hy * hy);
    S.cz = (var || grid->dim == 2) ? 0.0 : D_const / (hz * hz);
    S.fx = o->fx;
    S.fy = o->fy;
    S.fz = o->fz;
    *op = o;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

void rom_operator_destroy(rom_operator* op) { delete op; }

rom_status rom_apply_operator(const rom_operator* op, const rom_mu* p, const double* X,
                              double* Y, int k, void* scratch, size_t scratch_bytes,
                              void* stream) {
  try {
    if (!op || !X || !Y) throw Error(ROM_EINVAL, "null argument");
    rom::check_mu(p, op->grid.dim);
    if (k < 0) throw Error(ROM_EINVAL, "k must be >= 0");
    if (!scratch || scratch_bytes < sizeof(double) * (size_t)op->n)
      throw Error(ROM_ECAPACITY, "scratch too small");
    if (k == 0) return ROM_OK;
    hipStream_t st = (hipStream_t)stream;
    double* diag = (double*)scratch;
    // diag(A(p)) = diag(A_*) + mu(p); the bump part goes through Y's first column as
    // temporary storage before the product overwrites it
    rom::launch_mu_eval(op->S, rom::make_bumps(*p, op->grid.dim), op->diag_star, diag, Y, st);
    rom::launch_spmm(op->S, diag, X, op->n, k, Y, st);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_apply_operator_static(const rom_operator* op, const rom_mu* p, const double* X,
                                     double* Y, int k, void* stream) {
  try {
    if (!op || !X || !Y) throw Error(ROM_EINVAL, "null argument");
    rom::check_mu(p, op->grid.dim);
    if (k < 0) throw Error(ROM_EINVAL, "k must be >= 0");
    if (op->n > ROM_STATIC_MAX_N)
      throw Error(ROM_ECAPACITY, "rom_apply_operator_static: N = " + std::to_string(op->n) +
                                     " exceeds ROM_STATIC_MAX_N = " +
                                     std::to_string(ROM_STATIC_MAX_N));
    if (k == 0) return ROM_OK;
    hipStream_t st = (hipStream_t)stream;
    // every entry of the diagonal is written before the product reads it
    double* diag = rom::static_scratch_device();
    rom::launch_mu_eval(op->S, rom::make_bumps(*p, op->grid.dim), op->diag_star, diag, Y, st);
    rom::launch_spmm(op->S, diag, X, op->n, k, Y, st);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_sequence_bytes(const rom_operator* op, int n_src, int n_det, int k_u, int K,
                              const rom_opts* opts, size_t* bytes) {
  try {
    if (!op || !bytes) throw Error(ROM_EINVAL, "null argument");
    rom::check_opts(opts);
    rom::check_counts(n_src, n_det, k_u, K);
    rom::Sequencer s(const_cast<rom_operator*>(op), n_src, n_det, k_u, K, *opts);
    *bytes = s.layout(nullptr);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

}  // extern "C"

namespace rom {
namespace {
// Arguments shared by rom_solve_sequence and rom_sequence_begin.
void check_sequence_args(rom_operator* op, int K, const int64_t* src_idx, const double* src_scale,
                         int n_src, const int64_t* det_idx, const double* det_scale, int n_det,
                         const double* U0, int k_u, const rom_opts* opts, void* workspace) {
  if (!op || !workspace) throw Error(ROM_EINVAL, "null operator or workspace");
  check_opts(opts);
  check_counts(n_src, n_det, k_u, K);
  if (k_u > 0 && !U0) throw Error(ROM_EINVAL, "null U0 with k_u > 0");
  if ((n_src > 0 && (!src_idx || !src_scale)) || (n_det > 0 && (!det_idx || !det_scale)))
    throw Error(ROM_EINVAL, "null source/detector arrays");
  for (int j = 0; j < n_src + n_det; ++j) {
    const int64_t idx = j < n_src ? src_idx[j] : det_idx[j - n_src];
    const double sc = j < n_src ? src_scale[j] : det_scale[j - n_src];
    if (idx < 0 || idx >= op->n) throw Error(ROM_EINVAL, "source/detector index out of range");
    if (!(sc != 0.0) || !std::isfinite(sc)) throw Error(ROM_EINVAL, "scale must be finite and nonzero");
  }
  if ((uintptr_t)workspace % 16) throw Error(ROM_EINVAL, "workspace must be 16-byte aligned");
}
}  // namespace
}  // namespace rom

// A sequence solved one parameter point at a time (rom_sequence_begin/point/end).
struct rom_sequence {
  std::unique_ptr<rom::Sequencer> s;
  bool failed = false;
};

extern "C" {

rom_status rom_sequence_begin(rom_operator* op, int K, const int64_t* src_idx,
                              const double* src_scale, int n_src, const int64_t* det_idx,
                              const double* det_scale, int n_det, const double* U0, int k_u,
                              const rom_opts* opts, void* workspace, size_t ws_bytes,
                              rom_sequence** seq, void* stream) {
  try {
    if (!seq) throw Error(ROM_EINVAL, "null sequence handle");
    *seq = nullptr;
    rom::check_sequence_args(op, K, src_idx, src_scale, n_src, det_idx, det_scale, n_det, U0,
                             k_u, opts, workspace);
    std::unique_ptr<rom_sequence> h(new rom_sequence);
    h->s.reset(new rom::Sequencer(op, n_src, n_det, k_u, K, *opts));
    const size_t need = h->s->layout(nullptr);
    if (ws_bytes < need) throw Error(ROM_ECAPACITY, "workspace too small");
    h->s->layout(workspace);
    h->s->begin(src_idx, src_scale, det_idx, det_scale, U0, (hipStream_t)stream);
    *seq = h.release();
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  } catch (const std::exception& e) {
    rom::g_err = e.what();
    return ROM_EHIP;
  }
}

rom_status rom_sequence_point(rom_sequence* seq, const rom_mu* p, double* X_out,
                              rom_record* records) {
  try {
    if (!seq || !seq->s) throw Error(ROM_EINVAL, "null sequence");
    if (seq->failed) throw Error(ROM_EINVAL, "the sequence stopped at an earlier error");
    rom::check_mu(p, seq->s->grid_dim());
    if (seq->s->points_done() >= seq->s->points_max())
      throw Error(ROM_EINVAL, "the sequence was sized for " +
                                  std::to_string(seq->s->points_max()) + " points");
    try {
      return seq->s->point(*p, X_out, records);
    } catch (...) {
      seq->failed = true;
      throw;
    }
  } catch (const Error& e) {
    return rom::fail(e);
  } catch (const std::exception& e) {
    rom::g_err = e.what();
    return ROM_EHIP;
  }
}

rom_status rom_sequence_basis(rom_sequence* seq, const rom_basis** V) {
  try {
    if (!seq || !seq->s || !V) throw Error(ROM_EINVAL, "null argument");
    if (seq->failed) throw Error(ROM_EINVAL, "the sequence stopped at an earlier error");
    *V = seq->s->basis_view();
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_sequence_stats(rom_sequence* seq, rom_stats* stats) {
  try {
    if (!seq || !seq->s || !stats) throw Error(ROM_EINVAL, "null argument");
    seq->s->report(nullptr, stats);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_sequence_end(rom_sequence* seq, rom_basis** basis, rom_stats* stats) {
  try {
    if (!seq) throw Error(ROM_EINVAL, "null sequence");
    std::unique_ptr<rom_sequence> h(seq);
    if (basis) *basis = nullptr;
    if (h->failed) throw Error(ROM_EINVAL, "the sequence stopped at an earlier error");
    h->s->report(nullptr, stats);
    if (basis) *basis = h->s->make_basis();
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  } catch (const std::exception& e) {
    rom::g_err = e.what();
    return ROM_EHIP;
  }
}

rom_status rom_solve_sequence(rom_operator* op, const rom_mu* params, int K,
                              const int64_t* src_idx, const double* src_scale, int n_src,
                              const int64_t* det_idx, const double* det_scale, int n_det,
                              const double* U0, int k_u, const rom_opts* opts, void* workspace,
                              size_t ws_bytes, rom_basis** basis, double* X_out,
                              rom_record* records, rom_stats* stats, void* stream) {
  try {
    if (!op || !basis || !workspace) throw Error(ROM_EINVAL, "null operator, basis or workspace");
    rom::check_opts(opts);
    rom::check_counts(n_src, n_det, k_u, K);
    if (!params) throw Error(ROM_EINVAL, "null params");
    for (int i = 0; i < K; ++i) rom::check_mu(&params[i], op->grid.dim);
    if (k_u > 0 && !U0) throw Error(ROM_EINVAL, "null U0 with k_u > 0");
    if ((n_src > 0 && (!src_idx || !src_scale)) || (n_det > 0 && (!det_idx || !det_scale)))
      throw Error(ROM_EINVAL, "null source/detector arrays");
    for (int j = 0; j < n_src + n_det; ++j) {
      const int64_t idx = j < n_src ? src_idx[j] : det_idx[j - n_src];
      const double sc = j < n_src ? src_scale[j] : det_scale[j - n_src];
      if (idx < 0 || idx >= op->n) throw Error(ROM_EINVAL, "source/detector index out of range");
      if (!(sc != 0.0) || !std::isfinite(sc)) throw Error(ROM_EINVAL, "scale must be finite and nonzero");
    }
    if ((uintptr_t)workspace % 16) throw Error(ROM_EINVAL, "workspace must be 16-byte aligned");
    rom::Sequencer s(op, n_src, n_det, k_u, K, *opts);
    const size_t need = s.layout(nullptr);
    if (ws_bytes < need) throw Error(ROM_ECAPACITY, "workspace too small");
    s.layout(workspace);
    *basis = nullptr;
    return s.run(params, src_idx, src_scale, det_idx, det_scale, U0, X_out, records, stats,
                 (hipStream_t)stream, basis);
  } catch (const Error& e) {
    return rom::fail(e);
  } catch (const std::exception& e) {
    rom::g_err = e.what();
    return ROM_EHIP;
  }
}

rom_status rom_solve_sequences(rom_sequence_job* jobs, int count) {
  try {
    if (!jobs || count < 1) throw Error(ROM_EINVAL, "need at least one job");
    int dev = 0;
    ROM_HIP(hipGetDevice(&dev));
    std::vector<std::thread> th;
    th.reserve(count);
    for (int q = 0; q < count; ++q) {
      th.emplace_back([dev, q, jobs]() {
        rom_sequence_job& j = jobs[q];
        j.message[0] = 0;
        if (hipSetDevice(dev) != hipSuccess) {
          j.status = ROM_EHIP;
          std::snprintf(j.message, sizeof(j.message), "hipSetDevice failed");
          return;
        }
        j.status = rom_solve_sequence(j.op, j.params, j.K, j.src_idx, j.src_scale, j.n_src,
                                      j.det_idx, j.det_scale, j.n_det, j.U0, j.k_u, j.opts,
                                      j.workspace, j.ws_bytes, j.basis, j.X_out, j.records,
                                      j.stats, j.stream);
        if (j.status != ROM_OK)
          std::snprintf(j.message, sizeof(j.message), "%s", rom_last_error());
      });
    }
    for (auto& t : th) t.join();
    rom_status agg = ROM_OK;
    for (int q = 0; q < count; ++q) {
      const rom_status st = jobs[q].status;
      if (st != ROM_OK && st != ROM_ENOCONV) {
        rom::g_err = "job " + std::to_string(q) + ": " + jobs[q].message;
        return st;
      }
      if (st == ROM_ENOCONV) agg = ROM_ENOCONV;
    }
    return agg;
  } catch (const Error& e) {
    return rom::fail(e);
  } catch (const std::exception& e) {
    rom::g_err = e.what();
    return ROM_EHIP;
  }
}

rom_status rom_seednet_inputs(const rom_operator* op, const rom_mu* p, const int64_t* idx,
                              int count, float* out, void* scratch, size_t scratch_bytes,
                              void* stream) {
  try {
    if (!op || !p || !idx || !out || !scratch) throw Error(ROM_EINVAL, "null argument");
    if (count < 1) throw Error(ROM_EINVAL, "count must be >= 1");
    rom::check_mu(p, op->grid.dim);
    for (int b = 0; b < count; ++b)
      if (idx[b] < -1 || idx[b] >= op->n) throw Error(ROM_EINVAL, "node index out of range");
    if (scratch_bytes < 8 * (size_t)(op->n + count)) throw Error(ROM_ECAPACITY, "scratch too small");
    if ((uintptr_t)scratch % 8) throw Error(ROM_EINVAL, "scratch must be 8-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    double* dmu = (double*)scratch;
    int64_t* didx = (int64_t*)(dmu + op->n);
    ROM_HIP(hipMemcpyAsync(didx, idx, sizeof(int64_t) * count, hipMemcpyHostToDevice, st));
    rom::launch_mu_eval(op->S, rom::make_bumps(*p, op->grid.dim), op->diag_star, nullptr, dmu, st);
    rom::launch_seed_inputs(op->n, count, dmu, 0.03, op->var ? op->Dfield : nullptr, op->Dc, 0.03,
                            didx, out, st);
    ROM_HIP(hipStreamSynchronize(st));   // idx is pageable host memory
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

namespace rom {
namespace {

constexpr int SUBSPACE_MAX = 16;   // network outputs (recycle vectors) per sample

struct SubspaceLayout {
  double *Nd, *Xn, *R, *dN, *G, *Linv, *Ginv, *C, *T, *Z, *n2, *part;
  int* status;
  int64_t ld;
  size_t bytes;
};

SubspaceLayout subspace_layout(int64_t N, int k, int s, void* base) {
  Arena a(base);
  SubspaceLayout L;
  L.ld = round_up(N, 64);
  L.Nd = a.take<double>(L.ld * k);
  L.Xn = a.take<double>(L.ld * s);
  L.R = a.take<double>(L.ld * s);
  L.dN = a.take<double>(L.ld * k);
  L.G = a.take<double>(k * k);
  L.Linv = a.take<double>(k * k);
  L.Ginv = a.take<double>(k * k);
  L.C = a.take<double>((size_t)k * s);
  L.T = a.take<double>((size_t)k * s);
  L.Z = a.take<double>((size_t)s * k);
  L.n2 = a.take<double>(s);
  L.part = a.take<double>(std::max<size_t>({gram_partials(k, k, N, true),
                                            gram_partials(k, s, N, false), (size_t)256 * s}));
  L.status = a.take<int>(4);
  L.bytes = a.off + ALIGN;
  return L;
}

}  // namespace
}  // namespace rom

rom_status rom_subspace_loss_bytes(int64_t N, int k, int s, size_t* bytes) {
  try {
    if (!bytes) throw Error(ROM_EINVAL, "null argument");
    if (N < 1 || k < 1 || k > rom::SUBSPACE_MAX || s < 1) throw Error(ROM_EINVAL, "bad sizes");
    *bytes = rom::subspace_layout(N, k, s, nullptr).bytes;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_subspace_loss(const float* Y, int k, const double* X, int64_t N, int64_t ldx, int s,
                             double* loss, float* dY, void* scratch, size_t scratch_bytes,
                             void* stream) {
  try {
    if (!Y || !X || !loss) throw Error(ROM_EINVAL, "null argument");
    if (N < 1 || k < 1 || k > rom::SUBSPACE_MAX || s < 1 || ldx < N)
      throw Error(ROM_EINVAL, "bad sizes");
    const rom::SubspaceLayout L = rom::subspace_layout(N, k, s, scratch);
    if (!scratch || scratch_bytes < L.bytes) throw Error(ROM_ECAPACITY, "scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const int64_t ld = L.ld;
    // N (FP64) and the unit-norm targets
    rom::launch_convert_cols(N, k, Y, N, L.Nd, ld, st);
    rom::launch_col_norms(N, s, X, ldx, L.n2, L.part, st);
    rom::launch_scale_cols(N, s, X, ldx, L.n2, L.Xn, ld, st);
    // G = N^T N, C = N^T X^, G^{-1}; T = G^{-1} C; R = X^ - N T
    rom::launch_gram(L.Nd, ld, k, L.Nd, ld, k, N, nullptr, true, nullptr, 0, 0.0, L.G, k, L.part,
                     st);
    rom::launch_gram(L.Nd, ld, k, L.Xn, ld, s, N, nullptr, false, nullptr, 0, 0.0, L.C, k, L.part,
                     st);
    ROM_HIP(hipMemsetAsync(L.status, 0, sizeof(int), st));
    rom::launch_small_chol_inv(L.G, k, L.Linv, L.Ginv, L.status, st);
    rom::launch_gemm(k, s, k, 1.0, L.Ginv, k, false, L.C, k, false, 0.0, nullptr, 0, L.T, k, st);
    for (int c = 0; c < s; c += 16)
      rom::launch_gemvn_multi(L.Nd, ld, N, k, L.T + (size_t)c * k, k, std::min(16, s - c), 1.0,
                              L.Xn + c * ld, ld, -1.0, L.R + c * ld, ld, st);
    // loss = sum_c ||R_c||^2 / s
    rom::launch_col_norms(N, s, L.R, ld, L.n2, L.part, st);
    std::vector<double> r2(s), hG((size_t)k * k), hL((size_t)k * k);
    int status = 0;
    ROM_HIP(hipMemcpyAsync(r2.data(), L.n2, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    ROM_HIP(hipMemcpyAsync(&status, L.status, sizeof(int), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipMemcpyAsync(hG.data(), L.G, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    ROM_HIP(hipMemcpyAsync(hL.data(), L.Linv, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    // pivot c of the Cholesky factorisation of G is 1 / Linv[c][c]^2: an output whose pivot
    // is below 1e-12 of its own squared norm lies in the span of the outputs before it
    for (int c = 0; c < k && !status; ++c) {
      const double l = hL[c + (size_t)c * k];
      if (!(l * l * hG[c + (size_t)c * k] < 1e12)) status = 1;
    }
    if (status) throw Error(ROM_ENOTSPD, "subspace loss: the outputs are linearly dependent");
    double tot = 0.0;
    for (int c = 0; c < s; ++c) tot += r2[c];
    *loss = tot / s;
    if (dY) {
      // d loss / d N = -(2/s) R C^T G^{-1}
      rom::launch_gemm(s, k, k, 1.0, L.C, k, true, L.Ginv, k, false, 0.0, nullptr, 0, L.Z, s, st);
      rom::launch_gemvn_multi(L.R, ld, N, s, L.Z, s, k, 0.0, nullptr, 0, -2.0 / s, L.dN, ld, st);
      rom::launch_convert_cols(N, k, L.dN, ld, dY, N, st);
    }
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_seednet_targets(const double* X, int64_t N, int64_t ldx, int count, float* out,
                               void* scratch, size_t scratch_bytes, void* stream) {
  try {
    if (!X || !out || !scratch) throw Error(ROM_EINVAL, "null argument");
    if (N < 1 || count < 1 || ldx < N) throw Error(ROM_EINVAL, "bad sizes");
    if (scratch_bytes < 512 * (size_t)count) throw Error(ROM_ECAPACITY, "scratch too small");
    rom::launch_seed_targets(N, count, X, ldx, (double*)scratch, out, (hipStream_t)stream);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_reduced_bytes(const rom_basis* V, size_t* bytes) {
  try {
    if (!V || !bytes) throw Error(ROM_EINVAL, "null argument");
    rom::Arena a(nullptr);
    a.take<double>(V->ld);
    a.take<double>(std::max<size_t>(rom::gram_partials(V->m, V->m, V->n, true), 1));
    *bytes = a.off + rom::ALIGN;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

namespace rom {
namespace {

// Scratch of rom_reduced_jacobian (the same carving for the size query and the call).
struct JacLayout {
  double *dmu, *part, *Ar, *Lc, *Lr, *lwork, *Br, *Cr, *T, *X, *Y, *U, *Z, *wk;
  int* status;
  int64_t ldr;
  size_t bytes;
};

JacLayout jac_layout(const rom_basis* V, int dim, void* base) {
  Arena a(base);
  JacLayout L;
  const int m = std::max(V->m, 1);
  const int64_t ld = V->ld;
  const int ns = std::max(V->n_src, 1), nd = std::max(V->n_det, 1);
  L.ldr = round_up(m, 2);
  L.dmu = a.take<double>(ld);
  L.part = a.take<double>(std::max<size_t>(
      {gram_partials(m, m, V->n, true), gram_partials(nd, ns, V->n, false), 1}));
  L.Ar = a.take<double>(L.ldr * m);
  L.Lc = a.take<double>(L.ldr * m);
  L.Lr = a.take<double>(L.ldr * m);
  L.lwork = a.take<double>(linv_rebuild_work(m));
  L.Br = a.take<double>(L.ldr * ns);
  L.Cr = a.take<double>(L.ldr * nd);
  L.T = a.take<double>(L.ldr * std::max(ns, nd));
  L.X = a.take<double>(L.ldr * ns);
  L.Y = a.take<double>(L.ldr * nd);
  L.U = a.take<double>(ld * ns);
  L.Z = a.take<double>(ld * nd);
  L.wk = a.take<double>(ld * (dim + 2));
  L.status = a.take<int>(4);
  L.bytes = a.off + ALIGN;
  return L;
}

}  // namespace
}  // namespace rom

rom_status rom_reduced_jacobian_bytes(const rom_basis* V, size_t* bytes) {
  try {
    if (!V || !bytes) throw Error(ROM_EINVAL, "null argument");
    *bytes = rom::jac_layout(V, V->op->grid.dim, nullptr).bytes;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_reduced_jacobian(const rom_basis* V, const rom_mu* p, double* J, void* scratch,
                                size_t scratch_bytes, void* stream) {
  try {
    if (!V || !J) throw Error(ROM_EINVAL, "null argument");
    const int dim = V->op->grid.dim;
    rom::check_mu(p, dim);
    const int m = V->m, ns = V->n_src, nd = V->n_det;
    if (m == 0) throw Error(ROM_EINVAL, "empty basis");
    const rom::JacLayout L = rom::jac_layout(V, dim, scratch);
    if (!scratch || scratch_bytes < L.bytes) throw Error(ROM_ECAPACITY, "scratch too small");
    if (ns == 0 || nd == 0 || p->nb == 0) return ROM_OK;
    hipStream_t st = (hipStream_t)stream;
    const rom::Bumps bm = rom::make_bumps(*p, dim);
    const int64_t ld = V->ld, ldr = L.ldr;
    // A_r = V^T A_* V + mu0 I + V^T diag(mu - mu0) V and its inverse Cholesky factor
    rom::launch_mu_eval(V->op->S, bm, V->op->diag_star, nullptr, L.dmu, st);
    rom::launch_gram(V->Q, ld, m, V->Q, ld, m, V->n, L.dmu, true, V->Gstar, V->ldg, p->mu0, L.Ar,
                     ldr, L.part, st);
    ROM_HIP(hipMemsetAsync(L.status, 0, sizeof(int), st));
    rom::launch_linv_rebuild(L.Ar, ldr, m, L.Lc, L.Lr, L.lwork, L.status, st);
    // B_r = V^T B~, C_r = V^T C~ (row gathers); X = A_r^{-1} B_r, Y = A_r^{-1} C_r
    rom::launch_gather_rows(V->Q, ld, m, V->idx_dev, V->scale_dev, ns, L.Br, ldr, st);
    rom::launch_gather_rows(V->Q, ld, m, V->idx_dev + ns, V->scale_dev + ns, nd, L.Cr, ldr, st);
    auto solve = [&](const double* R, int k, double* out) {
      rom::launch_gemm(m, k, m, 1.0, L.Lc, ldr, false, R, ldr, false, 0.0, nullptr, 0, L.T, ldr, st);
      rom::launch_gemm(m, k, m, 1.0, L.Lc, ldr, true, L.T, ldr, false, 0.0, nullptr, 0, out, ldr,
                       st);
    };
    solve(L.Br, ns, L.X);
    solve(L.Cr, nd, L.Y);
    // lifted states U = V X (N x n_src) and co-states Z = V Y (N x n_det), 16 per pass
    for (int c = 0; c < ns; c += 16)
      rom::launch_gemvn_multi(V->Q, ld, V->n, m, L.X + c * ldr, ldr, std::min(16, ns - c), 0.0,
                              nullptr, 0, 1.0, L.U + c * ld, ld, st);
    for (int c = 0; c < nd; c += 16)
      rom::launch_gemvn_multi(V->Q, ld, V->n, m, L.Y + c * ldr, ldr, std::min(16, nd - c), 0.0,
                              nullptr, 0, 1.0, L.Z + c * ld, ld, st);
    // J_k = -Z^T diag(d mu / d p_k) U = -C_r^T A_r^{-1} (V^T diag(d mu / d p_k) V) A_r^{-1} B_r,
    // over the rows of bump b's support only (the weights vanish elsewhere)
    const int npb = dim + 2;
    for (int b = 0; b < p->nb; ++b) {
      rom::launch_mu_grad(V->op->S, bm, b, L.wk, ld, st);
      for (int j = 0; j < npb; ++j) {
        const int64_t k = (int64_t)b * npb + j;
        rom::launch_gram(L.Z, ld, nd, L.U, ld, ns, V->n, L.wk + j * ld, false, nullptr, 0, 0.0,
                         J + k * nd * ns, nd, L.part, st);
      }
    }
    int status = 0;
    ROM_HIP(hipMemcpyAsync(&status, L.status, sizeof(int), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    if (status) throw Error(ROM_ENOTSPD, "reduced matrix A_r(p) not positive definite");
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

namespace rom {
namespace {

constexpr int MODES_MAX = 32;   // block columns (guard columns included)
constexpr int CHEB_DEGREE = 24; // filter degree per sweep

struct ModesLayout {
  double *diag, *dmu, *a1, *Y, *AY, *B1, *B2, *B3, *G, *Linv, *Ginv, *LT, *H, *Z, *lam, *res2,
      *bmax, *part, *gpart;
  int* status;
  size_t bytes;
};

ModesLayout modes_layout(const rom_operator* op, int kb, void* base) {
  Arena a(base);
  ModesLayout L;
  const int64_t n = op->n, ld = round_up(n, 64);
  L.diag = a.take<double>(ld);
  L.dmu = a.take<double>(ld);
  L.a1 = a.take<double>(ld);
  L.Y = a.take<double>(ld * kb);
  L.AY = a.take<double>(ld * kb);
  L.B1 = a.take<double>(ld * kb);
  L.B2 = a.take<double>(ld * kb);
  L.B3 = a.take<double>(ld * kb);
  L.G = a.take<double>(kb * kb);
  L.Linv = a.take<double>(kb * kb);
  L.Ginv = a.take<double>(kb * kb);
  L.LT = a.take<double>(kb * kb);
  L.H = a.take<double>(kb * kb);
  L.Z = a.take<double>(kb * kb);
  L.lam = a.take<double>(kb);
  L.res2 = a.take<double>(kb);
  L.bmax = a.take<double>(1);
  L.part = a.take<double>(std::max<size_t>(gram_partials(kb, kb, n, true), (size_t)256 * kb));
  L.gpart = a.take<double>(1024);
  L.status = a.take<int>(4);
  L.bytes = a.off + ALIGN;
  return L;
}

}  // namespace
}  // namespace rom

rom_status rom_lowest_modes_bytes(const rom_operator* op, int kx, size_t* bytes) {
  try {
    if (!op || !bytes) throw Error(ROM_EINVAL, "null argument");
    if (kx < 1 || kx > rom::MODES_MAX) throw Error(ROM_EINVAL, "block size out of range");
    *bytes = rom::modes_layout(op, kx, nullptr).bytes;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_lowest_modes(const rom_operator* op, const rom_mu* p, int k, const double* X0,
                            int kx, double tol, int maxit, double* U, double* lambda,
                            int* sweeps, void* scratch, size_t scratch_bytes, void* stream) {
  try {
    if (!op || !X0 || !U || !lambda) throw Error(ROM_EINVAL, "null argument");
    rom::check_mu(p, op->grid.dim);
    if (kx < 1 || kx > rom::MODES_MAX || k < 1 || k > kx)
      throw Error(ROM_EINVAL, "need 1 <= k <= kx <= 32");
    if (!(tol > 0.0) || maxit < 1) throw Error(ROM_EINVAL, "tol and maxit must be positive");
    const rom::ModesLayout L = rom::modes_layout(op, kx, scratch);
    if (!scratch || scratch_bytes < L.bytes) throw Error(ROM_ECAPACITY, "scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const rom::Stencil& S = op->S;
    const int64_t n = op->n, ld = rom::round_up(n, 64);
    const int kb = kx;
    // A(p) diagonal and the Gershgorin bound b of its spectrum
    rom::launch_mu_eval(S, rom::make_bumps(*p, op->grid.dim), op->diag_star, L.diag, L.dmu, st);
    rom::launch_fill(n, 1.0, L.B1, st);
    rom::launch_spmv(S, L.diag, L.B1, L.a1, st);
    rom::launch_gersh(n, L.diag, L.a1, L.gpart, L.bmax, st);
    double b = 0.0;
    ROM_HIP(hipMemcpyAsync(&b, L.bmax, sizeof(double), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipMemcpy2DAsync(L.Y, ld * sizeof(double), X0, n * sizeof(double), n * sizeof(double),
                             kx, hipMemcpyDeviceToDevice, st));
    ROM_HIP(hipStreamSynchronize(st));
    double* Y = L.Y;
    double* AY = L.AY;
    double* F[3] = {L.B1, L.B2, L.B3};   // free blocks
    // orthonormalise X (N x kb) into out: Cholesky QR twice
    auto cholqr2 = [&](double* X, double* out) {
      double* src = X;
      for (int pass = 0; pass < 2; ++pass) {
        rom::launch_gram(src, ld, kb, src, ld, kb, n, nullptr, true, nullptr, 0, 0.0, L.G, kb,
                         L.part, st);
        rom::launch_small_chol_inv(L.G, kb, L.Linv, L.Ginv, L.status, st);
        rom::launch_transpose_small(kb, L.Linv, L.LT, st);   // R^{-1} = L^{-T}
        double* dst = pass == 0 ? out : X;
        rom::launch_gemvn_multi(src, ld, n, kb, L.LT, kb, std::min(16, kb), 0.0, nullptr, 0, 1.0,
                                dst, ld, st);
        if (kb > 16)
          rom::launch_gemvn_multi(src, ld, n, kb, L.LT + 16 * kb, kb, kb - 16, 0.0, nullptr, 0, 1.0,
                                  dst + 16 * ld, ld, st);
        src = dst;
      }
      // the result is in X after the second pass; copy it to out
      ROM_HIP(hipMemcpyAsync(out, X, sizeof(double) * ld * kb, hipMemcpyDeviceToDevice, st));
    };
    auto mult = [&](const double* X, const double* C, double* out) {   // out = X C (kb x kb)
      rom::launch_gemvn_multi(X, ld, n, kb, C, kb, std::min(16, kb), 0.0, nullptr, 0, 1.0, out, ld,
                              st);
      if (kb > 16)
        rom::launch_gemvn_multi(X, ld, n, kb, C + 16 * kb, kb, kb - 16, 0.0, nullptr, 0, 1.0,
                                out + 16 * ld, ld, st);
    };
    ROM_HIP(hipMemsetAsync(L.status, 0, sizeof(int), st));
    cholqr2(Y, F[0]);   // Y orthonormal (F[0] holds a copy)
    std::vector<double> lam(kb), res2(kb);
    int sw = 0;
    bool converged = false;
    for (;; ++sw) {
      // Rayleigh-Ritz: H = Y^T A Y, H = Z diag(lam) Z^T, Y <- Y Z, AY <- AY Z
      rom::launch_spmm(S, L.diag, Y, ld, kb, AY, st);
      rom::launch_gram(Y, ld, kb, AY, ld, kb, n, nullptr, true, nullptr, 0, 0.0, L.H, kb, L.part,
                       st);
      rom::launch_sym_eig(L.H, kb, kb, L.lam, L.Z, st);
      mult(Y, L.Z, F[0]);
      mult(AY, L.Z, F[1]);
      std::swap(Y, F[0]);
      std::swap(AY, F[1]);
      rom::launch_ritz_resid(n, k, AY, Y, L.lam, ld, F[2], st);
      rom::launch_col_norms(n, k, F[2], ld, L.res2, L.part, st);
      int status = 0;
      ROM_HIP(hipMemcpyAsync(lam.data(), L.lam, sizeof(double) * kb, hipMemcpyDeviceToHost, st));
      ROM_HIP(hipMemcpyAsync(res2.data(), L.res2, sizeof(double) * k, hipMemcpyDeviceToHost, st));
      ROM_HIP(hipMemcpyAsync(&status, L.status, sizeof(int), hipMemcpyDeviceToHost, st));
      ROM_HIP(hipStreamSynchronize(st));
      if (status) throw Error(ROM_ENOTSPD, "lowest modes: the block lost rank (Cholesky QR failed)");
      double worst = 0.0;
      for (int i = 0; i < k; ++i) worst = std::max(worst, std::sqrt(std::max(res2[i], 0.0)));
      if (!(worst == worst)) throw Error(ROM_ENONFINITE, "lowest modes: non-finite residual");
      converged = worst <= tol * b;
      if (converged || sw + 1 >= maxit) break;
      // Chebyshev filter of degree CHEB_DEGREE damping [lam_max of the block, b]
      const double lo = lam[kb - 1], e = 0.5 * (b - lo), c = 0.5 * (b + lo);
      if (!(e > 0.0)) break;
      double* prev = Y;        // T_0 block
      double* cur = F[2];      // T_1 block = (A - c) Y / e
      rom::launch_cheb_step(S, L.diag, Y, ld, kb, 1.0 / e, -c / e, 0.0, nullptr, cur, st);
      for (int j = 2; j <= rom::CHEB_DEGREE; ++j) {
        // next = 2 (A - c) cur / e - prev, written over prev, fused with the product
        rom::launch_cheb_step(S, L.diag, cur, ld, kb, 2.0 / e, -2.0 * c / e, -1.0, prev, prev,
                              st);
        std::swap(prev, cur);
      }
      // the filtered block is cur; orthonormalise it into Y's buffer
      if (cur != Y) {
        cholqr2(cur, Y);
      } else {
        cholqr2(cur, F[0]);
      }
    }
    ROM_HIP(hipMemcpy2DAsync(U, n * sizeof(double), Y, ld * sizeof(double), n * sizeof(double), k,
                             hipMemcpyDeviceToDevice, st));
    ROM_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < k; ++i) lambda[i] = lam[i];
    if (sweeps) *sweeps = sw + 1;
    if (!converged) {
      rom::report_message("lowest modes: the residual test did not pass (maxit, or a filter "
                          "interval that vanished)");
      return ROM_ENOCONV;
    }
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

namespace rom {
namespace {

constexpr int MS_CHUNK = 8;   // iterations between host checks of the multi-shift solver

struct ShiftLayout {
  double *diag, *dmu, *r, *p, *w, *Pr, *Pi, *part, *res;
  MsState* state;
  size_t bytes;
};

ShiftLayout shift_layout(const rom_operator* op, int nb, int ns, void* base) {
  Arena a(base);
  ShiftLayout L;
  const int64_t n = op->n, ld = round_up(n, 64);
  const StencilShape sh = stencil_shape(op->S, 512);
  L.diag = a.take<double>(ld);
  L.dmu = a.take<double>(ld);
  L.r = a.take<double>(ld * nb);
  L.p = a.take<double>(ld * nb);
  L.w = a.take<double>(ld * nb);
  L.Pr = a.take<double>(ld * nb * ns);
  L.Pi = a.take<double>(ld * nb * ns);
  L.part = a.take<double>(std::max<size_t>({(size_t)nb * sh.blocks, (size_t)nb * ms_vec_blocks(n),
                                            (size_t)2 * nb * ns * sh.blocks}));
  L.res = a.take<double>(2 * (size_t)nb * ns);
  L.state = a.take<MsState>(nb);
  L.bytes = a.off + ALIGN;
  return L;
}

struct ResponseLayout {
  double *dmu, *part, *Ar, *Lc, *Lr, *Ainv, *N, *Nc, *Nr, *lwork, *Br, *Cr, *T, *Yr, *Yi;
  int* status;
  int64_t ldr;
  size_t bytes;
};

ResponseLayout response_layout(const rom_basis* V, void* base) {
  Arena a(base);
  ResponseLayout L;
  const int m = std::max(V->m, 1);
  const int ns = std::max(V->n_src, 1), nd = std::max(V->n_det, 1);
  L.ldr = round_up(m, 2);
  const size_t mm = (size_t)L.ldr * m;
  L.dmu = a.take<double>(V->ld);
  L.part = a.take<double>(std::max<size_t>(gram_partials(m, m, V->n, true), 1));
  L.Ar = a.take<double>(mm);
  L.Lc = a.take<double>(mm);
  L.Lr = a.take<double>(mm);
  L.Ainv = a.take<double>(mm);
  L.N = a.take<double>(mm);
  L.Nc = a.take<double>(mm);
  L.Nr = a.take<double>(mm);
  L.lwork = a.take<double>(linv_rebuild_work(m));
  L.Br = a.take<double>(L.ldr * ns);
  L.Cr = a.take<double>(L.ldr * nd);
  L.T = a.take<double>(L.ldr * ns);
  L.Yr = a.take<double>(L.ldr * ns);
  L.Yi = a.take<double>(L.ldr * ns);
  L.status = a.take<int>(4);
  L.bytes = a.off + ALIGN;
  return L;
}

}  // namespace
}  // namespace rom

rom_status rom_shifted_solve_bytes(const rom_operator* op, int nb, int ns, size_t* bytes) {
  try {
    if (!op || !bytes) throw Error(ROM_EINVAL, "null argument");
    if (nb < 1 || ns < 1 || ns > rom::MS_MAX) throw Error(ROM_EINVAL, "need nb >= 1, 1 <= ns <= 8");
    *bytes = rom::shift_layout(op, nb, ns, nullptr).bytes;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_shifted_solve(const rom_operator* op, const rom_mu* p, const double* B, int nb,
                             const double* sigma, int ns, double tol, int maxit, double* Xr,
                             double* Xi, int* its, double* resid, void* scratch,
                             size_t scratch_bytes, void* stream) {
  try {
    if (!op || !B || !sigma || !Xr || !Xi) throw Error(ROM_EINVAL, "null argument");
    rom::check_mu(p, op->grid.dim);
    if (nb < 1 || ns < 1 || ns > rom::MS_MAX) throw Error(ROM_EINVAL, "need nb >= 1, 1 <= ns <= 8");
    if (!(tol > 0.0) || maxit < 1) throw Error(ROM_EINVAL, "tol and maxit must be positive");
    rom::MsShifts sh{};
    sh.ns = ns;
    for (int s = 0; s < ns; ++s) {
      if (!std::isfinite(sigma[s])) throw Error(ROM_EINVAL, "non-finite shift");
      sh.sigma[s] = sigma[s];
    }
    const rom::ShiftLayout L = rom::shift_layout(op, nb, ns, scratch);
    if (!scratch || scratch_bytes < L.bytes) throw Error(ROM_ECAPACITY, "scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const rom::Stencil& S = op->S;
    const int64_t n = op->n, ld = rom::round_up(n, 64);
    const rom::StencilShape shp = rom::stencil_shape(S, 512);
    const int Pv = rom::ms_vec_blocks(n);
    rom::launch_mu_eval(S, rom::make_bumps(*p, op->grid.dim), op->diag_star, L.diag, L.dmu, st);
    rom::launch_ms_init(n, B, n, nb, ns, L.r, L.p, ld, L.Pr, L.Pi, Xr, Xi, n, L.part, st);
    rom::launch_ms_start(L.part, Pv, L.state, nb, ns, tol, maxit, st);
    std::vector<rom::MsState> hs(nb);
    for (int it = 0;; it += rom::MS_CHUNK) {
      for (int c = 0; c < rom::MS_CHUNK; ++c) {
        const int Pa = rom::launch_ms_apply(S, shp, L.diag, L.p, ld, L.w, nb, L.state, L.part, st);
        rom::launch_ms_alpha(L.part, Pa, L.state, nb, sh, st);
        rom::launch_ms_update(n, nb, ns, L.w, L.r, ld, L.Pr, L.Pi, Xr, Xi, n, L.state, L.part, st);
        rom::launch_ms_beta(L.part, Pv, L.state, nb, ns, st);
        rom::launch_ms_dir(n, nb, L.r, L.p, ld, L.state, st);
      }
      ROM_HIP(hipMemcpyAsync(hs.data(), L.state, sizeof(rom::MsState) * nb, hipMemcpyDeviceToHost,
                             st));
      ROM_HIP(hipStreamSynchronize(st));
      bool all = true;
      for (int j = 0; j < nb; ++j) all = all && hs[j].done;
      // every column stops by maxit (its own counter); the bound below is a safety net
      if (all || it > maxit + 2 * rom::MS_CHUNK) break;
    }
    // true residuals ||b_j - (A + i sigma_s) X||, FP64
    rom::launch_ms_resid(S, shp, L.diag, Xr, Xi, n, B, n, nb, sh, L.part, L.res, st);
    std::vector<double> r2(2 * (size_t)nb * ns);
    ROM_HIP(hipMemcpyAsync(r2.data(), L.res, sizeof(double) * r2.size(), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    int flag = 0;
    bool noconv = false;
    for (int j = 0; j < nb; ++j) {
      if (its) its[j] = hs[j].its;
      flag = std::max(flag, hs[j].flag);
      for (int s = 0; s < ns; ++s) noconv = noconv || !hs[j].sdone[s];
    }
    if (resid) {
      const size_t cols = (size_t)nb * ns;
      for (int s = 0; s < ns; ++s)
        for (int j = 0; j < nb; ++j) {
          const size_t c = (size_t)s * nb + j;
          const double bb = hs[j].bb;
          resid[c] = bb > 0.0 ? std::sqrt((r2[c] + r2[cols + c]) / bb) : 0.0;
        }
    }
    if (flag == 1) throw Error(ROM_ENOTSPD, "shifted solve: non-positive curvature in the seed CG");
    if (flag == 2) throw Error(ROM_ENONFINITE, "shifted solve: non-finite value");
    if (noconv) {
      rom::report_message("shifted solve: some shift reached maxit");
      return ROM_ENOCONV;
    }
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_reduced_response_bytes(const rom_basis* V, size_t* bytes) {
  try {
    if (!V || !bytes) throw Error(ROM_EINVAL, "null argument");
    *bytes = rom::response_layout(V, nullptr).bytes;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_reduced_response(const rom_basis* V, const rom_mu* p, const double* sigma, int ns,
                                double* Psi_re, double* Psi_im, void* scratch,
                                size_t scratch_bytes, void* stream) {
  try {
    if (!V || !sigma || !Psi_re || !Psi_im) throw Error(ROM_EINVAL, "null argument");
    rom::check_mu(p, V->op->grid.dim);
    if (ns < 0) throw Error(ROM_EINVAL, "negative shift count");
    const int m = V->m, nsrc = V->n_src, nd = V->n_det;
    if (m == 0) throw Error(ROM_EINVAL, "empty basis");
    const rom::ResponseLayout L = rom::response_layout(V, scratch);
    if (!scratch || scratch_bytes < L.bytes) throw Error(ROM_ECAPACITY, "scratch too small");
    for (int s = 0; s < ns; ++s)
      if (!std::isfinite(sigma[s])) throw Error(ROM_EINVAL, "non-finite shift");
    if (ns == 0 || nsrc == 0 || nd == 0) return ROM_OK;
    hipStream_t st = (hipStream_t)stream;
    const int64_t ld = V->ld, ldr = L.ldr;
    // A_r = V^T A_* V + mu0 I + V^T diag(mu - mu0) V, its inverse Cholesky factor Lc and
    // A_r^{-1} = Lc^T Lc; B_r, C_r by row gathers (E_r = I: V has orthonormal columns)
    rom::launch_mu_eval(V->op->S, rom::make_bumps(*p, V->op->grid.dim), V->op->diag_star, nullptr,
                        L.dmu, st);
    rom::launch_gram(V->Q, ld, m, V->Q, ld, m, V->n, L.dmu, true, V->Gstar, V->ldg, p->mu0, L.Ar,
                     ldr, L.part, st);
    ROM_HIP(hipMemsetAsync(L.status, 0, sizeof(int), st));
    rom::launch_linv_rebuild(L.Ar, ldr, m, L.Lc, L.Lr, L.lwork, L.status, st);
    rom::launch_gemm(m, m, m, 1.0, L.Lc, ldr, true, L.Lc, ldr, false, 0.0, nullptr, 0, L.Ainv, ldr,
                     st);
    rom::launch_gather_rows(V->Q, ld, m, V->idx_dev, V->scale_dev, nsrc, L.Br, ldr, st);
    rom::launch_gather_rows(V->Q, ld, m, V->idx_dev + nsrc, V->scale_dev + nsrc, nd, L.Cr, ldr, st);
    for (int s = 0; s < ns; ++s) {
      const double sg = sigma[s];
      double* Pr = Psi_re + (size_t)s * nd * nsrc;
      double* Pi = Psi_im + (size_t)s * nd * nsrc;
      // (A_r + i sg I)(y_r + i y_i) = B_r  <=>  (A_r + sg^2 A_r^{-1}) y_r = B_r,
      // y_i = -sg A_r^{-1} y_r; A_r + sg^2 A_r^{-1} is SPD (it commutes with A_r)
      const double* Lc = L.Lc;
      if (sg != 0.0) {
        rom::launch_axpby_cols(m, m, 1.0, L.Ar, ldr, sg * sg, L.Ainv, ldr, L.N, ldr, st);
        rom::launch_linv_rebuild(L.N, ldr, m, L.Nc, L.Nr, L.lwork, L.status, st);
        Lc = L.Nc;
      }
      rom::launch_gemm(m, nsrc, m, 1.0, Lc, ldr, false, L.Br, ldr, false, 0.0, nullptr, 0, L.T, ldr,
                       st);
      rom::launch_gemm(m, nsrc, m, 1.0, Lc, ldr, true, L.T, ldr, false, 0.0, nullptr, 0, L.Yr, ldr,
                       st);
      rom::launch_gemm(nd, nsrc, m, 1.0, L.Cr, ldr, true, L.Yr, ldr, false, 0.0, nullptr, 0, Pr, nd,
                       st);
      if (sg != 0.0) {
        rom::launch_gemm(m, nsrc, m, -sg, L.Ainv, ldr, false, L.Yr, ldr, false, 0.0, nullptr, 0,
                         L.Yi, ldr, st);
        rom::launch_gemm(nd, nsrc, m, 1.0, L.Cr, ldr, true, L.Yi, ldr, false, 0.0, nullptr, 0, Pi,
                         nd, st);
      } else {
        ROM_HIP(hipMemsetAsync(Pi, 0, sizeof(double) * nd * nsrc, st));
      }
    }
    int status = 0;
    ROM_HIP(hipMemcpyAsync(&status, L.status, sizeof(int), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    if (status) throw Error(ROM_ENOTSPD, "reduced matrix not positive definite");
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_reduced_transfer(const rom_basis* V, const rom_mu* p, double* Ar, double* Br,
                                double* Cr, double* Er, void* scratch, size_t scratch_bytes,
                                void* stream) {
  try {
    if (!V) throw Error(ROM_EINVAL, "null basis");
    rom::check_mu(p, V->op->grid.dim);
    size_t need = 0;
    rom_reduced_bytes(V, &need);
    if (!scratch || scratch_bytes < need) throw Error(ROM_ECAPACITY, "scratch too small");
    hipStream_t st = (hipStream_t)stream;
    rom::Arena a(scratch);
    double* dmu = a.take<double>(V->ld);
    double* part = a.take<double>(std::max<size_t>(rom::gram_partials(V->m, V->m, V->n, true), 1));
    const int m = V->m;
    if (m == 0) return ROM_OK;
    if (Ar) {
      // A_r = V^T A_* V + mu0 V^T V + V^T diag(mu - mu0) V with V^T V = I (orthonormal V)
      rom::launch_mu_eval(V->op->S, rom::make_bumps(*p, V->op->grid.dim), V->op->diag_star,
                          nullptr, dmu, st);
      rom::launch_gram(V->Q, V->ld, m, V->Q, V->ld, m, V->n, dmu, true, V->Gstar, V->ldg, p->mu0,
                       Ar, m, part, st);
    }
    if (Er)
      rom::launch_gram(V->Q, V->ld, m, V->Q, V->ld, m, V->n, nullptr, true, nullptr, 0, 0.0, Er,
                       m, part, st);
    if (Br && V->n_src > 0)
      rom::launch_gather_rows(V->Q, V->ld, m, V->idx_dev, V->scale_dev, V->n_src, Br, m, st);
    if (Cr && V->n_det > 0)
      rom::launch_gather_rows(V->Q, V->ld, m, V->idx_dev + V->n_src, V->scale_dev + V->n_src,
                              V->n_det, Cr, m, st);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

rom_status rom_basis_dims(const rom_basis* V, int64_t* N, int* m) {
  if (!V) {
    rom::g_err = "null basis";
    return ROM_EINVAL;
  }
  if (N) *N = V->n;
  if (m) *m = V->m;
  return ROM_OK;
}

rom_status rom_basis_copy(const rom_basis* V, double* dst, void* stream) {
  try {
    if (!V || !dst) throw Error(ROM_EINVAL, "null argument");
    if (V->m == 0) return ROM_OK;
    ROM_HIP(hipMemcpy2DAsync(dst, V->n * sizeof(double), V->Q, V->ld * sizeof(double),
                             V->n * sizeof(double), V->m, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
    return ROM_OK;
  } catch (const Error& e) {
    return rom::fail(e);
  }
}

void rom_basis_destroy(rom_basis* V) { delete V; }

}  // extern "C"
