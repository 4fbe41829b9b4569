// C ABI of the stfdfd library: contexts, problems, factorisation and the FGMRES
// solve preconditioned by one source-transfer round (Sec. 2.3, Algorithm 1;
// Sec. 2.4, Eqs. (22)-(23)).  Host code only orchestrates: every arithmetic
// step on problem data runs in the kernels of kernels_*.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <numeric>

#include "cplx.h"
#include "stf_internal.h"

using namespace stf;

thread_local KernelTimer* stf::t_kernel_timer = nullptr;

namespace {

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) b = 16;
    HIP_CHECK(hipMalloc(&p, b));
    bytes = b;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

template <typename T>
void upload(DBuf& d, const std::vector<T>& h, hipStream_t st) {
  d.alloc(std::max<size_t>(h.size() * sizeof(T), 16));
  if (!h.empty()) HIP_CHECK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

struct Level {
  int off = 0, n = 0, max_m = 0, max_pm = 0, max_p = 0;
};

}  // namespace

// Workspace of the allocation-free round (stf_precond_apply_noalloc): the front
// vectors and the local fields of one right-hand side.  Each device holds its
// own copy until the process ends; host code uses only the per-device address
// that hipGetSymbolAddress returns (g_scratch), never the symbol itself.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

// Address of this device's scratch array (the device must be current).
void* scratch_address(int device) {
  STF_REQUIRE(device >= 0 && device < MAX_DEVICES, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    STF_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}
}  // namespace

struct BatchState;
void destroy_batch(BatchState* b);

// Level signature for the autotuner: operation (0 factorisation, 1 forward
// sweep, 2 backward sweep), bytes per complex entry, right-hand sides per
// sweep (0 for the factorisation), fronts in the level, largest m and p.  The
// shapes that run a level and their speed depend on nothing else.
struct TuneKey {
  int op, elem, nr, nlevel, max_m, max_p;
  bool operator<(const TuneKey& o) const {
    return std::tie(op, elem, nr, nlevel, max_m, max_p) <
           std::tie(o.op, o.elem, o.nr, o.nlevel, o.max_m, o.max_p);
  }
};
// The fastest shape measured for a signature (factorisation: kind, nb, ntf;
// sweeps: kind, kp, ntl, parts), its time and that of the built-in shape.
struct TuneEntry {
  int kind = 0, a = 0, b = 0, c = 0;
  double ms = 0.0, ms_default = 0.0;
};

struct stf_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  std::map<std::tuple<int, int, int>, std::shared_ptr<const SymShape>> shapes;
  // Timing: pending event pairs per kernel class, folded totals.
  bool timing = false;
  uint32_t timing_mask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[STF_K_COUNT];
  std::vector<hipEvent_t> pool;
  double total_ms[STF_K_COUNT] = {};
  int64_t launches[STF_K_COUNT] = {};
  double* pinned = nullptr;     // pinned host staging: 64 doubles per right-hand side
  double* pinned_dev = nullptr; // the same memory as the device addresses it
  hipEvent_t iter_ev[2] = {nullptr, nullptr};   // per-iteration estimate copies
  hipEvent_t cycle_ev = nullptr;                // true residuals of a restart copied
  stf_nn nn = nullptr;          // network for STF_X0_LEARNED (not owned)
  void* scratch = nullptr;      // this device's scratch array (allocation-free round)
  BatchState* batch = nullptr;  // state of the last stf_batch_solve (owned)
  std::map<TuneKey, TuneEntry> tune;   // autotuned launch shapes (this device)
  std::string arch;             // the device's architecture name (tune files)
  // Second stream (default priority) for work that overlaps the main stream's
  // (the network's guesses during a factorisation), and the two events that
  // order it against the main stream.
  hipStream_t side = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    return e;
  }
  void fold() {
    HIP_CHECK(hipStreamSynchronize(stream));
    if (side) HIP_CHECK(hipStreamSynchronize(side));   // kernels timed on the second stream
    for (int c = 0; c < STF_K_COUNT; ++c) {
      for (auto& pr : pending[c]) {
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, pr.first, pr.second));
        total_ms[c] += ms;
        launches[c] += 1;
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[c].clear();
    }
  }
  size_t npending() const {
    size_t s = 0;
    for (int c = 0; c < STF_K_COUNT; ++c) s += pending[c].size();
    return s;
  }
};

namespace {

// Message of the last failure that happened without a context (stf_ctx_create).
thread_local std::string g_noctx_error;

// While in scope (and timing is on for its class), every kernel launched on
// this thread is timed on its own: the start and stop events are recorded by
// its dispatch, and the pair is added to the class.  Nested scopes time their
// kernels in the innermost class.  Kernels captured into a graph are not timed.
struct Timed final : KernelTimer {
  stf_ctx c;
  int cls;
  KernelTimer* prev = nullptr;
  bool on = false;
  Timed(stf_ctx c_, int cls_) : c(c_), cls(cls_) {
    if (c && c->timing && (c->timing_mask >> cls & 1u)) {
      on = true;
      prev = t_kernel_timer;
      t_kernel_timer = this;
    }
  }
  Timed(const Timed&) = delete;
  Timed& operator=(const Timed&) = delete;
  bool events(hipStream_t st, hipEvent_t* start, hipEvent_t* stop) override {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    if (c->npending() > 16384) c->fold();
    *start = c->get_event();
    *stop = c->get_event();
    c->pending[cls].push_back({*start, *stop});
    return true;
  }
  ~Timed() {
    if (on) t_kernel_timer = prev;
  }
};

}  // namespace

// Fronts, subdomains and round workspaces of one or more problems in one set of
// device arrays.  Problem p's nodes are the segment [gbase[p], gbase[p] + nx*ny)
// of concatenated global vectors; the fronts of all problems are ordered by tree
// level (largest first within a level), so one launch per level serves them all.
// Stages of a sweeping order over a set: stage t holds, for every problem,
// that problem's stage t (problems with fewer stages contribute nothing).
// Subtree sweeps of a set over subtrees of the deep levels (see FuseArgs).
struct FusePlan {
  FuseArgs args;                // device pointers into lev / fl
  DBuf lev, fl;
};

struct SweepPlan {
  int nstage = 0;
  std::vector<int> s_first, s_count;          // per stage: its members in slist
  std::vector<std::vector<Level>> lv;         // per stage and depth: range in flist
  DBuf slist, flist, inst;                    // members, front instances, membership flags
  DBuf fdev;                                  // the descriptors of flist's fronts, in its order
  std::vector<int> h_flist;                   // host copy of flist
  // subtree sweeps per choice (16 D + T): per stage, the tables over the
  // stage's fronts at depth D (null where the stage has none)
  std::map<int, std::vector<std::unique_ptr<FusePlan>>> fuse;
};

struct Mf {
  int prec = STF_C128;
  int nprob = 0, nsub = 0, max_depth = -1, max_nx = 0, max_ny = 0;
  int max_oxl = 0, max_oyl = 0, max_ixl = 0, max_iyl = 0;   // largest Omega_k and I_k boxes
  std::vector<int> sub_prob, sub_kx, sub_ky, prob_px, prob_py;   // host copies for the stages
  std::vector<int> front_sub, front_depth;                        // per front instance
  std::map<int, std::unique_ptr<SweepPlan>> sweeps;              // by order
  int64_t n_fronts = 0, fac_elems = 0, lpk_elems = 0, upk_elems = 0, vec_elems = 0,
          piv_elems = 0, u_elems = 0;
  std::vector<Level> levels;     // by depth
  std::vector<FrontDev> h_fronts;  // host copies of the front instances and children
  std::vector<int> h_children;
  std::map<int, std::unique_ptr<FusePlan>> fuse;   // subtree sweeps by choice (fuse_code)
  DBuf lcoef, subs, fronts, vars, cmap, ents, children, cover_x, cover_y, scat;
  DBuf fac, lpk, upk, piv, vec, u;
  int ws_nr = 0;                 // right-hand sides the vec / u workspaces hold

  LevelArgs level_args(int d, const double2* keps, const int* pact = nullptr) const {
    LevelArgs a{};
    a.fronts = fronts.as<FrontDev>();
    a.first = levels[d].off;
    a.nlevel = levels[d].n;
    a.subs = subs.as<SubDev>();
    a.vars = vars.as<int>();
    a.cmap = cmap.as<int>();
    a.ents = ents.as<SymEntry>();
    a.children = children.as<int>();
    a.keps = keps;
    a.lcoef = lcoef.as<double2>();
    a.pact = pact;
    a.max_m = levels[d].max_m;
    a.max_pm = levels[d].max_pm;
    a.max_p = levels[d].max_p;
    return a;
  }
  int64_t device_bytes() const {
    const DBuf* all[] = {&lcoef, &subs, &fronts, &vars, &cmap, &ents, &children, &cover_x,
                         &cover_y, &scat, &fac, &lpk, &upk, &piv, &vec, &u};
    int64_t t = 0;
    for (const DBuf* d : all) t += (int64_t)d->bytes;
    for (const auto& kv : fuse) t += (int64_t)(kv.second->lev.bytes + kv.second->fl.bytes);
    return t;
  }
  // Shallowest root depth D of subtree sweeps: every level from D down is one
  // the wavefront kernels take, and a subtree spans two levels or more; -1 if
  // there is none.
  int fuse_min_depth() const {
    int d = max_depth;
    if (d < 1 || levels[d].max_m > 128 || levels[d].max_p > 64) return -1;
    while (d - 1 >= 0 && levels[d - 1].max_m <= 128 && levels[d - 1].max_p <= 64) --d;
    return d <= max_depth - 1 ? d : -1;
  }
  // Subtree sweep tables for the given roots (fronts at depth D), T subtrees
  // (consecutive roots) per workgroup.
  std::unique_ptr<FusePlan> build_fuse(const std::vector<int>& roots, int D, int T, hipStream_t st) const {
    STF_REQUIRE(D >= 0 && D < max_depth && T >= 1, "internal: subtree choice out of range");
    std::unique_ptr<FusePlan> fp(new FusePlan());
    FuseArgs& z = fp->args;
    z.K = max_depth - D + 1;
    const int nr = (int)roots.size();
    z.ntrees = (nr + T - 1) / T;
    for (int d = D; d <= max_depth; ++d) {
      z.max_m = std::max(z.max_m, levels[d].max_m);
      z.max_p = std::max(z.max_p, levels[d].max_p);
    }
    std::vector<int> lev;
    std::vector<int4> fl;
    std::vector<int> slot(h_fronts.size(), -1);
    std::vector<std::vector<int>> byl(z.K);
    for (int t = 0; t < z.ntrees; ++t) {
      for (auto& v : byl) v.clear();
      for (int i = t * T; i < std::min(nr, (t + 1) * T); ++i) byl[0].push_back(roots[i]);
      for (int j = 1; j < z.K; ++j)
        for (int f : byl[j - 1])
          for (int c = 0; c < h_fronts[f].nchild; ++c) byl[j].push_back(h_children[h_fronts[f].child_off + c]);
      int q = 0;
      for (int j = z.K - 1; j >= 1; --j)
        for (int f : byl[j]) {
          slot[f] = q;
          q += h_fronts[f].q;
        }
      z.slot_q = std::max(z.slot_q, q);
      for (int j = 0; j < z.K; ++j) {
        lev.push_back((int)fl.size());
        for (int f : byl[j]) {
          const FrontDev& d = h_fronts[f];
          const int c0 = d.nchild > 0 ? h_children[d.child_off] : -1;
          const int c1 = d.nchild > 1 ? h_children[d.child_off + 1] : -1;
          fl.push_back(make_int4(f, j == 0 ? -1 : slot[f], c0 >= 0 ? slot[c0] : -1, c1 >= 0 ? slot[c1] : -1));
        }
      }
      lev.push_back((int)fl.size());
    }
    STF_REQUIRE(fl.size() < (1ULL << 31), "internal: subtree tables too large");
    upload(fp->lev, lev, st);
    upload(fp->fl, fl, st);
    z.lev = fp->lev.as<int>();
    z.fl = fp->fl.as<int4>();
    HIP_CHECK(hipStreamSynchronize(st));
    return fp;
  }
  // The subtree sweep tables for `code` = 16 D + T over every front at depth
  // D (built once, kept).
  const FusePlan& fuse_plan(int code, hipStream_t st) {
    auto it = fuse.find(code);
    if (it != fuse.end()) return *it->second;
    const int D = code / 16, T = code % 16;
    STF_REQUIRE(D >= 0 && D < max_depth, "internal: subtree root depth out of range");
    std::vector<int> roots(levels[D].n);
    std::iota(roots.begin(), roots.end(), levels[D].off);
    std::unique_ptr<FusePlan> fp = build_fuse(roots, D, T, st);
    FusePlan& ref = *fp;
    fuse[code] = std::move(fp);
    return ref;
  }
};

// Builds the set of problems `plans` (all with the front precision `prec`),
// problem p at node offset gbase[p] of the global vectors; allocates the
// factors and the workspaces of one right-hand side.
void build_mf(Mf& mf, const std::vector<const Plan*>& plans, const std::vector<long long>& gbase,
              int prec, hipStream_t st, const std::vector<int>& gc_off = {}) {
  mf.prec = prec;
  mf.nprob = (int)plans.size();
  // Subdomains of every problem (problem after problem) and their local coefficients.
  std::vector<double2> lc;
  std::vector<SubDev> sd;
  std::vector<ScatDev> sc;
  std::vector<int4> cvx, cvy;
  std::vector<int> sub0(mf.nprob);
  long long uoff = 0;
  for (int pi = 0; pi < mf.nprob; ++pi) {
    const Plan& pl = *plans[pi];
    sub0[pi] = (int)sd.size();
    ScatDev g{};
    g.sub0 = (int)sd.size();
    g.px = pl.prm.px;
    g.nx = pl.prm.nx;
    g.ny = pl.prm.ny;
    g.cx_off = (int)cvx.size();
    g.cy_off = (int)cvy.size();
    g.gbase = gbase[pi];
    g.gc_off = gc_off.empty() ? 0 : gc_off[pi];
    sc.push_back(g);
    mf.prob_px.push_back(pl.prm.px);
    mf.prob_py.push_back(pl.prm.py);
    cvx.insert(cvx.end(), pl.cover_x.begin(), pl.cover_x.end());
    cvy.insert(cvy.end(), pl.cover_y.begin(), pl.cover_y.end());
    mf.max_nx = std::max(mf.max_nx, pl.prm.nx);
    mf.max_ny = std::max(mf.max_ny, pl.prm.ny);
    for (const SubDesc& s : pl.subs) {
      SubDev d{};
      d.ox0 = s.ox0; d.oy0 = s.oy0; d.nxl = s.nxl; d.nyl = s.nyl;
      d.ix0 = s.ix0; d.ix1 = s.ix1; d.iy0 = s.iy0; d.iy1 = s.iy1;
      d.gbase = gbase[pi];
      d.gnx = pl.prm.nx;
      d.prob = pi;
      d.cx_off = (int)lc.size();
      for (int t = 0; t < s.nxl; ++t) {
        lc.push_back(make_double2(s.cx.w[t].real(), s.cx.w[t].imag()));
        lc.push_back(make_double2(s.cx.e[t].real(), s.cx.e[t].imag()));
      }
      d.cy_off = (int)lc.size();
      for (int t = 0; t < s.nyl; ++t) {
        lc.push_back(make_double2(s.cy.w[t].real(), s.cy.w[t].imag()));
        lc.push_back(make_double2(s.cy.e[t].real(), s.cy.e[t].imag()));
      }
      d.u_off = uoff;
      uoff += (long long)s.nxl * s.nyl;
      sd.push_back(d);
      mf.sub_prob.push_back(pi);
      mf.sub_kx.push_back(s.kx);
      mf.sub_ky.push_back(s.ky);
      mf.max_oxl = std::max(mf.max_oxl, s.nxl);
      mf.max_oyl = std::max(mf.max_oyl, s.nyl);
      mf.max_ixl = std::max(mf.max_ixl, s.ix1 - s.ix0);
      mf.max_iyl = std::max(mf.max_iyl, s.iy1 - s.iy0);
    }
  }
  mf.nsub = (int)sd.size();
  mf.u_elems = uoff;
  STF_REQUIRE(lc.size() < (1ULL << 31), "problem set too large for int32 coefficient offsets");
  upload(mf.lcoef, lc, st);
  upload(mf.subs, sd, st);
  upload(mf.cover_x, cvx, st);
  upload(mf.cover_y, cvy, st);
  upload(mf.scat, sc, st);

  // Concatenated symbolic arrays of the distinct shapes (shared between problems).
  std::map<const SymShape*, int> shape_id;
  std::vector<const SymShape*> shapes;
  for (const Plan* pl : plans)
    for (const auto& sh : pl->shapes)
      if (shape_id.emplace(sh.get(), (int)shapes.size()).second) shapes.push_back(sh.get());
  std::vector<int> vars, cmap, sh_var(shapes.size()), sh_cmap(shapes.size()), sh_ent(shapes.size());
  std::vector<SymEntry> ents;
  for (size_t k = 0; k < shapes.size(); ++k) {
    const SymShape& sh = *shapes[k];
    sh_var[k] = (int)vars.size();
    sh_cmap[k] = (int)cmap.size();
    sh_ent[k] = (int)ents.size();
    vars.insert(vars.end(), sh.vars.begin(), sh.vars.end());
    cmap.insert(cmap.end(), sh.cmap.begin(), sh.cmap.end());
    ents.insert(ents.end(), sh.ents.begin(), sh.ents.end());
  }
  STF_REQUIRE(vars.size() < (1ULL << 31) && ents.size() < (1ULL << 31), "symbolic plans too large");
  upload(mf.vars, vars, st);
  upload(mf.cmap, cmap, st);
  upload(mf.ents, ents, st);

  // Front instances of every subdomain of every problem, in level order
  // (largest first within a level) so that each level is a contiguous range.
  struct Rec { int prob, sub, idx, depth, m; const SymShape* sh; };
  std::vector<Rec> recs;
  std::vector<int> sub_base(mf.nsub);
  for (int pi = 0; pi < mf.nprob; ++pi) {
    const Plan& pl = *plans[pi];
    for (size_t k = 0; k < pl.subs.size(); ++k) {
      const int gk = sub0[pi] + (int)k;
      const SymShape* sh = pl.shapes[pl.subs[k].shape].get();
      sub_base[gk] = (int)recs.size();
      for (size_t i = 0; i < sh->fronts.size(); ++i)
        recs.push_back({pi, gk, (int)i, sh->fronts[i].depth, sh->fronts[i].p + sh->fronts[i].q, sh});
    }
  }
  std::vector<int> order(recs.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (recs[x].depth != recs[y].depth) return recs[x].depth < recs[y].depth;
    return recs[x].m > recs[y].m;
  });
  std::vector<int> inst(recs.size());      // record -> instance index
  for (size_t t = 0; t < order.size(); ++t) inst[order[t]] = (int)t;
  std::vector<FrontDev> fr(recs.size());
  std::vector<int> kids;
  // Working blocks: a front's block is read after its own level only by its
  // parent's assembly, one level up, so the levels share two arenas, the even
  // depths one and the odd depths the other, each sized for its largest level
  // (offsets within a level here, the odd arena's base added below).
  long long fac_off = 0, lpk_off = 0, upk_off = 0;
  long long vec_off = 0, piv_off = 0;
  std::vector<long long> lvl_fac;          // working-block entries per depth
  for (size_t t = 0; t < order.size(); ++t) {
    const Rec& rc = recs[order[t]];
    if ((int)lvl_fac.size() <= rc.depth) {
      lvl_fac.resize(rc.depth + 1, 0);
      fac_off = 0;
    }
    const SubDev& s = sd[rc.sub];
    const SymShape& sh = *rc.sh;
    const int sid = shape_id[rc.sh];
    const SymFront& f = sh.fronts[rc.idx];
    FrontDev& d = fr[t];
    int m = f.p + f.q;
    d.fac_off = fac_off;
    d.lpk_off = lpk_off;
    d.upk_off = upk_off;
    d.vec_off = (int)vec_off;
    d.piv_off = (int)piv_off;
    d.p = f.p;
    d.q = f.q;
    d.sub = rc.sub;
    d.gx0 = s.ox0 + f.sx0;
    d.gy0 = s.oy0 + f.sy0;
    d.sw = f.sw;
    d.ix0 = s.ix0;
    d.ix1 = s.ix1;
    d.iy0 = s.iy0;
    d.iy1 = s.iy1;
    d.gbase = s.gbase;
    d.gnx = s.gnx;
    d.prob = rc.prob;
    d.var_off = sh_var[sid] + f.var_off;
    d.cmap_off = sh_cmap[sid] + f.cmap_off;
    d.ent_off = sh_ent[sid] + f.ent_off;
    d.ent_cnt = f.ent_cnt;
    d.parent = f.parent >= 0 ? inst[sub_base[rc.sub] + f.parent] : -1;
    STF_REQUIRE(f.nchild <= 2, "internal: more than two children");
    d.child_off = (int)kids.size();
    d.nchild = f.nchild;
    for (int c = 0; c < f.nchild; ++c)
      kids.push_back(inst[sub_base[rc.sub] + sh.children[f.child_off + c]]);
    fac_off += (long long)m * m;
    lvl_fac[rc.depth] = fac_off;
    // Packed sweep operators: the strictly lower trapezoid of the first p
    // columns (forward) and the upper trapezoid of the first p rows (backward).
    lpk_off += (long long)f.p * f.q + (long long)f.p * (f.p - 1) / 2;
    upk_off += (long long)f.p * f.q + (long long)f.p * (f.p + 1) / 2;
    vec_off += m;
    piv_off += f.p;
  }
  mf.upk_elems = upk_off;
  mf.lpk_elems = lpk_off;
  STF_REQUIRE(vec_off < (1LL << 31) && piv_off < (1LL << 31), "problem too large for int32 offsets");
  // Embedded children vector offsets and maps (all offsets are known now).
  for (size_t t = 0; t < fr.size(); ++t) {
    FrontDev& d = fr[t];
    for (int c = 0; c < 2; ++c) {
      if (c < d.nchild) {
        const FrontDev& cf = fr[kids[d.child_off + c]];
        d.cvec[c] = cf.vec_off + cf.p;
        d.ccmap[c] = cf.cmap_off;
        d.cq[c] = cf.q;
      } else {
        d.cvec[c] = 0;
        d.ccmap[c] = 0;
        d.cq[c] = 0;
      }
    }
  }
  mf.n_fronts = (int64_t)fr.size();
  mf.front_sub.resize(fr.size());
  mf.front_depth.resize(fr.size());
  for (size_t t = 0; t < order.size(); ++t) {
    mf.front_sub[t] = recs[order[t]].sub;
    mf.front_depth[t] = recs[order[t]].depth;
  }
  long long arena[2] = {0, 0};
  for (size_t dd = 0; dd < lvl_fac.size(); ++dd) arena[dd & 1] = std::max(arena[dd & 1], lvl_fac[dd]);
  for (size_t t = 0; t < order.size(); ++t)
    if (recs[order[t]].depth & 1) fr[t].fac_off += arena[0];
  mf.fac_elems = arena[0] + arena[1];
  mf.vec_elems = vec_off;
  mf.piv_elems = piv_off;
  mf.levels.clear();
  for (size_t t = 0; t < order.size(); ++t) {
    int dpt = recs[order[t]].depth;
    if ((int)mf.levels.size() <= dpt) {
      mf.levels.resize(dpt + 1);
      mf.levels[dpt].off = (int)t;
    }
    Level& L = mf.levels[dpt];
    L.n += 1;
    L.max_m = std::max(L.max_m, fr[t].p + fr[t].q);
    L.max_pm = std::max(L.max_pm, fr[t].p * (fr[t].p + fr[t].q));
    L.max_p = std::max(L.max_p, fr[t].p);
  }
  mf.max_depth = (int)mf.levels.size() - 1;
  upload(mf.fronts, fr, st);
  upload(mf.children, kids, st);
  mf.fuse.clear();
  mf.h_fronts = std::move(fr);
  mf.h_children = std::move(kids);

  const size_t es = prec == STF_C64 ? sizeof(float2) : sizeof(double2);
  mf.fac.alloc((size_t)mf.fac_elems * es);
  mf.upk.alloc((size_t)mf.upk_elems * es);
  mf.lpk.alloc((size_t)mf.lpk_elems * es);
  mf.piv.alloc((size_t)mf.piv_elems * sizeof(int));
  mf.vec.alloc((size_t)mf.vec_elems * es);
  mf.u.alloc((size_t)mf.u_elems * es);
  mf.ws_nr = 1;
  HIP_CHECK(hipStreamSynchronize(st));
}

struct stf_problem_s {
  stf_ctx ctx = nullptr;
  uint64_t uid = 0;                // unique per problem object
  uint64_t generation = 0;         // incremented by every assembly
  Plan plan;
  stf_params prm{};
  long long N = 0;
  bool assembled = false, factored = false;
  int prec = STF_C128;
  std::unique_ptr<Mf> mf;          // fronts and workspaces (built at the first factorisation)

  // Device state.
  DBuf keps, gcoef, flag;
  DBuf partial, npartial, scal;    // reduction scratch, device scalars
  DBuf kV, kZ, kw, kr, kH, kcs, ksn, kg, ky, kh1, kh2, kt, kt2;
  DBuf ksr;                        // stage residuals of a staged order (one vector per slot)
  DBuf hb, hx, cells;              // staging for host inputs
  int krylov_m = 0, krylov_nr = 0;
  long long kpart_stride = 0;   // double2 entries of one right-hand side's Gram-Schmidt partials
  long long knpart_stride = 0;  // doubles of one right-hand side's norm partials
  // Phase timers: [0, 1] the last factorisation, [2, 3] a solve group, [4 + 2 s, 5 + 2 s]
  // the network's guess of right-hand side s of the group.
  hipEvent_t ev[4 + 2 * MAX_RHS] = {};
  bool fac_timed = false;

  ~stf_problem_s() {
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void make_events() {
    for (hipEvent_t& e : ev)
      if (!e) HIP_CHECK(hipEventCreate(&e));
  }
  // Elapsed ms between events a and b (both recorded and complete), else 0.
  double elapsed(int a, int b) const {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, ev[a], ev[b]) == hipSuccess ? (double)ms : 0.0;
  }

  const double2* cxw() const { return gcoef.as<double2>(); }
  const double2* cxe() const { return gcoef.as<double2>() + prm.nx; }
  const double2* cyw() const { return gcoef.as<double2>() + 2 * prm.nx; }
  const double2* cye() const { return gcoef.as<double2>() + 2 * prm.nx + prm.ny; }

  Mf& ensure_mf() {
    if (!mf) {
      std::unique_ptr<Mf> m(new Mf());
      build_mf(*m, {&plan}, {0LL}, prm.front_prec, ctx->stream);
      mf = std::move(m);
    }
    return *mf;
  }
  int max_depth() const { return mf ? mf->max_depth : -1; }
  int64_t device_bytes() const {
    const DBuf* all[] = {&keps, &gcoef, &flag, &partial, &npartial, &scal, &kV, &kZ, &kw, &kr,
                         &kH, &kcs, &ksn, &kg, &ky, &kh1, &kh2, &kt, &kt2, &ksr, &hb, &hx,
                         &cells};
    int64_t t = 0;
    for (const DBuf* d : all) t += (int64_t)d->bytes;
    return t + (mf ? mf->device_bytes() : 0);
  }
};

// Learned warm start: network parameters, Adam moments, twiddle tables and
// the activations of one batch (kept for the backward pass).
struct stf_nn_s {
  stf_ctx ctx = nullptr;
  stf_nn_config cfg{};
  long long np = 0;
  long long offP = 0, offQ = 0;
  std::vector<long long> offR, offW;   // per layer: Re R (Im R follows), W_l (c_l follows)
  DBuf par, grad, am, av;
  DBuf wq;                             // par rounded to BF16: the weights the kernels read
  DBuf exT;      // (n, 2M) floats: [cos | -sin](2 pi k x / n), the forward x transform
  DBuf ey;       // (2M, n) float2: exp(-2 pi i ky(a) y / n)
  DBuf exi;      // (M, n) float2: exp(+2 pi i k x / n)
  DBuf ainv;     // (n, 4M) floats: [cos | -sin](2 pi ky(a) y / n), the inverse y transform
  int cap = 0;   // batch capacity of the activation buffers
  std::vector<DBuf> h, pre, H;
  DBuf T, G, S, g, dh, dh2, dpre, dG, dH, y, dy, pwpart, lpart, den, loss;
  // Tiling of the last problem passed to stf_nn_initial_guess.
  DBuf org, oy, ox, tf, tpred;
  std::vector<int> hoy, hox;

  int NM() const { return 2 * cfg.modes * cfg.modes; }
  long long npix() const { return (long long)cfg.n * cfg.n; }
};

namespace {

template <typename F>
stf_status guard(stf_ctx c, F&& fn) {
  try {
    if (c) HIP_CHECK(hipSetDevice(c->device));
    fn();
    return STF_OK;
  } catch (const Error& e) {
    if (c) c->last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    return STF_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->last_error = e.what();
    return STF_EDEVICE;
  }
}

bool host_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Rejects non-finite values in a caller array (host or device).
void require_finite(stf_problem pb, const double* a, size_t n, int on_device, const char* what) {
  if (!on_device) {
    STF_REQUIRE(host_finite(a, n), std::string(what) + " holds NaN or Inf");
    return;
  }
  hipStream_t st = pb->ctx->stream;
  HIP_CHECK(hipMemsetAsync(pb->flag.p, 0, sizeof(int), st));
  launch_check_finite(st, a, (long long)n, pb->flag.as<int>());
  int h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, pb->flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  STF_REQUIRE(h == 0, std::string(what) + " holds NaN or Inf");
}

void build_device_state(stf_problem pb) {
  const Plan& pl = pb->plan;
  const stf_params& p = pb->prm;
  hipStream_t st = pb->ctx->stream;
  pb->N = (long long)p.nx * p.ny;
  pb->prec = p.front_prec;

  // Global coupling arrays: cxw | cxe | cyw | cye.
  std::vector<double2> gc;
  for (auto& v : pl.g.cx.w) gc.push_back(make_double2(v.real(), v.imag()));
  for (auto& v : pl.g.cx.e) gc.push_back(make_double2(v.real(), v.imag()));
  for (auto& v : pl.g.cy.w) gc.push_back(make_double2(v.real(), v.imag()));
  for (auto& v : pl.g.cy.e) gc.push_back(make_double2(v.real(), v.imag()));
  upload(pb->gcoef, gc, st);
  pb->keps.alloc((size_t)pb->N * sizeof(double2));
  pb->flag.alloc(sizeof(int) * (4 + MAX_RHS));   // [0] pivot / finite flag, [4 + s] Gram-Schmidt gates
  pb->scal.alloc(sizeof(double) * 64);
  int nblk = std::max(stencil_partial_blocks(p.nx, p.ny), krylov_blocks(pb->N));
  pb->partial.alloc((size_t)nblk * sizeof(double2) * 4);
  pb->npartial.alloc((size_t)std::max(krylov_blocks(pb->N), gs_blocks(pb->N, 32)) * sizeof(double));
  HIP_CHECK(hipStreamSynchronize(st));
}

void assemble_eps(stf_problem pb, const double* eps, int on_device) {
  const stf_params& p = pb->prm;
  size_t ncell = (size_t)(p.nx + 1) * (p.ny + 1);
  require_finite(pb, eps, 2 * ncell, on_device, "eps_cells");
  hipStream_t st = pb->ctx->stream;
  const double2* src = reinterpret_cast<const double2*>(eps);
  if (!on_device) {
    pb->cells.alloc(ncell * sizeof(double2));
    HIP_CHECK(hipMemcpyAsync(pb->cells.p, eps, ncell * sizeof(double2), hipMemcpyHostToDevice, st));
    src = pb->cells.as<double2>();
  }
  {
    Timed t(pb->ctx, K_ASSEMBLE);
    launch_node_keps(st, src, pb->keps.as<double2>(), p.nx, p.ny, p.k0 * p.k0);
  }
  if (!on_device) HIP_CHECK(hipStreamSynchronize(st));   // staging buffer reuse
  pb->assembled = true;
  pb->factored = false;
  pb->generation += 1;
}

// The autotuned shape of a level, or the built-in rule (kind 0) when the
// context has none for its signature.
FactorShape tuned_factor(stf_ctx c, const LevelArgs& a, size_t elem) {
  auto it = c->tune.find(TuneKey{0, (int)elem, 0, a.nlevel, a.max_m, a.max_p});
  if (it == c->tune.end()) return FactorShape{};
  const FactorShape s{it->second.kind, it->second.a, it->second.b};
  return factor_shape_ok(a, elem, s) ? s : FactorShape{};
}

SweepShape tuned_sweep(stf_ctx c, const LevelArgs& a, bool fwd, size_t elem, int nr) {
  auto it = c->tune.find(TuneKey{fwd ? 1 : 2, (int)elem, nr, a.nlevel, a.max_m, a.max_p});
  if (it == c->tune.end()) return SweepShape{};
  const SweepShape s{it->second.kind, it->second.a, it->second.b, it->second.c};
  return sweep_shape_ok(a, fwd, elem, nr, s) ? s : SweepShape{};
}

// Numeric factorisation of every level of a set; with `fault`, the first front
// of tree level 1 gets the planted zero pivot column (test hook): its first
// column carries fill in the update rows after assembly, so the perturbation
// has a nonzero column maximum to scale.  e0 / e1 (may be null) bracket the
// launches.  Returns the perturbation flag (synchronises the stream).
// Launches level d of the factorisation with shape sh.  A level on the
// one-wavefront LDS kernel goes in runs of fronts of similar order (instances
// are stored largest first within a level; a run ends where the order falls
// below 85% of its first), each run with LDS for its own largest front, so
// that the smaller fronts fit more workgroups per CU.
template <typename T>
void factor_level(hipStream_t st, const Mf& mf, int d, const double2* keps, int* flag, double tau, bool fault,
                  FactorShape sh) {
  LevelArgs la = mf.level_args(d, keps);
  if (fault && d == 1) la.fault = la.first;
  const FactorShape s = sh.kind == 0 ? factor_default(la, sizeof(T)) : sh;
  T* fac = mf.fac.as<T>();
  if (s.kind != 1) {
    launch_front_factor<T>(st, la, fac, mf.lpk.as<T>(), mf.upk.as<T>(), mf.piv.as<int>(), flag, tau, s);
    return;
  }
  const int off = mf.levels[d].off, n = mf.levels[d].n;
  for (int i = 0; i < n;) {
    const int m0 = mf.h_fronts[off + i].p + mf.h_fronts[off + i].q;
    int j = i + 1;
    while (j < n && 20 * (mf.h_fronts[off + j].p + mf.h_fronts[off + j].q) >= 17 * m0) ++j;
    LevelArgs run = la;
    run.first = off + i;
    run.nlevel = j - i;
    run.max_m = m0;
    launch_front_factor<T>(st, run, fac, mf.lpk.as<T>(), mf.upk.as<T>(), mf.piv.as<int>(), flag, tau, s);
    i = j;
  }
}

template <typename T>
int factor_mf(stf_ctx c, Mf& mf, const double2* keps, int* flag, bool fault, hipEvent_t e0,
              hipEvent_t e1) {
  STF_REQUIRE(!fault || mf.max_depth >= 1, "the planted fault needs a tree of two levels or more");
  hipStream_t st = c->stream;
  HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), st));
  double tau = sizeof(T) == 16 ? 1e-10 : 1e-5;
  if (e0) HIP_CHECK(hipEventRecord(e0, st));
  for (int d = mf.max_depth; d >= 0; --d) {
    Timed t(c, K_FRONT_LU);
    factor_level<T>(st, mf, d, keps, flag, tau, fault, tuned_factor(c, mf.level_args(d, keps), sizeof(T)));
  }
  if (e1) HIP_CHECK(hipEventRecord(e1, st));
  HIP_CHECK(hipGetLastError());
  int h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return h;
}

// The context's second stream: fork() makes its next work wait for what the
// main stream holds so far, run(f) issues f's launches (those of the context
// and of the network's context) on it, join() makes the main stream wait for
// everything issued on it.
struct SideStream {
  stf_ctx c, nc;
  hipStream_t main;
  SideStream(stf_ctx c_, stf_ctx nc_) : c(c_), nc(nc_), main(c_->stream) {
    if (!c->side) HIP_CHECK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    for (int e = 0; e < 2; ++e)
      if (!c->side_ev[e]) HIP_CHECK(hipEventCreateWithFlags(&c->side_ev[e], hipEventDisableTiming));
  }
  // The side stream's next work waits for what the main stream holds so far.
  void fork() {
    HIP_CHECK(hipEventRecord(c->side_ev[0], main));
    HIP_CHECK(hipStreamWaitEvent(c->side, c->side_ev[0], 0));
  }
  template <typename F>
  void run(F&& f) {
    c->stream = c->side;
    if (nc) nc->stream = c->side;
    try {
      f();
    } catch (...) {
      c->stream = main;
      if (nc) nc->stream = main;
      throw;
    }
    c->stream = main;
    if (nc) nc->stream = main;
  }
  void join() {
    HIP_CHECK(hipEventRecord(c->side_ev[1], c->side));
    HIP_CHECK(hipStreamWaitEvent(main, c->side_ev[1], 0));
  }
};


void fuse_prepare(stf_ctx c, Mf& mf);

int factor_problem(stf_problem pb, bool fault = false) {
  Mf& mf = pb->ensure_mf();
  const double2* keps = pb->keps.as<double2>();
  int* flag = pb->flag.as<int>();
  const int h = mf.prec == STF_C64
                    ? factor_mf<float2>(pb->ctx, mf, keps, flag, fault, pb->ev[0], pb->ev[1])
                    : factor_mf<double2>(pb->ctx, mf, keps, flag, fault, pb->ev[0], pb->ev[1]);
  pb->fac_timed = true;
  fuse_prepare(pb->ctx, mf);
  return h;
}

// Subtree sweeps of a set for nr right-hand sides, as a code 16 D + T (roots
// at depth D, T subtrees per workgroup) or -1 (level by level): the
// autotuned choice when the context has one for the set's signature, else
// -1 (on the 1064^2 metasurface at 8 x 8 subdomains the subtree sweeps
// measure slower, since a workgroup takes its subtrees' fronts one level
// after another).
TuneKey fuse_key(const Mf& mf, size_t elem, int nr) {
  return TuneKey{3, (int)elem, nr, (int)std::min<int64_t>(mf.n_fronts, INT32_MAX), mf.max_depth, mf.nsub};
}

// With build = false, only tables already built count (no allocation).
int fuse_depth_for(stf_ctx c, Mf& mf, size_t elem, int nr, bool build = true) {
  auto it = c->tune.find(fuse_key(mf, elem, nr));
  const int dmin = mf.fuse_min_depth();
  if (it == c->tune.end()) return -1;
  const int D = it->second.a, T = it->second.b;
  if (D < 0 || dmin < 0 || D < dmin || D >= mf.max_depth || T < 1 || T > 8) return -1;
  const int code = 16 * D + T;
  if (!build && !mf.fuse.count(code)) return -1;
  return subtree_ok(mf.fuse_plan(code, c->stream).args, elem, nr) ? code : -1;
}

// Builds the subtree tables the rounds of a set will use (outside graph
// captures and allocation-free calls).
void fuse_prepare(stf_ctx c, Mf& mf) {
  const size_t elem = mf.prec == STF_C64 ? sizeof(float2) : sizeof(double2);
  for (int nr = 1; nr <= MAX_RHS; ++nr) (void)fuse_depth_for(c, mf, elem, nr, true);
}

// Subtree-sweep choices for a set: the built-in one (level by level, -1)
// first, then every root depth and subtrees per workgroup (1, 2, 4, 8) that
// fit, as codes 16 D + T.
std::vector<int> fuse_options(stf_ctx c, Mf& mf, size_t elem, int nr) {
  std::vector<int> out{-1};
  const int dmin = mf.fuse_min_depth();
  if (dmin >= 0)
    for (int D = dmin; D < mf.max_depth; ++D)
      for (int T : {1, 2, 4, 8})
        if (subtree_ok(mf.fuse_plan(16 * D + T, c->stream).args, elem, nr)) out.push_back(16 * D + T);
  return out;
}

// z_s = sum_k P_k A_k^{-1} R_k^I v_s (one source-transfer round) for the
// right-hand sides of r, swept together, over every problem of the set (those
// with pact[p] == 0 skipped when pact is given).  Explicit workspaces: front
// vectors `vec` and local fields `u` (vec_elems and u_elems entries per
// right-hand side).  With timed = false no event is recorded (the
// allocation-free entry point).
// The forward and backward sweeps of a round: with a subtree choice
// (code = 16 D + T >= 0) the deep levels (depth >= D) as subtree sweeps, the
// rest level by level.  r: strides set.
template <typename T>
void sweeps_launch(stf_ctx c, Mf& mf, const RhsSet& r, T* vec, T* u, stf_ctx tc, const int* pact, int code) {
  hipStream_t st = c->stream;
  const T* lpk = mf.lpk.as<T>();
  const int D = code >= 0 ? code / 16 : -1;
  const int top = D >= 0 ? D : mf.max_depth + 1;
  if (D >= 0) {
    Timed t(tc, K_SWEEP_FWD);
    launch_fwd_subtree<T>(st, mf.level_args(mf.max_depth, nullptr, pact), mf.fuse_plan(code, st).args, lpk,
                          mf.piv.as<int>(), vec, r);
  }
  for (int d = top - 1; d >= 0; --d) {
    Timed t(tc, K_SWEEP_FWD);
    const LevelArgs la = mf.level_args(d, nullptr, pact);
    launch_sweep_fwd<T>(st, la, lpk, mf.piv.as<int>(), vec, r, tuned_sweep(c, la, true, sizeof(T), r.nr));
  }
  for (int d = 0; d < top; ++d) {
    Timed t(tc, K_SWEEP_BWD);
    const LevelArgs la = mf.level_args(d, nullptr, pact);
    launch_sweep_bwd<T>(st, la, mf.upk.as<T>(), vec, u, r, tuned_sweep(c, la, false, sizeof(T), r.nr));
  }
  if (D >= 0) {
    Timed t(tc, K_SWEEP_BWD);
    launch_bwd_subtree<T>(st, mf.level_args(mf.max_depth, nullptr, pact), mf.fuse_plan(code, st).args,
                          mf.upk.as<T>(), vec, u, r);
  }
}

// fuse: 0 level by level only, 1 subtree sweeps whose tables exist, 2 also
// building the tables.
template <typename T>
void precond_launch(stf_ctx c, Mf& mf, RhsSet r, T* vec, T* u, bool timed,
                    const int* pact = nullptr, int fuse = 2) {
  hipStream_t st = c->stream;
  stf_ctx tc = timed ? c : nullptr;
  r.vec_stride = mf.vec_elems;
  r.u_stride = mf.u_elems;
  const int D = fuse > 0 ? fuse_depth_for(c, mf, sizeof(T), r.nr, fuse == 2) : -1;
  sweeps_launch<T>(c, mf, r, vec, u, tc, pact, D);
  Timed t(tc, K_SCATTER);
  launch_scatter<T>(st, u, mf.subs.as<SubDev>(), mf.cover_x.as<int4>(), mf.cover_y.as<int4>(),
                    mf.scat.as<ScatDev>(), mf.nprob, mf.max_nx, mf.max_ny, pact, r);
}

// The same with the set's own workspaces, grown to r.nr right-hand sides.
template <typename T>
void precond_mf(stf_ctx c, Mf& mf, const RhsSet& r, const int* pact = nullptr) {
  if (mf.ws_nr < r.nr) {
    const size_t es = sizeof(T);
    mf.vec.alloc((size_t)mf.vec_elems * es * r.nr);
    mf.u.alloc((size_t)mf.u_elems * es * r.nr);
    mf.ws_nr = r.nr;
  }
  precond_launch<T>(c, mf, r, mf.vec.as<T>(), mf.u.as<T>(), true, pact);
}

// Stages of problem p (subdomain k = ky * px + kx of that problem) for a
// staged order: 1 symmetric rows, 2 symmetric rows then symmetric columns,
// 3 four diagonal sweeps (kx + ky rising and falling, then kx + (py-1-ky)
// rising and falling), 4 two colours (kx + ky even, then odd; a single
// subdomain has one stage).
std::vector<std::vector<int>> order_stages(int order, int px, int py) {
  std::vector<std::vector<int>> rows(py), cols(px), out;
  for (int ky = 0; ky < py; ++ky)
    for (int kx = 0; kx < px; ++kx) {
      rows[ky].push_back(ky * px + kx);
      cols[kx].push_back(ky * px + kx);
    }
  auto there_and_back = [&](const std::vector<std::vector<int>>& seq) {
    for (size_t i = 0; i < seq.size(); ++i) out.push_back(seq[i]);
    for (int i = (int)seq.size() - 2; i >= 0; --i) out.push_back(seq[i]);
  };
  if (order == STF_ORDER_ROWS) {
    there_and_back(rows);
  } else if (order == STF_ORDER_ROWS_COLS) {
    there_and_back(rows);
    there_and_back(cols);
  } else if (order == STF_ORDER_DIAGONAL) {
    const int nd = px + py - 1;
    std::vector<std::vector<int>> d1(nd), d2(nd);
    for (int ky = 0; ky < py; ++ky)
      for (int kx = 0; kx < px; ++kx) {
        d1[kx + ky].push_back(ky * px + kx);
        d2[kx + (py - 1 - ky)].push_back(ky * px + kx);
      }
    there_and_back(d1);
    there_and_back(d2);
  } else if (order == STF_ORDER_CHECKER) {
    for (int c = 0; c < 2; ++c) {
      std::vector<int> st;
      for (int ky = 0; ky < py; ++ky)
        for (int kx = 0; kx < px; ++kx)
          if ((kx + ky) % 2 == c) st.push_back(ky * px + kx);
      if (!st.empty()) out.push_back(st);
    }
  } else {
    throw Error(STF_EINVAL, "unknown sweeping order");
  }
  return out;
}

const SweepPlan& sweep_plan(Mf& mf, int order, hipStream_t st) {
  auto it = mf.sweeps.find(order);
  if (it != mf.sweeps.end()) return *it->second;
  std::unique_ptr<SweepPlan> sp(new SweepPlan());
  // first subdomain of every problem
  std::vector<int> sub0(mf.nprob, -1);
  for (int k = 0; k < mf.nsub; ++k)
    if (sub0[mf.sub_prob[k]] < 0) sub0[mf.sub_prob[k]] = k;
  std::vector<std::vector<std::vector<int>>> per(mf.nprob);
  int nst = 0;
  for (int p = 0; p < mf.nprob; ++p) {
    per[p] = order_stages(order, mf.prob_px[p], mf.prob_py[p]);
    nst = std::max(nst, (int)per[p].size());
  }
  // front instances of every subdomain by depth (level order, largest first)
  const int nd = mf.max_depth + 1;
  std::vector<std::vector<std::vector<int>>> fsd(mf.nsub, std::vector<std::vector<int>>(nd));
  for (size_t t = 0; t < mf.front_sub.size(); ++t) fsd[mf.front_sub[t]][mf.front_depth[t]].push_back((int)t);
  std::vector<int> slist, flist, inst((size_t)nst * mf.nsub, 0);
  sp->nstage = nst;
  sp->lv.assign(nst, std::vector<Level>(nd));
  for (int t = 0; t < nst; ++t) {
    std::vector<int> mem;
    for (int p = 0; p < mf.nprob; ++p)
      if (t < (int)per[p].size())
        for (int k : per[p][t]) mem.push_back(sub0[p] + k);
    sp->s_first.push_back((int)slist.size());
    sp->s_count.push_back((int)mem.size());
    slist.insert(slist.end(), mem.begin(), mem.end());
    for (int k : mem) inst[(size_t)t * mf.nsub + k] = 1;
    for (int d = 0; d < nd; ++d) {
      std::vector<int> fl;
      for (int k : mem) fl.insert(fl.end(), fsd[k][d].begin(), fsd[k][d].end());
      // largest first: instance order within a level is by descending order m
      std::sort(fl.begin(), fl.end());
      Level L = mf.levels[d];
      L.off = (int)flist.size();
      L.n = (int)fl.size();
      sp->lv[t][d] = L;
      flist.insert(flist.end(), fl.begin(), fl.end());
    }
  }
  upload(sp->slist, slist, st);
  upload(sp->flist, flist, st);
  upload(sp->inst, inst, st);
  // A stage level's launch reads its fronts' descriptors from this copy
  // directly (one dependent load per workgroup instead of two).
  std::vector<FrontDev> fd(flist.size());
  for (size_t i = 0; i < flist.size(); ++i) fd[i] = mf.h_fronts[flist[i]];
  upload(sp->fdev, fd, st);
  sp->h_flist = flist;
  HIP_CHECK(hipStreamSynchronize(st));
  const SweepPlan& ref = *sp;
  mf.sweeps[order] = std::move(sp);
  return ref;
}

// The per-stage subtree tables of a staged order for choice `code`
// (16 D + T), built on first use.
const std::vector<std::unique_ptr<FusePlan>>& stage_fuse(const Mf& mf, const SweepPlan& spc, int code,
                                                          hipStream_t st) {
  SweepPlan& sp = const_cast<SweepPlan&>(spc);
  auto it = sp.fuse.find(code);
  if (it != sp.fuse.end()) return it->second;
  const int D = code / 16, T = code % 16;
  std::vector<std::unique_ptr<FusePlan>> per(sp.nstage);
  for (int t = 0; t < sp.nstage; ++t) {
    const Level& L = sp.lv[t][D];
    if (L.n == 0) continue;
    std::vector<int> roots(sp.h_flist.begin() + L.off, sp.h_flist.begin() + L.off + L.n);
    per[t] = mf.build_fuse(roots, D, T, st);
  }
  return sp.fuse[code] = std::move(per);
}

// Subtree choice (16 D + T) for the stages of `order` on a set with nr
// right-hand sides: the autotuned one (operation 3 + order) or -1 (level by
// level).  With build = false only tables already built count.
TuneKey staged_fuse_key(const Mf& mf, size_t elem, int nr, int order) {
  return TuneKey{3 + order, (int)elem, nr, (int)std::min<int64_t>(mf.n_fronts, INT32_MAX), mf.max_depth,
                 mf.nsub};
}

int staged_fuse_for(stf_ctx c, Mf& mf, const SweepPlan& sp, size_t elem, int nr, int order, bool build) {
  auto it = c->tune.find(staged_fuse_key(mf, elem, nr, order));
  const int dmin = mf.fuse_min_depth();
  if (it == c->tune.end()) return -1;
  const int D = it->second.a, T = it->second.b;
  if (D < 0 || dmin < 0 || D < dmin || D >= mf.max_depth || T < 1 || T > 8) return -1;
  const int code = 16 * D + T;
  if (!build && !sp.fuse.count(code)) return -1;
  for (const auto& f : stage_fuse(mf, sp, code, c->stream))
    if (f && !subtree_ok(f->args, elem, nr)) return -1;
  return code;
}

// Level d of stage t as launch arguments: the stage's fronts of that level
// (their descriptors from the stage plan's copy), the level's largest orders.
LevelArgs stage_level_args(const Mf& mf, const SweepPlan& sp, int t, int d, const int* pact) {
  LevelArgs la = mf.level_args(d, nullptr, pact);
  la.fronts = sp.fdev.as<FrontDev>();
  la.flist = nullptr;
  la.first = sp.lv[t][d].off;
  la.nlevel = sp.lv[t][d].n;
  return la;
}

// One application of the staged order for the right-hand sides of r: for
// every stage r_s = v_s - A z_s on its own boxes (skipped for the first stage,
// where z = 0), its sweeps, z_s += its full local fields (the first stage's
// sum writes every node of z_s, so no zero fill comes first).
// keps / gc: the set's concatenated node permittivity and coupling arrays;
// rbuf: one global vector per slot (rstride apart) for the stage residuals.
// code: subtree choice (16 D + T) for the deep levels of every stage, or -1
// (level by level); its tables must exist (stage_fuse) when the call is
// captured into a graph.
template <typename T>
void sweep_launch(stf_ctx c, Mf& mf, const SweepPlan& sp, RhsSet r, T* vec, T* u,
                  const double2* keps, const double2* gc, double2* rbuf, long long rstride,
                  bool timed, const int* pact = nullptr, int code = -1) {
  hipStream_t st = c->stream;
  stf_ctx tc = timed ? c : nullptr;
  r.vec_stride = mf.vec_elems;
  r.u_stride = mf.u_elems;
  const T* lpk = mf.lpk.as<T>();
  const int* sl = sp.slist.as<int>();
  const std::vector<std::unique_ptr<FusePlan>>* sfz = code >= 0 ? &stage_fuse(mf, sp, code, st) : nullptr;
  const int Dz = code >= 0 ? code / 16 : mf.max_depth + 1;
  for (int t = 0; t < sp.nstage; ++t) {
    const FusePlan* fz = sfz ? (*sfz)[t].get() : nullptr;
    const int top = fz ? Dz : mf.max_depth + 1;
    const int sf = sp.s_first[t], sc = sp.s_count[t];
    RhsSet rr = r;
    if (t > 0) {
      Timed tm(tc, K_STENCIL);
      launch_stage_residual(st, keps, gc, mf.subs.as<SubDev>(), mf.scat.as<ScatDev>(), sl, sf, sc,
                            mf.max_ixl, mf.max_iyl, pact, r, rbuf, rstride);
      for (int s = 0; s < r.nr; ++s) rr.v[s] = rbuf + s * rstride;
    }
    if (fz) {
      Timed tm(tc, K_SWEEP_FWD);
      launch_fwd_subtree<T>(st, mf.level_args(mf.max_depth, nullptr, pact), fz->args, lpk, mf.piv.as<int>(),
                            vec, rr);
    }
    for (int d = top - 1; d >= 0; --d) {
      if (sp.lv[t][d].n == 0) continue;
      Timed tm(tc, K_SWEEP_FWD);
      const LevelArgs la = stage_level_args(mf, sp, t, d, pact);
      launch_sweep_fwd<T>(st, la, lpk, mf.piv.as<int>(), vec, rr, tuned_sweep(c, la, true, sizeof(T), rr.nr));
    }
    for (int d = 0; d < top; ++d) {
      if (sp.lv[t][d].n == 0) continue;
      Timed tm(tc, K_SWEEP_BWD);
      const LevelArgs la = stage_level_args(mf, sp, t, d, pact);
      launch_sweep_bwd<T>(st, la, mf.upk.as<T>(), vec, u, rr, tuned_sweep(c, la, false, sizeof(T), rr.nr));
    }
    if (fz) {
      Timed tm(tc, K_SWEEP_BWD);
      launch_bwd_subtree<T>(st, mf.level_args(mf.max_depth, nullptr, pact), fz->args, mf.upk.as<T>(), vec,
                            u, rr);
    }
    Timed tm(tc, K_SCATTER);
    if (t == 0)
      launch_stage_scatter_first<T>(st, u, mf.subs.as<SubDev>(), mf.cover_x.as<int4>(), mf.cover_y.as<int4>(),
                                    mf.scat.as<ScatDev>(), mf.nprob, mf.max_nx, mf.max_ny,
                                    sp.inst.as<int>(), pact, r);
    else
      launch_stage_scatter<T>(st, u, mf.subs.as<SubDev>(), mf.scat.as<ScatDev>(), mf.cover_x.as<int4>(),
                              mf.cover_y.as<int4>(), sl, sf, sc, mf.max_oxl, mf.max_oyl,
                              sp.inst.as<int>() + (size_t)t * mf.nsub, pact, r);
  }
}

// ---------------------------------------------------------------------------
// Autotuner: every candidate launch shape of every level is timed with HIP
// events over `reps` passes (the fastest pass per shape counts, so the first
// launch of a variant, which loads its code, does not), and the fastest shape
// per level signature is kept in the context.  The factorisation trials run
// whole factorisations (each re-assembles every front from keps, so passes
// do not depend on each other); the sweep trials run the forward and backward
// sweeps of whole rounds on zero right-hand sides (a round is a pure function
// of its input).  Levels with fewer candidates repeat their last one.
// ---------------------------------------------------------------------------
struct EventSet {
  std::vector<hipEvent_t> e;
  explicit EventSet(size_t n) : e(n, nullptr) {
    for (hipEvent_t& x : e) HIP_CHECK(hipEventCreate(&x));
  }
  ~EventSet() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
  double ms(size_t i, size_t j) const {
    float v = 0.f;
    HIP_CHECK(hipEventElapsedTime(&v, e[i], e[j]));
    return v;
  }
};

struct TuneTally {
  int levels = 0, changed = 0;
  double ms_default = 0.0, ms_tuned = 0.0;
  int fuse_depth = -1;                              // chosen subtree root depth (-1: none)
  double ms_round_default = 0.0, ms_round_tuned = 0.0;
};



// Keeps the fastest of `times` (one per candidate, candidate 0 = built-in).
template <typename S>
void tune_keep(stf_ctx c, const TuneKey& key, const std::vector<S>& cand, const std::vector<double>& times,
               TuneTally& tally, TuneEntry (*enc)(const S&)) {
  size_t best = 0;
  for (size_t k = 1; k < cand.size(); ++k)
    if (times[k] < times[best]) best = k;
  TuneEntry e = enc(cand[best]);
  e.ms = times[best];
  e.ms_default = times[0];
  c->tune[key] = e;
  tally.levels += 1;
  tally.changed += best != 0;
  tally.ms_default += times[0];
  tally.ms_tuned += times[best];
}

TuneEntry enc_factor(const FactorShape& s) { return TuneEntry{s.kind, s.nb, s.ntf, 0, 0.0, 0.0}; }
TuneEntry enc_sweep(const SweepShape& s) { return TuneEntry{s.kind, s.kp, s.ntl, s.parts, 0.0, 0.0}; }

template <typename T>
void tune_factor_mf(stf_ctx c, Mf& mf, const double2* keps, int* flag, int reps, TuneTally& tally) {
  hipStream_t st = c->stream;
  const int L = mf.max_depth + 1;
  std::vector<std::vector<FactorShape>> cand(L);
  std::vector<std::vector<double>> best(L);
  size_t ntr = 1;
  for (int d = 0; d < L; ++d) {
    cand[d] = factor_candidates(mf.level_args(d, keps), sizeof(T));
    best[d].assign(cand[d].size(), 1e300);
    ntr = std::max(ntr, cand[d].size());
  }
  const double tau = sizeof(T) == 16 ? 1e-10 : 1e-5;
  EventSet ev((size_t)L + 1);
  for (int rep = 0; rep < reps; ++rep)
    for (size_t t = 0; t < ntr; ++t) {
      HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), st));
      HIP_CHECK(hipEventRecord(ev.e[0], st));
      for (int d = mf.max_depth, i = 1; d >= 0; --d, ++i) {
        const size_t k = std::min(t, cand[d].size() - 1);
        factor_level<T>(st, mf, d, keps, flag, tau, false, cand[d][k]);
        HIP_CHECK(hipEventRecord(ev.e[i], st));
      }
      HIP_CHECK(hipEventSynchronize(ev.e[L]));
      for (int d = mf.max_depth, i = 1; d >= 0; --d, ++i)
        if (t < cand[d].size()) best[d][t] = std::min(best[d][t], ev.ms(i - 1, i));
    }
  for (int d = 0; d < L; ++d) {
    const LevelArgs a = mf.level_args(d, keps);
    tune_keep(c, TuneKey{0, (int)sizeof(T), 0, a.nlevel, a.max_m, a.max_p}, cand[d], best[d], tally,
              enc_factor);
  }
}

template <typename T>
void tune_sweeps_mf(stf_ctx c, Mf& mf, int nr, long long ntot, int reps, TuneTally& tally) {
  hipStream_t st = c->stream;
  if (mf.ws_nr < nr) {
    mf.vec.alloc((size_t)mf.vec_elems * sizeof(T) * nr);
    mf.u.alloc((size_t)mf.u_elems * sizeof(T) * nr);
    mf.ws_nr = nr;
  }
  DBuf v0;
  v0.alloc((size_t)ntot * nr * sizeof(double2));
  launch_zero(st, v0.as<double2>(), ntot * nr);
  RhsSet r;
  r.nr = nr;
  r.vec_stride = mf.vec_elems;
  r.u_stride = mf.u_elems;
  for (int s = 0; s < nr; ++s) r.v[s] = v0.as<double2>() + (size_t)s * ntot;
  const int L = mf.max_depth + 1;
  std::vector<std::vector<SweepShape>> cand[2];
  std::vector<std::vector<double>> best[2];
  size_t ntr = 1;
  for (int w = 0; w < 2; ++w) {
    cand[w].resize(L);
    best[w].resize(L);
    for (int d = 0; d < L; ++d) {
      cand[w][d] = sweep_candidates(mf.level_args(d, nullptr), w == 0, sizeof(T), nr);
      best[w][d].assign(cand[w][d].size(), 1e300);
      ntr = std::max(ntr, cand[w][d].size());
    }
  }
  EventSet ev(2 * (size_t)L + 1);
  T* vec = mf.vec.as<T>();
  T* u = mf.u.as<T>();
  for (int rep = 0; rep < reps; ++rep)
    for (size_t t = 0; t < ntr; ++t) {
      HIP_CHECK(hipEventRecord(ev.e[0], st));
      int i = 1;
      for (int d = mf.max_depth; d >= 0; --d, ++i) {
        const size_t k = std::min(t, cand[0][d].size() - 1);
        launch_sweep_fwd<T>(st, mf.level_args(d, nullptr), mf.lpk.as<T>(), mf.piv.as<int>(), vec, r,
                            cand[0][d][k]);
        HIP_CHECK(hipEventRecord(ev.e[i], st));
      }
      for (int d = 0; d <= mf.max_depth; ++d, ++i) {
        const size_t k = std::min(t, cand[1][d].size() - 1);
        launch_sweep_bwd<T>(st, mf.level_args(d, nullptr), mf.upk.as<T>(), vec, u, r, cand[1][d][k]);
        HIP_CHECK(hipEventRecord(ev.e[i], st));
      }
      HIP_CHECK(hipEventSynchronize(ev.e[2 * L]));
      i = 1;
      for (int d = mf.max_depth; d >= 0; --d, ++i)
        if (t < cand[0][d].size()) best[0][d][t] = std::min(best[0][d][t], ev.ms(i - 1, i));
      for (int d = 0; d <= mf.max_depth; ++d, ++i)
        if (t < cand[1][d].size()) best[1][d][t] = std::min(best[1][d][t], ev.ms(i - 1, i));
    }
  HIP_CHECK(hipStreamSynchronize(st));
  for (int w = 0; w < 2; ++w)
    for (int d = 0; d < L; ++d) {
      const LevelArgs a = mf.level_args(d, nullptr);
      tune_keep(c, TuneKey{w == 0 ? 1 : 2, (int)sizeof(T), nr, a.nlevel, a.max_m, a.max_p}, cand[w][d],
                best[w][d], tally, enc_sweep);
    }
  // Then the subtree sweeps: whole rounds' sweeps (with the shapes just chosen)
  // for each root depth D that fits, against level by level (D = -1).
  const TuneKey fk = fuse_key(mf, sizeof(T), nr);
  c->tune.erase(fk);
  const std::vector<int> opts = fuse_options(c, mf, sizeof(T), nr);
  std::vector<double> tf(opts.size(), 1e300);
  EventSet fe(2);
  for (int rep = 0; rep < reps; ++rep)
    for (size_t k = 0; k < opts.size(); ++k) {
      HIP_CHECK(hipEventRecord(fe.e[0], st));
      sweeps_launch<T>(c, mf, r, vec, u, nullptr, nullptr, opts[k]);
      HIP_CHECK(hipEventRecord(fe.e[1], st));
      HIP_CHECK(hipEventSynchronize(fe.e[1]));
      tf[k] = std::min(tf[k], fe.ms(0, 1));
    }
  size_t bk = 0;
  for (size_t k = 1; k < opts.size(); ++k)
    if (tf[k] < tf[bk]) bk = k;
  c->tune[fk] = opts[bk] < 0 ? TuneEntry{1, -1, 1, 0, tf[bk], tf[0]}
                             : TuneEntry{1, opts[bk] / 16, opts[bk] % 16, 0, tf[bk], tf[0]};
  tally.fuse_depth = opts[bk] < 0 ? -1 : opts[bk] / 16;
  tally.ms_round_default = tf[0];
  tally.ms_round_tuned = tf[bk];
}

// Stage levels of a staged order grouped by launch signature (direction w:
// 0 forward, 1 backward), each with the (stage, depth) pairs that have it.
std::map<TuneKey, std::vector<std::pair<int, int>>> stage_level_groups(const Mf& mf, const SweepPlan& sp,
                                                                        size_t elem, int nr, int w) {
  std::map<TuneKey, std::vector<std::pair<int, int>>> g;
  for (int t = 0; t < sp.nstage; ++t)
    for (int d = 0; d <= mf.max_depth; ++d) {
      if (sp.lv[t][d].n == 0) continue;
      const LevelArgs la = stage_level_args(mf, sp, t, d, nullptr);
      g[TuneKey{w == 0 ? 1 : 2, (int)elem, nr, la.nlevel, la.max_m, la.max_p}].push_back({t, d});
    }
  return g;
}

// Staged orders: first the launch shape of every stage-level signature (every
// candidate timed over all the stage levels that have the signature, on zero
// right-hand sides), then whole applications of `order` for each subtree
// choice, level by level first; keeps the fastest for the set's signature
// (operation 3 + order).
template <typename T>
void tune_staged_mf(stf_ctx c, Mf& mf, int nr, long long ntot, const double2* keps, const double2* gc,
                    int order, int reps, TuneTally& tally) {
  hipStream_t st = c->stream;
  if (mf.ws_nr < nr) {
    mf.vec.alloc((size_t)mf.vec_elems * sizeof(T) * nr);
    mf.u.alloc((size_t)mf.u_elems * sizeof(T) * nr);
    mf.ws_nr = nr;
  }
  DBuf v0, z, rb;
  v0.alloc((size_t)ntot * nr * sizeof(double2));
  z.alloc((size_t)ntot * nr * sizeof(double2));
  rb.alloc((size_t)ntot * nr * sizeof(double2));
  launch_zero(st, v0.as<double2>(), ntot * nr);
  RhsSet r;
  r.nr = nr;
  for (int s = 0; s < nr; ++s) {
    r.v[s] = v0.as<double2>() + (size_t)s * ntot;
    r.z[s] = z.as<double2>() + (size_t)s * ntot;
  }
  const SweepPlan& sp = sweep_plan(mf, order, st);
  {
    RhsSet rz = r;
    rz.vec_stride = mf.vec_elems;
    rz.u_stride = mf.u_elems;
    EventSet ev(2);
    for (int w = 0; w < 2; ++w)
      for (const auto& kv : stage_level_groups(mf, sp, sizeof(T), nr, w)) {
        const auto& members = kv.second;
        const LevelArgs a0 = stage_level_args(mf, sp, members[0].first, members[0].second, nullptr);
        const std::vector<SweepShape> cand = sweep_candidates(a0, w == 0, sizeof(T), nr);
        std::vector<double> times(cand.size(), 1e300);
        for (int rep = 0; rep < reps; ++rep)
          for (size_t k = 0; k < cand.size(); ++k) {
            HIP_CHECK(hipEventRecord(ev.e[0], st));
            for (const auto& td : members) {
              const LevelArgs la = stage_level_args(mf, sp, td.first, td.second, nullptr);
              if (w == 0)
                launch_sweep_fwd<T>(st, la, mf.lpk.as<T>(), mf.piv.as<int>(), mf.vec.as<T>(), rz, cand[k]);
              else
                launch_sweep_bwd<T>(st, la, mf.upk.as<T>(), mf.vec.as<T>(), mf.u.as<T>(), rz, cand[k]);
            }
            HIP_CHECK(hipEventRecord(ev.e[1], st));
            HIP_CHECK(hipEventSynchronize(ev.e[1]));
            times[k] = std::min(times[k], ev.ms(0, 1));
          }
        tune_keep(c, kv.first, cand, times, tally, enc_sweep);
      }
  }
  const TuneKey key = staged_fuse_key(mf, sizeof(T), nr, order);
  c->tune.erase(key);
  const std::vector<int> opts = fuse_options(c, mf, sizeof(T), nr);
  std::vector<double> tf(opts.size(), 1e300);
  EventSet fe(2);
  for (int rep = 0; rep < reps; ++rep)
    for (size_t k = 0; k < opts.size(); ++k) {
      if (opts[k] >= 0) {
        bool ok = true;
        for (const auto& f : stage_fuse(mf, sp, opts[k], st))
          if (f && !subtree_ok(f->args, sizeof(T), nr)) ok = false;
        if (!ok) continue;
      }
      HIP_CHECK(hipEventRecord(fe.e[0], st));
      sweep_launch<T>(c, mf, sp, r, mf.vec.as<T>(), mf.u.as<T>(), keps, gc, rb.as<double2>(), ntot, false,
                      nullptr, opts[k]);
      HIP_CHECK(hipEventRecord(fe.e[1], st));
      HIP_CHECK(hipEventSynchronize(fe.e[1]));
      tf[k] = std::min(tf[k], fe.ms(0, 1));
    }
  size_t bk = 0;
  for (size_t k = 1; k < opts.size(); ++k)
    if (tf[k] < tf[bk]) bk = k;
  c->tune[key] = opts[bk] < 0 ? TuneEntry{1, -1, 1, 0, tf[bk], tf[0]}
                              : TuneEntry{1, opts[bk] / 16, opts[bk] % 16, 0, tf[bk], tf[0]};
  HIP_CHECK(hipStreamSynchronize(st));
}

// Sets every level's entry of a set to candidate `index` (clamped per level);
// returns the largest candidate count.
template <typename T>
int tune_pick_mf(stf_ctx c, Mf& mf, const double2* keps, int nr, int what, int index) {
  int most = 0;
  for (int d = 0; d <= mf.max_depth; ++d) {
    const LevelArgs a = mf.level_args(d, keps);
    if (what & 1) {
      const auto cand = factor_candidates(a, sizeof(T));
      most = std::max(most, (int)cand.size());
      TuneEntry e = enc_factor(cand[std::min<size_t>(index, cand.size() - 1)]);
      c->tune[TuneKey{0, (int)sizeof(T), 0, a.nlevel, a.max_m, a.max_p}] = e;
    }
    if (what & 2)
      for (int w = 0; w < 2; ++w) {
        const auto cand = sweep_candidates(a, w == 0, sizeof(T), nr);
        most = std::max(most, (int)cand.size());
        TuneEntry e = enc_sweep(cand[std::min<size_t>(index, cand.size() - 1)]);
        c->tune[TuneKey{w == 0 ? 1 : 2, (int)sizeof(T), nr, a.nlevel, a.max_m, a.max_p}] = e;
      }
  }
  for (int order = 1; order <= STF_ORDER_CHECKER; ++order) {
    if (!(what & (2 << order))) continue;
    const SweepPlan& sp = sweep_plan(mf, order, c->stream);
    for (int w = 0; w < 2; ++w)
      for (const auto& kv : stage_level_groups(mf, sp, sizeof(T), nr, w)) {
        const LevelArgs a0 = stage_level_args(mf, sp, kv.second[0].first, kv.second[0].second, nullptr);
        const auto cand = sweep_candidates(a0, w == 0, sizeof(T), nr);
        most = std::max(most, (int)cand.size());
        c->tune[kv.first] = enc_sweep(cand[std::min<size_t>(index, cand.size() - 1)]);
      }
  }
  for (int order = 0; order <= STF_ORDER_CHECKER; ++order) {
    const int bit = order == 0 ? 2 : (2 << order);
    if (!(what & bit)) continue;
    const TuneKey fk = order == 0 ? fuse_key(mf, sizeof(T), nr) : staged_fuse_key(mf, sizeof(T), nr, order);
    c->tune.erase(fk);
    const std::vector<int> opts = fuse_options(c, mf, sizeof(T), nr);
    most = std::max(most, (int)opts.size());
    const int o = opts[std::min<size_t>(index, opts.size() - 1)];
    c->tune[fk] = o < 0 ? TuneEntry{1, -1, 1, 0, 0.0, 0.0} : TuneEntry{1, o / 16, o % 16, 0, 0.0, 0.0};
  }
  return most;
}

// Entries of the front vectors and of the local fields of one right-hand side
// (from the host plan: a set's vec_elems and u_elems), and the bytes of that
// workspace with the local fields at a 256-byte boundary.
void round_workspace_elems(const Plan& pl, int64_t& vec, int64_t& u) {
  vec = 0;
  u = 0;
  for (const SubDesc& s : pl.subs) {
    vec += pl.shapes[s.shape]->vec_entries;
    u += (int64_t)s.nxl * s.nyl;
  }
}
size_t round_workspace_bytes(const Plan& pl, int prec) {
  int64_t vec = 0, u = 0;
  round_workspace_elems(pl, vec, u);
  const size_t es = prec == STF_C64 ? sizeof(float2) : sizeof(double2);
  const size_t a = (size_t)vec * es;
  return ((a + 255) & ~size_t(255)) + (size_t)u * es;
}

template <typename T>
void sweep_problem(stf_problem pb, const RhsSet& r, int order) {
  Mf& mf = *pb->mf;
  const SweepPlan& sp = sweep_plan(mf, order, pb->ctx->stream);
  if (mf.ws_nr < r.nr) {
    mf.vec.alloc((size_t)mf.vec_elems * sizeof(T) * r.nr);
    mf.u.alloc((size_t)mf.u_elems * sizeof(T) * r.nr);
    mf.ws_nr = r.nr;
  }
  pb->ksr.alloc((size_t)pb->N * sizeof(double2) * r.nr);
  const int code = staged_fuse_for(pb->ctx, mf, sp, sizeof(T), r.nr, order, true);
  sweep_launch<T>(pb->ctx, mf, sp, r, mf.vec.as<T>(), mf.u.as<T>(), pb->keps.as<double2>(),
                  pb->gcoef.as<double2>(), pb->ksr.as<double2>(), pb->N, true, nullptr, code);
}

// One preconditioner application for the right-hand sides of r in `order`.
void precond_set(stf_problem pb, const RhsSet& r, int order = STF_ORDER_ADDITIVE) {
  if (order != STF_ORDER_ADDITIVE) {
    if (pb->prec == STF_C64)
      sweep_problem<float2>(pb, r, order);
    else
      sweep_problem<double2>(pb, r, order);
    return;
  }
  if (pb->prec == STF_C64)
    precond_mf<float2>(pb->ctx, *pb->mf, r);
  else
    precond_mf<double2>(pb->ctx, *pb->mf, r);
}

void precond(stf_problem pb, const double2* v, double2* z) {
  RhsSet r;
  r.nr = 1;
  r.v[0] = v;
  r.z[0] = z;
  precond_set(pb, r);
}

void residual(stf_problem pb, const double2* x, const double2* b, double2* r, double* dst);

// `rounds` source-transfer rounds: z = B v, then z += B (v - A z).
void precond_rounds(stf_problem pb, const double2* v, double2* z, int rounds) {
  precond(pb, v, z);
  for (int r = 1; r < rounds; ++r) {
    double2* t = pb->kt.as<double2>();
    double2* t2 = pb->kt2.as<double2>();
    residual(pb, z, v, t, pb->scal.as<double>() + 7);
    precond(pb, t, t2);
    Timed tm(pb->ctx, K_UPDATE);
    launch_axpy(pb->ctx->stream, z, t2, pb->N);
  }
}

void apply_A(stf_problem pb, const double2* x, double2* y) {
  Timed t(pb->ctx, K_STENCIL);
  launch_stencil(pb->ctx->stream, 0, x, nullptr, y, pb->keps.as<double2>(), pb->cxw(), pb->cxe(),
                 pb->cyw(), pb->cye(), pb->prm.nx, pb->prm.ny, nullptr, nullptr);
}

// r = b - A x; dst receives |r|^2 on device.
void residual(stf_problem pb, const double2* x, const double2* b, double2* r, double* dst) {
  hipStream_t st = pb->ctx->stream;
  int nb = 0;
  {
    Timed t(pb->ctx, K_STENCIL);
    launch_stencil(st, 1, x, b, r, pb->keps.as<double2>(), pb->cxw(), pb->cxe(), pb->cyw(),
                   pb->cye(), pb->prm.nx, pb->prm.ny, pb->partial.as<double>(), &nb);
  }
  launch_reduce_sum(st, pb->partial.as<double>(), nb, dst);
}

// |v|^2 on device (real part of v^H v).
void norm2(stf_problem pb, const double2* v, double2* dst) {
  hipStream_t st = pb->ctx->stream;
  Timed t(pb->ctx, K_ARNOLDI);
  launch_mdot(st, v, pb->N, 1, v, pb->N, pb->partial.as<double2>(), nullptr, nullptr);
  launch_mdot_reduce(st, pb->partial.as<double2>(), krylov_blocks(pb->N), 1, dst, nullptr);
}

// Krylov storage for nr right-hand sides of cycle length m: per RHS V (m+1
// vectors), Z (m), r, H ((m+1) x m), Givens and least-squares vectors.
void ensure_krylov(stf_problem pb, int m, int nr) {
  if (pb->krylov_m >= m && pb->krylov_nr >= nr) return;
  m = std::max(m, pb->krylov_m);
  nr = std::max(nr, pb->krylov_nr);
  size_t vb = (size_t)pb->N * sizeof(double2);
  pb->kV.alloc(vb * (m + 1) * nr);
  pb->kZ.alloc(vb * m * nr);
  pb->kw.alloc(vb * nr);
  pb->kr.alloc(vb * nr);
  pb->kH.alloc(sizeof(double2) * (m + 1) * m * nr);
  pb->kcs.alloc(sizeof(double) * m * nr);
  pb->ksn.alloc(sizeof(double2) * m * nr);
  pb->kg.alloc(sizeof(double2) * (m + 1) * nr);
  pb->ky.alloc(sizeof(double2) * (m + 1) * nr);
  pb->kh1.alloc(sizeof(double2) * (m + 1) * nr);
  pb->kh2.alloc(sizeof(double2) * (m + 1) * nr);
  pb->scal.alloc(sizeof(double) * 16 * (nr + 1));
  // Gram-Schmidt partials and norm partials, one region per right-hand side.
  int nblk = krylov_blocks(pb->N);
  size_t need = (size_t)nblk * (m + 1) * sizeof(double2);
  const int stride = gs_stride(std::min(m + 1, 32));
  need = std::max(need, (size_t)gs_blocks(pb->N, 32) * stride * sizeof(double2));
  need = (need + 255) & ~size_t(255);
  pb->kpart_stride = (long long)(need / sizeof(double2));
  pb->partial.alloc(std::max<size_t>(pb->partial.bytes, need * nr));
  pb->knpart_stride = std::max(krylov_blocks(pb->N), gs_blocks(pb->N, 32));
  pb->npartial.alloc(std::max<size_t>(pb->npartial.bytes, sizeof(double) * pb->knpart_stride * nr));
  pb->krylov_m = m;
  pb->krylov_nr = nr;
}

// ---------------------------------------------------------------------------
// Learned warm start
// ---------------------------------------------------------------------------
long long nn_param_count(const stf_nn_config& c) {
  const long long W = c.width, M = c.modes;
  return W * c.cin + W + (long long)c.layers * (2 * W * W * 2 * M * M + W * W + W) + 2 * W + 2;
}

void nn_validate(const stf_nn_config& c) {
  STF_REQUIRE(c.n >= 4 && c.n <= 1024, "nn: tile side out of range");
  STF_REQUIRE(c.modes >= 1 && 2 * c.modes <= c.n && c.modes <= 22,
              "nn: modes out of range (2M <= n, M <= 22)");
  STF_REQUIRE(c.layers >= 1 && c.layers <= 16, "nn: layers out of range");
  STF_REQUIRE(c.cin == 3, "nn: three input features");
  STF_REQUIRE(nn_width_supported(c.cin, c.width) && nn_width_supported(c.width, c.width) &&
                  nn_width_supported(c.width, 2),
              "nn: width must be 4, 8, 16 or 32");
  STF_REQUIRE(c.max_batch >= 1 && c.max_batch <= 4096, "nn: max_batch out of range");
}

void nn_setup(stf_nn nn) {
  const stf_nn_config& c = nn->cfg;
  const long long W = c.width, NM = nn->NM();
  nn->np = nn_param_count(c);
  long long o = W * c.cin + W;
  nn->offP = 0;
  nn->offR.assign(c.layers, 0);
  nn->offW.assign(c.layers, 0);
  for (int l = 0; l < c.layers; ++l) {
    nn->offR[l] = o;
    o += 2 * W * W * NM;
    nn->offW[l] = o;
    o += W * W + W;
  }
  nn->offQ = o;
  const size_t pb = (size_t)nn->np * sizeof(float);
  nn->par.alloc(pb);
  nn->wq.alloc(pb);
  nn->grad.alloc(pb);
  nn->am.alloc(pb);
  nn->av.alloc(pb);
  // Twiddle tables (double precision angles, rounded to float).
  const int n = c.n, M = c.modes;
  const double tw = 2.0 * M_PI / n;
  std::vector<float> exT((size_t)n * 2 * M), ainv((size_t)n * 4 * M);
  std::vector<float2> ey((size_t)2 * M * n), exi((size_t)M * n);
  for (int x = 0; x < n; ++x)
    for (int k = 0; k < M; ++k) {
      const double ph = tw * (double)((long long)k * x % n);
      exT[(size_t)x * 2 * M + k] = (float)std::cos(ph);
      exT[(size_t)x * 2 * M + M + k] = (float)-std::sin(ph);
      exi[(size_t)k * n + x] = make_float2((float)std::cos(ph), (float)std::sin(ph));
    }
  for (int a = 0; a < 2 * M; ++a) {
    const long long ky = a < M ? a : n - 2 * M + a;
    for (int y = 0; y < n; ++y) {
      const double ph = tw * (double)(ky * y % n);
      ey[(size_t)a * n + y] = make_float2((float)std::cos(ph), (float)-std::sin(ph));
      ainv[(size_t)y * 4 * M + a] = (float)std::cos(ph);
      ainv[(size_t)y * 4 * M + 2 * M + a] = (float)-std::sin(ph);
    }
  }
  hipStream_t st = nn->ctx->stream;
  upload(nn->exT, exT, st);
  upload(nn->ainv, ainv, st);
  upload(nn->ey, ey, st);
  upload(nn->exi, exi, st);
  HIP_CHECK(hipStreamSynchronize(st));
}

void nn_ensure(stf_nn nn, int B) {
  STF_REQUIRE(B >= 1 && B <= nn->cfg.max_batch, "nn: batch out of range");
  if (nn->cap >= B) return;
  const stf_nn_config& c = nn->cfg;
  const int L = c.layers, W = c.width, M = c.modes;
  const size_t act = (size_t)B * W * nn->npix() * sizeof(float);
  const size_t spec = (size_t)B * W * nn->NM() * sizeof(float2);
  nn->h = std::vector<DBuf>(L + 1);
  nn->pre = std::vector<DBuf>(L);
  nn->H = std::vector<DBuf>(L);
  for (auto& d : nn->h) d.alloc(act);
  for (auto& d : nn->pre) d.alloc(act);
  for (auto& d : nn->H) d.alloc(spec);
  nn->T.alloc((size_t)B * W * c.n * 2 * M * sizeof(float));
  nn->G.alloc(spec);
  nn->dG.alloc(spec);
  nn->dH.alloc(spec);
  nn->S.alloc((size_t)B * W * 4 * M * c.n * sizeof(float));
  nn->g.alloc(act);
  nn->dh.alloc(act);
  nn->dh2.alloc(act);
  nn->dpre.alloc(act);
  nn->y.alloc((size_t)B * 2 * nn->npix() * sizeof(float));
  nn->dy.alloc((size_t)B * 2 * nn->npix() * sizeof(float));
  nn->pwpart.alloc((size_t)nn_pw_bwd_blocks() * (W * W + W + 8) * sizeof(float));
  nn->lpart.alloc((size_t)nn_loss_blocks() * B * 2 * sizeof(double));
  nn->den.alloc((size_t)B * sizeof(double));
  nn->loss.alloc(sizeof(double));
  nn->cap = B;
}

// y = network(f); with keep, the pre-activations are kept for nn_backward.
void nn_forward(stf_nn nn, int B, const float* f, float* y, bool keep = true) {
  const stf_nn_config& c = nn->cfg;
  hipStream_t st = nn->ctx->stream;
  Timed t(nn->ctx, K_NN);
  const int n = c.n, W = c.width, M = c.modes, L = c.layers, NM = nn->NM();
  const long long npix = nn->npix();
  const float* P = nn->wq.as<float>();              // the BF16 weights
  float* h0 = nn->h[0].as<float>();
  nn_pw_fwd(st, c.cin, W, false, f, P + nn->offP, P + nn->offP + W * c.cin, nullptr, npix, B,
            nullptr, h0);
  for (int l = 0; l < L; ++l) {
    const float* hl = nn->h[l].as<float>();
    float* T = nn->T.as<float>();
    // T = h_l (B W n rows x n) [cos | -sin]: the x transform of every row.
    nn_gemm(st, 1, B * W * n, 2 * M, n, hl, 0, n, 1, nn->exT.as<float>(), 0, 2 * M, 1, T, 0, 2 * M,
            1, 1.0f, 0.0f);
    float2* Hl = nn->H[l].as<float2>();
    nn_dft_y(st, T, nn->ey.as<float2>(), B * W, n, M, false, Hl);
    const float* Rre = P + nn->offR[l];
    nn_mix_fwd(st, Hl, Rre, Rre + (long long)W * W * NM, B, W, NM, nn->G.as<float2>());
    const float* Wl = P + nn->offW[l];
    if (!keep && nn_spec_pw_ok(n, M, W)) {
      // Inference: the x-inverse rows, then the y inverse transform fused with
      // the pointwise part (the spectral branch is not stored).
      float* S = nn->S.as<float>();
      nn_spec_rows(st, nn->G.as<float2>(), nn->exi.as<float2>(), B * W, n, M, S);
      nn_spec_pw(st, S, nn->ainv.as<float>(), 1.0f / ((float)n * (float)n), hl, Wl, Wl + W * W, npix, B, n,
                 M, W, l < L - 1, nn->h[l + 1].as<float>());
      continue;
    }
    // g_plane = n^-2 [cos | -sin] (n x 4M) [Re S; Im S] (4M x n)
    if (nn_spec_inv_ok(n, M)) {
      nn_spec_inv(st, nn->G.as<float2>(), nn->exi.as<float2>(), B * W, n, M, true, nn->ainv.as<float>(),
                  1.0f / ((float)n * (float)n), 0.0f, nn->g.as<float>(), npix);
    } else {
      float* S = nn->S.as<float>();
      nn_dft_x_inv(st, nn->G.as<float2>(), nn->exi.as<float2>(), B * W, n, M, true, S);
      nn_gemm(st, B * W, n, n, 4 * M, nn->ainv.as<float>(), 0, 4 * M, 1, S, 4LL * M * n, n, 1,
              nn->g.as<float>(), npix, n, 1, 1.0f / ((float)n * (float)n), 0.0f);
    }
    nn_pw_fwd(st, W, W, l < L - 1, hl, Wl, Wl + W * W, nn->g.as<float>(), npix, B,
              keep ? nn->pre[l].as<float>() : nullptr, nn->h[l + 1].as<float>());
  }
  nn_pw_fwd(st, W, 2, false, nn->h[L].as<float>(), P + nn->offQ, P + nn->offQ + 2 * W, nullptr,
            npix, B, nullptr, y);
}

// Parameter gradient of the loss (dL/dy = dy) into nn->grad.
void nn_backward(stf_nn nn, int B, const float* f, const float* dy) {
  const stf_nn_config& c = nn->cfg;
  hipStream_t st = nn->ctx->stream;
  Timed t(nn->ctx, K_NN);
  const int n = c.n, W = c.width, M = c.modes, L = c.layers, NM = nn->NM();
  const long long npix = nn->npix();
  const float* P = nn->wq.as<float>();              // gradients at the BF16 weights
  float* Gd = nn->grad.as<float>();
  float* part = nn->pwpart.as<float>();
  float* dh = nn->dh.as<float>();
  float* dh2 = nn->dh2.as<float>();
  nn_pw_bwd(st, W, 2, false, dy, nullptr, nn->h[L].as<float>(), P + nn->offQ, npix, B, nullptr, dh,
            part, Gd + nn->offQ);
  for (int l = L - 1; l >= 0; --l) {
    const float* Wl = P + nn->offW[l];
    float* dpre = nn->dpre.as<float>();
    nn_pw_bwd(st, W, W, l < L - 1, dh, nn->pre[l].as<float>(), nn->h[l].as<float>(), Wl, npix, B,
              dpre, dh2, part, Gd + nn->offW[l]);
    float* T = nn->T.as<float>();
    nn_gemm(st, 1, B * W * n, 2 * M, n, dpre, 0, n, 1, nn->exT.as<float>(), 0, 2 * M, 1, T, 0, 2 * M,
            1, 1.0f, 0.0f);
    nn_dft_y(st, T, nn->ey.as<float2>(), B * W, n, M, true, nn->dG.as<float2>());
    const float* Rre = P + nn->offR[l];
    const long long rs = (long long)W * W * NM;
    nn_mix_bwd(st, nn->H[l].as<float2>(), nn->dG.as<float2>(), Rre, Rre + rs, B, W, NM,
               nn->dH.as<float2>(), Gd + nn->offR[l], Gd + nn->offR[l] + rs);
    if (nn_spec_inv_ok(n, M)) {
      nn_spec_inv(st, nn->dH.as<float2>(), nn->exi.as<float2>(), B * W, n, M, false, nn->ainv.as<float>(),
                  1.0f, 1.0f, dh2, npix);
    } else {
      float* S = nn->S.as<float>();
      nn_dft_x_inv(st, nn->dH.as<float2>(), nn->exi.as<float2>(), B * W, n, M, false, S);
      nn_gemm(st, B * W, n, n, 4 * M, nn->ainv.as<float>(), 0, 4 * M, 1, S, 4LL * M * n, n, 1, dh2,
              npix, n, 1, 1.0f, 1.0f);
    }
    std::swap(dh, dh2);
  }
  nn_pw_bwd(st, c.cin, W, false, dh, nullptr, f, P + nn->offP, npix, B, nullptr, nullptr, part,
            Gd + nn->offP);
}

double nn_loss_grad(stf_nn nn, int B, const float* f, const float* t) {
  nn_ensure(nn, B);
  hipStream_t st = nn->ctx->stream;
  nn_forward(nn, B, f, nn->y.as<float>());
  {
    Timed tm(nn->ctx, K_NN);
    nn_loss(st, nn->y.as<float>(), t, 2 * nn->npix(), B, nn->lpart.as<double>(), nn->den.as<double>(),
            nn->loss.as<double>(), nn->dy.as<float>());
  }
  nn_backward(nn, B, f, nn->dy.as<float>());
  double L = 0.0;
  HIP_CHECK(hipMemcpyAsync(&L, nn->loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return L;
}

std::vector<int> nn_origins(int interior, int n) {
  std::vector<int> o;
  for (int v = 0; v + n <= interior; v += n / 2) o.push_back(v);
  if (o.empty() || o.back() != interior - n) o.push_back(interior - n);
  return o;
}

// Tile origins of problem pb for tiles of side n (interior coordinates),
// uploaded to the network's buffers; returns the tile count.
int nn_tiling(stf_problem pb, stf_nn nn, int n) {
  STF_REQUIRE(pb->assembled, "nn: problem not assembled");
  STF_REQUIRE(nn->ctx == pb->ctx, "nn: network and problem on different contexts");
  const stf_params& p = pb->prm;
  const int inx = p.nx - p.pml[0] - p.pml[1], iny = p.ny - p.pml[2] - p.pml[3];
  STF_REQUIRE(inx >= n && iny >= n, "nn: physical interior smaller than one tile");
  hipStream_t st = pb->ctx->stream;
  nn->hoy = nn_origins(iny, n);
  nn->hox = nn_origins(inx, n);
  const int nty = (int)nn->hoy.size(), ntx = (int)nn->hox.size();
  std::vector<int2> org;
  for (int a = 0; a < nty; ++a)
    for (int c2 = 0; c2 < ntx; ++c2) org.push_back(make_int2(nn->hox[c2], nn->hoy[a]));
  upload(nn->org, org, st);
  upload(nn->oy, nn->hoy, st);
  upload(nn->ox, nn->hox, st);
  return nty * ntx;
}

// x0 = blended tile predictions for source b (device).
void nn_initial_guess(stf_problem pb, stf_nn nn, const double2* b, double2* x0) {
  const stf_params& p = pb->prm;
  const int n = nn->cfg.n;
  const int inx = p.nx - p.pml[0] - p.pml[1], iny = p.ny - p.pml[2] - p.pml[3];
  hipStream_t st = pb->ctx->stream;
  const int nt = nn_tiling(pb, nn, n);
  const int nty = (int)nn->hoy.size(), ntx = (int)nn->hox.size();
  const long long per = nn->npix();
  nn->tf.alloc((size_t)nt * 3 * per * sizeof(float));
  nn->tpred.alloc((size_t)nt * 2 * per * sizeof(float));
  {
    Timed t(pb->ctx, K_NN);
    nn_features(st, pb->keps.as<double2>(), b, p.k0 * p.k0, p.nx, p.pml[0], p.pml[2],
                nn->org.as<int2>(), nt, n, nn->tf.as<float>());
  }
  const int bmax = nn->cfg.max_batch;
  nn_ensure(nn, std::min(bmax, nt));
  for (int t0 = 0; t0 < nt; t0 += bmax) {
    const int B = std::min(bmax, nt - t0);
    nn_forward(nn, B, nn->tf.as<float>() + (long long)t0 * 3 * per,
               nn->tpred.as<float>() + (long long)t0 * 2 * per, false);
  }
  Timed t(pb->ctx, K_NN);
  nn_blend(st, nn->tpred.as<float>(), nn->oy.as<int>(), nty, nn->ox.as<int>(), ntx, n, p.pml[0],
           p.pml[2], inx, iny, p.nx, p.ny, x0);
}

// Per right-hand side state of the lockstep FGMRES.  Device scalars sc:
// [0] |b|^2, [2] |r|^2, [3] |w|^2, [4] residual estimate; pinned host hp:
// [0..3] copies of sc, [16..19] |w|^2 and the estimate of
// the last two iterations (written by the Givens step itself through hpd, the
// device address of hp).
struct RhsRun {
  const double2* b = nullptr;
  double2* x = nullptr;
  double2 *V = nullptr, *Z = nullptr, *r = nullptr, *H = nullptr, *g = nullptr, *y = nullptr,
          *sn = nullptr;
  double *cs = nullptr, *sc = nullptr, *hp = nullptr, *hpd = nullptr;
  stf_solve_info* info = nullptr;
  double bnorm = 0.0, rnorm = 0.0, relres_guess = 0.0;
  int used_learned = 0, it = 0, restarts = 0, hlen = 0, k = 0, launched = 0;
  bool started = false;   // the next cycle's start is already enqueued
  bool done = false, stop = false;
  stf_status status = STF_ENOCONV;
  void hist(double v) {
    if (info && info->history && hlen < info->history_cap) info->history[hlen] = v;
    ++hlen;
  }
};

// Right-preconditioned FGMRES(m) for nr <= MAX_RHS right-hand sides in
// lockstep: every iteration applies one source-transfer round to all active
// right-hand sides together (the factors are read once), then runs the
// stencil, the Arnoldi step and the Givens update of each.  Each right-hand
// side keeps its own Krylov basis and stops on its own residual; the
// arithmetic of each equals that of a solo solve.
stf_status fgmres_multi(stf_problem pb, int nr, const double2* const* b, double2* const* x,
                        const stf_solve_opts& o, stf_solve_info* info, bool guess_ready = false) {
  stf_ctx c = pb->ctx;
  hipStream_t st = c->stream;
  const long long N = pb->N;
  const int m = o.restart;
  const int rounds = o.rounds < 1 ? 1 : o.rounds;
  ensure_krylov(pb, m, nr);
  if (rounds > 1) {
    pb->kt.alloc((size_t)N * sizeof(double2));
    pb->kt2.alloc((size_t)N * sizeof(double2));
  }
  double2* w = pb->kw.as<double2>();
  const int nblk = krylov_blocks(N);
  std::vector<RhsRun> R(nr);
  for (int s = 0; s < nr; ++s) {
    RhsRun& q = R[s];
    q.b = b[s];
    q.x = x[s];
    q.V = pb->kV.as<double2>() + (long long)s * (m + 1) * N;
    q.Z = pb->kZ.as<double2>() + (long long)s * m * N;
    q.r = pb->kr.as<double2>() + (long long)s * N;
    q.H = pb->kH.as<double2>() + (long long)s * (m + 1) * m;
    q.g = pb->kg.as<double2>() + (long long)s * (m + 1);
    q.y = pb->ky.as<double2>() + (long long)s * (m + 1);
    q.sn = pb->ksn.as<double2>() + (long long)s * m;
    q.cs = pb->kcs.as<double>() + (long long)s * m;
    q.sc = pb->scal.as<double>() + 16 * (s + 1);
    q.hp = c->pinned + 64 * s;
    q.hpd = c->pinned_dev + 64 * s;
    q.info = info ? info + s : nullptr;
  }
  // Initial guesses and residuals.
  HIP_CHECK(hipEventRecord(pb->ev[2], st));
  for (int s = 0; s < nr; ++s) {
    RhsRun& q = R[s];
    if (o.x0_mode == STF_X0_ZERO) HIP_CHECK(hipMemsetAsync(q.x, 0, N * sizeof(double2), st));
    if (o.x0_mode == STF_X0_LEARNED && !guess_ready) {
      STF_REQUIRE(c->nn, "STF_X0_LEARNED needs a network (stf_ctx_set_nn)");
      HIP_CHECK(hipEventRecord(pb->ev[4 + 2 * s], st));
      nn_initial_guess(pb, c->nn, q.b, q.x);
      HIP_CHECK(hipEventRecord(pb->ev[5 + 2 * s], st));
    }
    norm2(pb, q.b, reinterpret_cast<double2*>(q.sc));     // sc[0] = |b|^2
    residual(pb, q.x, q.b, q.r, q.sc + 2);                // sc[2] = |r|^2
    HIP_CHECK(hipMemcpyAsync(q.hp, q.sc, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIP_CHECK(hipStreamSynchronize(st));
  bool refresh = false;
  for (auto& q : R) {
    q.bnorm = std::sqrt(q.hp[0]);
    q.rnorm = std::sqrt(q.hp[2]);
    q.relres_guess = q.bnorm > 0.0 ? q.rnorm / q.bnorm : 0.0;
    if (o.x0_mode == STF_X0_LEARNED) {
      // Fallback: the zero guess whenever the network's residual is not below |b|.
      if (!(q.rnorm < q.bnorm)) {
        HIP_CHECK(hipMemsetAsync(q.x, 0, N * sizeof(double2), st));
        residual(pb, q.x, q.b, q.r, q.sc + 2);
        HIP_CHECK(hipMemcpyAsync(q.hp + 2, q.sc + 2, sizeof(double), hipMemcpyDeviceToHost, st));
        refresh = true;
      } else {
        q.used_learned = 1;
      }
    }
  }
  if (refresh) {
    HIP_CHECK(hipStreamSynchronize(st));
    for (auto& q : R) q.rnorm = std::sqrt(q.hp[2]);
  }
  for (auto& q : R) {
    if (q.bnorm == 0.0) {
      HIP_CHECK(hipMemsetAsync(q.x, 0, N * sizeof(double2), st));
      q.done = true;
      q.status = STF_OK;
      q.rnorm = 0.0;
      q.relres_guess = 0.0;
      continue;
    }
    if (!std::isfinite(q.rnorm)) throw Error(STF_ENAN, "non-finite initial residual");
    if (o.x0_mode != STF_X0_LEARNED) q.relres_guess = q.rnorm / q.bnorm;
    q.hist(q.rnorm / q.bnorm);
  }

  auto launch_iter = [&](int j, const std::vector<int>& cur) {
    if (rounds == 1) {
      RhsSet rs;
      rs.nr = (int)cur.size();
      for (int i = 0; i < rs.nr; ++i) {
        rs.v[i] = R[cur[i]].V + (long long)j * N;
        rs.z[i] = R[cur[i]].Z + (long long)j * N;
      }
      precond_set(pb, rs, o.order);
    } else {
      for (int s : cur)
        precond_rounds(pb, R[s].V + (long long)j * N, R[s].Z + (long long)j * N, rounds);
    }
    // A z_j, then classical Gram-Schmidt with re-orthogonalisation: h1 = V^H w
    // with |w|^2, w -= V h1 with the new |w|^2; a second pass (gated on the
    // device) when more than half of |w|^2 cancelled.  Every right-hand side
    // has its own w, partials, coefficients and gate; with a basis of at most
    // 32 vectors each pass is one launch for all of them.
    const int nv = j + 1, stride = gs_stride(nv);
    auto wof = [&](int s) { return w + (long long)s * N; };
    auto partof = [&](int s) { return pb->partial.as<double2>() + (long long)s * pb->kpart_stride; };
    auto npartof = [&](int s) { return pb->npartial.as<double>() + (long long)s * pb->knpart_stride; };
    auto gateof = [&](int s) { return pb->flag.as<int>() + 4 + s; };
    auto h1of = [&](int s) { return pb->kh1.as<double2>() + (long long)s * (m + 1); };
    auto h2of = [&](int s) { return pb->kh2.as<double2>() + (long long)s * (m + 1); };
    const int nc = (int)cur.size();
    {
      StencilSet sa;
      for (int i = 0; i < nc; ++i) {
        sa.x[i] = R[cur[i]].Z + (long long)j * N;
        sa.y[i] = wof(cur[i]);
      }
      Timed t(c, K_STENCIL);
      launch_stencil_set(st, nc, sa, pb->keps.as<double2>(), pb->cxw(), pb->cxe(), pb->cyw(), pb->cye(),
                         pb->prm.nx, pb->prm.ny);
    }
    {
      Timed t(c, K_ARNOLDI);
      if (stride > 0) {
        // The first pass's update and the second pass's products share one
        // read of the basis (the products are discarded when the gate stays
        // closed).  The second update writes v_{j+1} itself, normalised by
        // |w|^2 = |w1|^2 - |h2|^2 (kept in sc[8]); the Givens step adds h2 to
        // the column.  With the gate closed, the scale below makes v_{j+1}.
        const int gb = gs_blocks(N, nv);
        GsSet ga;
        GsRedSet ra;
        for (int i = 0; i < nc; ++i) {
          const int s = cur[i];
          ga.V[i] = R[s].V;
          ga.w[i] = wof(s);
          ga.partial[i] = partof(s);
          ga.npart[i] = npartof(s);
          ra.partial[i] = partof(s);
          ra.npart[i] = npartof(s);
        }
        launch_gs_set(st, GS_DOT, nc, ga, N, nv, N);
        for (int i = 0; i < nc; ++i) {
          ra.h[i] = h1of(cur[i]);
          ra.out[i] = R[cur[i]].sc + 6;
        }
        launch_gs_reduce_set(st, nc, ra, gb, stride, nv);
        for (int i = 0; i < nc; ++i) ga.h[i] = h1of(cur[i]);
        launch_gs_set(st, GS_UPDATE_DOT, nc, ga, N, nv, N);
        for (int i = 0; i < nc; ++i) {
          const int s = cur[i];
          ra.h[i] = h2of(s);
          ra.out[i] = R[s].sc + 3;
          ra.ref[i] = R[s].sc + 6;
          ra.gate[i] = gateof(s);
        }
        launch_gs_reduce_set(st, nc, ra, gb, stride, nv);
        for (int i = 0; i < nc; ++i) {
          const int s = cur[i];
          ga.h[i] = h2of(s);
          ga.gate[i] = gateof(s);
          ga.vout[i] = R[s].V + (long long)(j + 1) * N;
          ga.nrm_in[i] = R[s].sc + 3;
          ga.nrm_out[i] = R[s].sc + 8;
        }
        launch_gs_set(st, GS_UPDATE_NORMALIZE, nc, ga, N, nv, N);
      } else {
        for (int s : cur) {
          RhsRun& q = R[s];
          double2* part = partof(s);
          double* npart = npartof(s);
          int* gate = gateof(s);
          double2* h1 = h1of(s);
          double2* h2 = h2of(s);
          double2* ws = wof(s);
          launch_mdot(st, q.V, N, nv, ws, N, part, npart, nullptr);
          launch_mdot_reduce(st, part, nblk, nv, h1, nullptr);
          launch_norm_reduce(st, npart, nblk, q.sc + 6, nullptr, nullptr, 0);
          launch_mupdate(st, q.V, N, nv, h1, ws, N, npart, nullptr);
          launch_norm_reduce(st, npart, nblk, q.sc + 3, q.sc + 6, gate, 1);
          launch_mdot(st, q.V, N, nv, ws, N, part, nullptr, gate);
          launch_mdot_reduce(st, part, nblk, nv, h2, gate);
          launch_mupdate(st, q.V, N, nv, h2, ws, N, npart, gate);
          launch_norm_reduce(st, npart, nblk, q.sc + 3, nullptr, gate, 0);
          launch_hacc(st, h1, h2, nv, gate);
        }
      }
    }
    {
      Timed t(c, K_UPDATE);
      const bool reg = stride > 0;
      GivensSet gv;
      for (int i = 0; i < nc; ++i) {
        const int s = cur[i];
        RhsRun& q = R[s];
        gv.w[i] = wof(s);
        gv.v[i] = q.V + (long long)(j + 1) * N;
        gv.H[i] = q.H;
        gv.h[i] = h1of(s);
        gv.wnorm2[i] = q.sc + 3;
        gv.cs[i] = q.cs;
        gv.sn[i] = q.sn;
        gv.g[i] = q.g;
        gv.est[i] = q.sc + 4;
        gv.h2[i] = reg ? h2of(s) : nullptr;
        gv.gate[i] = reg ? gateof(s) : nullptr;
        gv.wnorm2_alt[i] = reg ? q.sc + 8 : nullptr;
        gv.host_out[i] = q.hpd + 16 + 2 * (j & 1);
      }
      launch_scale_givens_set(st, nc, gv, N, j, m + 1);
    }
    HIP_CHECK(hipEventRecord(c->iter_ev[j & 1], st));
  };
  // Iteration j's estimate of right-hand side s (after its event); true on
  // convergence or breakdown.
  auto check = [&](RhsRun& q, int j) {
    const double wn = q.hp[16 + 2 * (j & 1)], est = q.hp[17 + 2 * (j & 1)];
    q.hist(est / q.bnorm);
    if (!std::isfinite(est)) throw Error(STF_ENAN, "non-finite residual estimate");
    return est <= o.tol * q.bnorm || wn == 0.0;
  };

  while (true) {
    std::vector<int> active;
    for (int s = 0; s < nr; ++s) {
      RhsRun& q = R[s];
      if (q.done) continue;
      if (q.rnorm <= o.tol * q.bnorm) {
        q.status = STF_OK;
        q.done = true;
      } else if (q.it >= o.max_iter) {
        q.status = STF_ENOCONV;
        q.done = true;
      } else {
        active.push_back(s);
      }
    }
    if (active.empty()) break;
    {
      CycleSet cs;                               // v_0 = r / |r|, g = |r| e_1
      int ns = 0;
      for (int s : active) {
        RhsRun& q = R[s];
        if (!q.started) {
          cs.r[ns] = q.r;
          cs.nrm2[ns] = q.sc + 2;
          cs.v[ns] = q.V;
          cs.gs[ns] = q.g;
          ++ns;
        }
        q.started = false;
        q.stop = false;
        q.k = 0;
        q.launched = 0;
      }
      if (ns > 0) {
        Timed t(c, K_UPDATE);
        launch_cycle_start_set(st, ns, cs, N, m + 1);
      }
    }
    // Iteration j+1 is enqueued before the host waits for iteration j's
    // estimates, so the GPU queue does not drain between iterations.  A right-
    // hand side whose iteration j met the tolerance has its speculative
    // iteration j+1 discarded, so its iterates equal those of the synchronous
    // algorithm.
    std::vector<int> cur = active, prev;
    int last = -1;
    for (int j = 0; j < m && !cur.empty(); ++j) {
      launch_iter(j, cur);
      last = j;
      for (int s : cur) {
        ++R[s].it;
        R[s].launched = j + 1;
      }
      if (!prev.empty()) {
        HIP_CHECK(hipEventSynchronize(c->iter_ev[(j - 1) & 1]));
        for (int s : prev) {
          RhsRun& q = R[s];
          if (q.stop) continue;                  // its iteration j-1 was a discarded one
          if (check(q, j - 1)) {
            q.stop = true;
            q.k = j;
            if (q.launched == j + 1) {
              --q.it;
              q.launched = j;
            }
          }
        }
      }
      prev = cur;
      std::vector<int> nxt;
      for (int s : cur)
        if (!R[s].stop && R[s].it < o.max_iter) nxt.push_back(s);
      cur.swap(nxt);
    }
    // The cycle's length k is fixed by the checks above (the last iteration's
    // own estimate only adds to the history), so the update and the true
    // residual are enqueued before the host waits for that estimate.
    // One launch each for every right-hand side of the cycle: y = R^{-1} g,
    // x += Z y, r = b - A x with |r|^2 on the device and in the pinned host
    // staging (written by the reduction itself).
    {
      CycleSet cs;
      ResidualSet rs;
      const int na = (int)active.size();
      for (int i = 0; i < na; ++i) {
        RhsRun& q = R[active[i]];
        if (!q.stop) q.k = q.launched;
        cs.H[i] = q.H;
        cs.g[i] = q.g;
        cs.y[i] = q.y;
        cs.k[i] = q.k;
        cs.Z[i] = q.Z;
        cs.x[i] = q.x;
        rs.x[i] = q.x;
        rs.b[i] = q.b;
        rs.r[i] = q.r;
        rs.partial[i] = reinterpret_cast<double*>(pb->partial.as<double2>() + (long long)active[i] * pb->kpart_stride);
        rs.out[i] = q.sc + 2;
        rs.host_out[i] = q.hpd + 2;
      }
      {
        Timed t(c, K_UPDATE);
        launch_trisolve_set(st, na, cs, m + 1);
        launch_xupdate_set(st, na, cs, N, N);
      }
      Timed t(c, K_STENCIL);
      launch_residual_set(st, na, rs, pb->keps.as<double2>(), pb->cxw(), pb->cxe(), pb->cyw(), pb->cye(),
                          pb->prm.nx, pb->prm.ny);
    }
    HIP_CHECK(hipEventRecord(c->cycle_ev, st));
    // The next cycle's start needs only device values: enqueued now, it runs
    // while the host reads the true residuals; a right-hand side that has
    // converged or run out of iterations ignores it (it writes v_0 and g only).
    {
      CycleSet cs;
      const int na = (int)active.size();
      for (int i = 0; i < na; ++i) {
        RhsRun& q = R[active[i]];
        cs.r[i] = q.r;
        cs.nrm2[i] = q.sc + 2;
        cs.v[i] = q.V;
        cs.gs[i] = q.g;
        q.started = true;
      }
      Timed t(c, K_UPDATE);
      launch_cycle_start_set(st, na, cs, N, m + 1);
    }
    if (last >= 0) {
      HIP_CHECK(hipEventSynchronize(c->iter_ev[last & 1]));
      for (int s : prev)
        if (!R[s].stop && R[s].launched == last + 1) check(R[s], last);
    }
    HIP_CHECK(hipEventSynchronize(c->cycle_ev));
    for (int s : active) {
      RhsRun& q = R[s];
      q.rnorm = std::sqrt(q.hp[2]);
      ++q.restarts;
      if (!std::isfinite(q.rnorm)) throw Error(STF_ENAN, "non-finite true residual");
    }
  }
  HIP_CHECK(hipEventRecord(pb->ev[3], st));
  HIP_CHECK(hipEventSynchronize(pb->ev[3]));
  const double t_solve = pb->elapsed(2, 3), t_fac = pb->fac_timed ? pb->elapsed(0, 1) : 0.0;
  stf_status worst = STF_OK;
  for (int s = 0; s < nr; ++s) {
    RhsRun& q = R[s];
    if (q.info) {
      stf_solve_info loc{};
      loc.t_factor_ms = t_fac;
      loc.t_solve_ms = t_solve;
      loc.t_nn_ms = o.x0_mode == STF_X0_LEARNED ? pb->elapsed(4 + 2 * s, 5 + 2 * s) : 0.0;
      loc.iters = q.it;
      loc.restarts = q.restarts;
      loc.relres_true = q.bnorm > 0.0 ? q.rnorm / q.bnorm : 0.0;
      loc.relres_x0 = q.relres_guess;
      loc.used_learned = q.used_learned;
      loc.status = q.status;
      loc.history = q.info->history;
      loc.history_cap = q.info->history_cap;
      loc.history_len = std::min(q.hlen, q.info->history_cap);
      *q.info = loc;
    }
    if (q.status != STF_OK && worst == STF_OK) worst = q.status;
  }
  return worst;
}

// ---------------------------------------------------------------------------
// Batched solve: many problems, several right-hand sides each
// ---------------------------------------------------------------------------
//
// All problems of a batch form one multifrontal set (one launch per tree level
// over the fronts of every problem) and every (problem, right-hand side) pair is
// a system of one lockstep FGMRES whose kernels cover all systems per launch.
// Batch vectors hold nslot slots of ntot entries; problem p's nodes are at
// gbase[p] inside each slot, so system s = slot * nprob + p is the segment
// slot * ntot + gbase[p] .. + nx * ny.  One cycle (start, m iterations, update,
// true residuals, status) is captured in a HIP graph and replayed.

constexpr int BATCH_MAX_RESTART = 32;   // register Gram-Schmidt passes (nv <= 32)

}  // namespace

struct BatchState {
  std::vector<uint64_t> key;      // (uid, generation) of every problem, in order
  int prec = STF_C128, nprob = 0;
  std::vector<long long> gbase;   // per problem
  std::vector<long long> npts;    // per problem: nx * ny
  long long ntot = 0;             // entries of one slot
  Mf mf;
  DBuf keps, gc;                  // concatenated k0^2 eps_bar and coupling arrays
  std::vector<int> gc_off;        // per problem
  DBuf flag;
  // Systems of the current shape (nslot slots, cycle length m).
  int nslot = 0, nsys = 0, m = 0, hcap = 0;
  long long T = 0;                // batch vector length: nslot * ntot
  std::vector<SysDev> hsys;
  DBuf sysd, tsys, bsys[4];
  int ntiles = 0, nblk[4] = {0, 0, 0, 0};
  DBuf V, Z, W, R, X, B, RS;      // RS: stage residuals of a staged order
  DBuf H, g, y, h1, h2, cs, sn, sc, act, cyc, kcol, it, rg, pact, hist;
  DBuf part, npart, spart;
  double* status = nullptr;       // pinned, device-visible: 4 doubles per system
  double* status_dev = nullptr;
  hipGraphExec_t graph = nullptr;
  double graph_tol = -1.0;
  int graph_max_iter = -1, graph_order = -1;
  hipEvent_t ev[4] = {};          // [0, 1] factorisation, [2, 3] a slot group's solve
  hipStream_t cap = nullptr;      // capture stream

  ~BatchState() { release_graph(); if (status) (void)hipHostFree(status);
    for (hipEvent_t& e : ev) if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap); }
  void release_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
  }
};

void destroy_batch(BatchState* b) { delete b; }

namespace {

// The batch state for `probs` on context c: reused while the problems and
// their assemblies are the same, else rebuilt.
BatchState& batch_state(stf_ctx c, int nprob, const stf_problem* probs) {
  std::vector<uint64_t> key;
  for (int p = 0; p < nprob; ++p) {
    key.push_back(probs[p]->uid);
    key.push_back(probs[p]->generation);
  }
  if (c->batch && c->batch->key == key) return *c->batch;
  if (c->batch) {
    HIP_CHECK(hipStreamSynchronize(c->stream));
    destroy_batch(c->batch);
    c->batch = nullptr;
  }
  std::unique_ptr<BatchState> b(new BatchState());
  hipStream_t st = c->stream;
  b->key = key;
  b->nprob = nprob;
  b->prec = probs[0]->prec;
  std::vector<const Plan*> plans;
  long long off = 0;
  for (int p = 0; p < nprob; ++p) {
    plans.push_back(&probs[p]->plan);
    b->gbase.push_back(off);
    b->npts.push_back(probs[p]->N);
    off += (probs[p]->N + 63) / 64 * 64;          // segments start on 1 KiB boundaries
  }
  b->ntot = off;
  long long gcn = 0;
  for (int p = 0; p < nprob; ++p) {
    b->gc_off.push_back((int)gcn);
    gcn += 2LL * probs[p]->prm.nx + 2LL * probs[p]->prm.ny;
  }
  STF_REQUIRE(gcn < (1LL << 31), "batch too large for int32 coupling offsets");
  build_mf(b->mf, plans, b->gbase, b->prec, st, b->gc_off);
  b->keps.alloc((size_t)b->ntot * sizeof(double2));
  HIP_CHECK(hipMemsetAsync(b->keps.p, 0, (size_t)b->ntot * sizeof(double2), st));
  b->gc.alloc((size_t)gcn * sizeof(double2));
  for (int p = 0; p < nprob; ++p) {
    HIP_CHECK(hipMemcpyAsync(b->keps.as<double2>() + b->gbase[p], probs[p]->keps.p,
                             (size_t)probs[p]->N * sizeof(double2), hipMemcpyDeviceToDevice, st));
    HIP_CHECK(hipMemcpyAsync(b->gc.as<double2>() + b->gc_off[p], probs[p]->gcoef.p,
                             (size_t)(2 * probs[p]->prm.nx + 2 * probs[p]->prm.ny) * sizeof(double2),
                             hipMemcpyDeviceToDevice, st));
  }
  b->flag.alloc(sizeof(int) * 4);
  for (hipEvent_t& e : b->ev) HIP_CHECK(hipEventCreate(&e));
  HIP_CHECK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  HIP_CHECK(hipStreamSynchronize(st));
  c->batch = b.release();
  return *c->batch;
}

// System tables, block maps and Krylov storage for nslot slots and cycle length m.
void batch_systems(BatchState& b, const int32_t* nrhs, int slot0, int nslot, int m, int hcap,
                   hipStream_t st) {
  const bool same = b.nslot == nslot && b.m == m && b.hcap >= hcap;
  // presence depends on the slot group: always rewrite the table
  const int nsys = nslot * b.nprob;
  std::vector<SysDev> sys(nsys);
  std::vector<int> tsys, bsys[4];
  int ntiles = 0, nblk[4] = {0, 0, 0, 0};
  for (int k = 0; k < nslot; ++k)
    for (int p = 0; p < b.nprob; ++p) {
      const int s = k * b.nprob + p;
      SysDev& d = sys[s];
      d.off = (long long)k * b.ntot + b.gbase[p];
      d.koff = b.gbase[p];
      d.n = (int)b.npts[p];
      d.gc = b.gc_off[p];
      d.present = (slot0 + k) < nrhs[p] ? 1 : 0;
      d.tile0 = ntiles;
      sys[s] = d;
    }
  // grids come from the scatter table of the set (per problem nx, ny)
  std::vector<ScatDev> scat(b.nprob);
  HIP_CHECK(hipMemcpyAsync(scat.data(), b.mf.scat.p, sizeof(ScatDev) * b.nprob, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int s = 0; s < nsys; ++s) {
    SysDev& d = sys[s];
    const ScatDev& g = scat[s % b.nprob];
    d.nx = g.nx;
    d.ny = g.ny;
    d.tile0 = ntiles;
    const int nt = ((d.nx + 63) / 64) * ((d.ny + 3) / 4);
    for (int t = 0; t < nt; ++t) tsys.push_back(s);
    ntiles += nt;
    for (int ci = 0; ci < 4; ++ci) {
      const long long ch = 256LL << ci;
      const int nb = (int)((d.n + ch - 1) / ch);
      d.blk0[ci] = nblk[ci];
      d.nblk[ci] = nb;
      for (int t = 0; t < nb; ++t) bsys[ci].push_back(s);
      nblk[ci] += nb;
    }
  }
  b.hsys = sys;
  b.nsys = nsys;
  b.ntiles = ntiles;
  upload(b.sysd, sys, st);
  upload(b.tsys, tsys, st);
  for (int ci = 0; ci < 4; ++ci) {
    b.nblk[ci] = nblk[ci];
    upload(b.bsys[ci], bsys[ci], st);
  }
  HIP_CHECK(hipStreamSynchronize(st));
  if (same) return;
  b.release_graph();
  b.nslot = nslot;
  b.m = m;
  b.hcap = hcap;
  b.T = (long long)nslot * b.ntot;
  const size_t vb = (size_t)b.T * sizeof(double2);
  b.V.alloc(vb * (m + 1));
  b.Z.alloc(vb * m);
  b.RS.alloc(vb);
  b.W.alloc(vb);
  b.R.alloc(vb);
  b.X.alloc(vb);
  b.B.alloc(vb);
  for (DBuf* d : {&b.V, &b.Z, &b.W, &b.R, &b.X, &b.B, &b.RS})
    HIP_CHECK(hipMemsetAsync(d->p, 0, d->bytes, st));
  const int hs = m + 1;
  b.H.alloc(sizeof(double2) * hs * m * nsys);
  b.g.alloc(sizeof(double2) * hs * nsys);
  b.y.alloc(sizeof(double2) * hs * nsys);
  b.h1.alloc(sizeof(double2) * hs * nsys);
  b.h2.alloc(sizeof(double2) * hs * nsys);
  b.cs.alloc(sizeof(double) * m * nsys);
  b.sn.alloc(sizeof(double2) * m * nsys);
  b.sc.alloc(sizeof(double) * 16 * nsys);
  for (DBuf* d : {&b.act, &b.cyc, &b.kcol, &b.it, &b.rg}) d->alloc(sizeof(int) * nsys);
  b.pact.alloc(sizeof(int) * b.nprob);
  b.hist.alloc(sizeof(double) * (size_t)hcap * nsys);
  const int maxblk = std::max({nblk[0], nblk[1], nblk[2], nblk[3], ntiles});
  b.part.alloc(sizeof(double) * 64 * (size_t)std::max(1, maxblk));
  b.npart.alloc(sizeof(double) * (size_t)std::max(1, maxblk));
  b.spart.alloc(sizeof(double) * (size_t)std::max(1, ntiles));
  if (b.status) (void)hipHostFree(b.status);
  b.status = nullptr;
  HIP_CHECK(hipHostMalloc((void**)&b.status, sizeof(double) * 4 * nsys, hipHostMallocCoherent));
  HIP_CHECK(hipHostGetDevicePointer((void**)&b.status_dev, b.status, 0));
  HIP_CHECK(hipStreamSynchronize(st));
}

// r = b - A x per system with |r|^2 into sc[s][dst] (gated).
void batch_residual(stf_ctx c, BatchState& b, const int* gate, int dst) {
  hipStream_t st = c->stream;
  launch_bstencil(st, 1, b.X.as<double2>(), b.B.as<double2>(), b.R.as<double2>(),
                  b.keps.as<double2>(), b.gc.as<double2>(), b.sysd.as<SysDev>(), b.tsys.as<int>(),
                  b.ntiles, gate, b.spart.as<double>());
  launch_bsum(st, b.spart.as<double>(), b.sysd.as<SysDev>(), b.nsys, -1, gate, b.sc.as<double>(), dst);
}

// One FGMRES cycle for every system, enqueued on c->stream: start (device
// decision), m iterations gated by act, update and true residual of the
// systems of the cycle, status to pinned host memory.
template <typename T>
void batch_cycle(stf_ctx c, BatchState& b, double tol, int max_iter, int order) {
  hipStream_t st = c->stream;
  const int m = b.m, hs = m + 1, nsys = b.nsys;
  const SysDev* sys = b.sysd.as<SysDev>();
  const int* bs3 = b.bsys[3].as<int>();
  double2* V = b.V.as<double2>();
  double2* Z = b.Z.as<double2>();
  double2* W = b.W.as<double2>();
  double* sc = b.sc.as<double>();
  int* act = b.act.as<int>();
  int* cyc = b.cyc.as<int>();
  int* rg = b.rg.as<int>();
  const long long Tn = b.T;
  launch_bcycle_start(st, b.R.as<double2>(), V, sys, bs3, b.nblk[3], nsys, sc, b.g.as<double2>(), hs,
                      act, cyc, b.kcol.as<int>(), b.it.as<int>(), tol, max_iter);
  launch_bpact(st, act, b.nslot, b.nprob, b.pact.as<int>());
  for (int j = 0; j < m; ++j) {
    RhsSet rs;
    rs.nr = b.nslot;
    for (int k = 0; k < b.nslot; ++k) {
      rs.v[k] = V + (long long)j * Tn + (long long)k * b.ntot;
      rs.z[k] = Z + (long long)j * Tn + (long long)k * b.ntot;
    }
    if (order == STF_ORDER_ADDITIVE) {
      precond_launch<T>(c, b.mf, rs, b.mf.vec.as<T>(), b.mf.u.as<T>(), false, b.pact.as<int>(), 1);
    } else {
      const SweepPlan& sp = sweep_plan(b.mf, order, st);
      const int code = staged_fuse_for(c, b.mf, sp, sizeof(T), rs.nr, order, false);
      sweep_launch<T>(c, b.mf, sp, rs, b.mf.vec.as<T>(), b.mf.u.as<T>(), b.keps.as<double2>(),
                      b.gc.as<double2>(), b.RS.as<double2>(), b.ntot, false, b.pact.as<int>(), code);
    }
    launch_bstencil(st, 0, Z + (long long)j * Tn, nullptr, W, b.keps.as<double2>(), b.gc.as<double2>(),
                    sys, b.tsys.as<int>(), b.ntiles, act, nullptr);
    // Classical Gram-Schmidt with the device-gated second pass, as in the solo solve.
    const int nv = j + 1, ci = bgs_class(nv);
    const int* bsg = b.bsys[ci].as<int>();
    const int nbg = b.nblk[ci];
    double2* h1 = b.h1.as<double2>();
    double2* h2 = b.h2.as<double2>();
    double* part = b.part.as<double>();
    double* npart = b.npart.as<double>();
    launch_bgs(st, GS_DOT, V, Tn, nv, nullptr, hs, W, sys, bsg, nbg, act, nullptr, part, npart,
               nullptr, sc, 0, 0);
    launch_bgs_reduce(st, part, nv, sys, nsys, act, nullptr, h1, hs, npart, sc, 6, -1, nullptr);
    launch_bgs(st, GS_UPDATE_DOT, V, Tn, nv, h1, hs, W, sys, bsg, nbg, act, nullptr, part, npart,
               nullptr, sc, 0, 0);
    launch_bgs_reduce(st, part, nv, sys, nsys, act, nullptr, h2, hs, npart, sc, 3, 6, rg);
    launch_bgs(st, GS_UPDATE_NORMALIZE, V, Tn, nv, h2, hs, W, sys, bsg, nbg, act, rg, part, npart,
               V + (long long)(j + 1) * Tn, sc, 3, 8);
    launch_bgivens_scale(st, W, V + (long long)(j + 1) * Tn, sys, bs3, b.nblk[3], nsys,
                         b.H.as<double2>(), h1, h2, m, sc, b.cs.as<double>(), b.sn.as<double2>(),
                         b.g.as<double2>(), j, act, rg, b.kcol.as<int>(), b.it.as<int>(),
                         b.hist.as<double>(), b.hcap, tol, max_iter);
    launch_bpact(st, act, b.nslot, b.nprob, b.pact.as<int>());
  }
  launch_btrisolve(st, b.H.as<double2>(), m, b.g.as<double2>(), b.y.as<double2>(), b.kcol.as<int>(),
                   cyc, nsys);
  launch_bxupdate(st, Z, Tn, b.y.as<double2>(), hs, b.X.as<double2>(), sys, bs3, b.nblk[3],
                  b.kcol.as<int>(), cyc);
  batch_residual(c, b, cyc, 2);
  launch_bstatus(st, sc, b.it.as<int>(), cyc, nsys, b.status_dev);
}

// The cycle as a HIP graph (captured on the batch's own stream, replayed on the
// context stream); rebuilt when the systems, m, tol or max_iter change.
template <typename T>
void batch_run_cycle(stf_ctx c, BatchState& b, double tol, int max_iter, int order, bool use_graph) {
  if (order != STF_ORDER_ADDITIVE) {                  // tables built outside a capture
    const SweepPlan& sp = sweep_plan(b.mf, order, c->stream);
    (void)staged_fuse_for(c, b.mf, sp, sizeof(T), b.nslot, order, true);
  } else {
    fuse_prepare(c, b.mf);
  }
  if (!use_graph) {
    batch_cycle<T>(c, b, tol, max_iter, order);
    return;
  }
  if (!b.graph || b.graph_tol != tol || b.graph_max_iter != max_iter || b.graph_order != order) {
    b.release_graph();
    hipStream_t keep = c->stream;
    c->stream = b.cap;
    hipGraph_t gr = nullptr;
    HIP_CHECK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeRelaxed));
    try {
      batch_cycle<T>(c, b, tol, max_iter, order);
    } catch (...) {
      (void)hipStreamEndCapture(b.cap, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      c->stream = keep;
      throw;
    }
    c->stream = keep;
    HIP_CHECK(hipStreamEndCapture(b.cap, &gr));
    const hipError_t e = hipGraphInstantiate(&b.graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIP_CHECK(e);
    b.graph_tol = tol;
    b.graph_max_iter = max_iter;
    b.graph_order = order;
  }
  HIP_CHECK(hipGraphLaunch(b.graph, c->stream));
}

bool batch_use_graph() {
  const char* e = std::getenv("STF_BATCH_EAGER");
  return !(e && e[0] == '1');
}

template <typename T>
stf_status batch_solve_t(stf_ctx c, int nprob, const stf_problem* probs, const int32_t* nrhs,
                         const double* const* b_in, double* const* x_out, int on_device,
                         const stf_solve_opts& o, stf_solve_info* const* info, bool& perturbed) {
  hipStream_t st = c->stream;
  BatchState& bs = batch_state(c, nprob, probs);
  int maxr = 0;
  for (int p = 0; p < nprob; ++p) maxr = std::max(maxr, (int)nrhs[p]);
  const int m = o.restart;
  int hcap = 2;
  for (int p = 0; p < nprob; ++p)
    if (info && info[p])
      for (int r = 0; r < nrhs[p]; ++r) hcap = std::max(hcap, info[p][r].history_cap);
  hcap = std::min(hcap, o.max_iter + 1);
  // A slot group's systems, workspaces, right-hand sides and initial guesses
  // (zero or the user's) in the batch vectors.
  auto prepare = [&](int slot0, int nslot) {
    batch_systems(bs, nrhs, slot0, nslot, m, hcap, st);
    if (bs.mf.ws_nr < nslot) {
      const size_t es = sizeof(T);
      bs.mf.vec.alloc((size_t)bs.mf.vec_elems * es * nslot);
      bs.mf.u.alloc((size_t)bs.mf.u_elems * es * nslot);
      bs.mf.ws_nr = nslot;
    }
    const size_t vb = (size_t)bs.T * sizeof(double2);
    HIP_CHECK(hipMemsetAsync(bs.B.p, 0, vb, st));
    HIP_CHECK(hipMemsetAsync(bs.X.p, 0, vb, st));
    const hipMemcpyKind hk = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int k = 0; k < nslot; ++k)
      for (int p = 0; p < nprob; ++p) {
        const int r = slot0 + k;
        if (r >= nrhs[p]) continue;
        const size_t n = (size_t)bs.npts[p];
        const long long off = (long long)k * bs.ntot + bs.gbase[p];
        HIP_CHECK(hipMemcpyAsync(bs.B.as<double2>() + off, b_in[p] + 2 * n * r, n * sizeof(double2),
                                 hk, st));
        if (o.x0_mode == STF_X0_USER)
          HIP_CHECK(hipMemcpyAsync(bs.X.as<double2>() + off, x_out[p] + 2 * n * r,
                                   n * sizeof(double2), hk, st));
      }
  };
  // The network's guesses of a slot group (system s of problem s % nprob in
  // slot s / nprob), bracketed by that problem's events of the slot.
  auto guesses = [&] {
    for (int s = 0; s < bs.nsys; ++s) {
      if (!bs.hsys[s].present) continue;
      const int p = s % nprob, k = s / nprob;
      HIP_CHECK(hipEventRecord(probs[p]->ev[4 + 2 * k], c->stream));
      nn_initial_guess(probs[p], c->nn, bs.B.as<double2>() + bs.hsys[s].off,
                       bs.X.as<double2>() + bs.hsys[s].off);
      HIP_CHECK(hipEventRecord(probs[p]->ev[5 + 2 * k], c->stream));
    }
  };
  if (o.x0_mode == STF_X0_LEARNED) STF_REQUIRE(c->nn, "STF_X0_LEARNED needs a network (stf_ctx_set_nn)");
  // With one slot group, its guesses run on the side stream beside the whole
  // factorisation.
  const bool overlap = o.x0_mode == STF_X0_LEARNED && maxr <= MAX_RHS;
  std::unique_ptr<SideStream> side;
  if (overlap) {
    prepare(0, maxr);
    side.reset(new SideStream(c, c->nn->ctx != c ? c->nn->ctx : nullptr));
    side->fork();
    side->run(guesses);
  }
  // Factorisation of every problem, one launch per tree level over all fronts.
  perturbed = factor_mf<T>(c, bs.mf, bs.keps.as<double2>(), bs.flag.as<int>(), false, bs.ev[0],
                           bs.ev[1]) != 0;
  if (overlap) side->join();
  const double t_fac = [&] {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, bs.ev[0], bs.ev[1]) == hipSuccess ? (double)ms : 0.0;
  }();
  stf_status worst = STF_OK;
  const bool graph = batch_use_graph();
  for (int slot0 = 0; slot0 < maxr; slot0 += MAX_RHS) {
    const int nslot = std::min(MAX_RHS, maxr - slot0);
    if (!overlap) prepare(slot0, nslot);
    const int nsys = bs.nsys;
    HIP_CHECK(hipEventRecord(bs.ev[2], st));
    if (o.x0_mode == STF_X0_LEARNED && !overlap) guesses();
    // (the guesses' times are read once the stream has been synchronised below)
    // |b|^2, initial residuals, cleared flags and counters.
    HIP_CHECK(hipMemsetAsync(bs.sc.p, 0, bs.sc.bytes, st));
    HIP_CHECK(hipMemsetAsync(bs.it.p, 0, bs.it.bytes, st));
    launch_bnorm2(st, bs.B.as<double2>(), bs.sysd.as<SysDev>(), bs.bsys[3].as<int>(), bs.nblk[3],
                  bs.npart.as<double>());
    launch_bsum(st, bs.npart.as<double>(), bs.sysd.as<SysDev>(), nsys, 3, nullptr, bs.sc.as<double>(), 0);
    batch_residual(c, bs, nullptr, 2);
    std::vector<double> sch(16 * (size_t)nsys);
    HIP_CHECK(hipMemcpyAsync(sch.data(), bs.sc.p, sizeof(double) * 16 * nsys, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::vector<double> t_nn(nsys, 0.0);
    if (o.x0_mode == STF_X0_LEARNED)
      for (int s = 0; s < nsys; ++s) {
        if (!bs.hsys[s].present) continue;
        const int p = s % nprob, k = s / nprob;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, probs[p]->ev[4 + 2 * k], probs[p]->ev[5 + 2 * k]) == hipSuccess)
          t_nn[s] = ms;
      }
    std::vector<double> bnorm(nsys), rx0(nsys);
    std::vector<int> used(nsys, 0);
    bool refresh = false;
    for (int s = 0; s < nsys; ++s) {
      bnorm[s] = std::sqrt(sch[16 * s]);
      const double rn = std::sqrt(sch[16 * s + 2]);
      if (!std::isfinite(rn)) throw Error(STF_ENAN, "non-finite initial residual");
      rx0[s] = bnorm[s] > 0.0 ? rn / bnorm[s] : 0.0;
      if (o.x0_mode == STF_X0_LEARNED && bs.hsys[s].present) {
        if (!(rn < bnorm[s])) {          // fallback: the zero guess
          HIP_CHECK(hipMemsetAsync(bs.X.as<double2>() + bs.hsys[s].off, 0,
                                   (size_t)bs.hsys[s].n * sizeof(double2), st));
          refresh = true;
        } else {
          used[s] = 1;
        }
      }
    }
    if (refresh) {
      batch_residual(c, bs, nullptr, 2);
      HIP_CHECK(hipMemcpyAsync(sch.data(), bs.sc.p, sizeof(double) * 16 * nsys, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
    std::vector<double> rn2(nsys), itc(nsys, 0.0);
    std::vector<int> restarts(nsys, 0);
    for (int s = 0; s < nsys; ++s) rn2[s] = sch[16 * s + 2];
    auto running = [&](int s) {
      const double rn = std::sqrt(rn2[s]);
      return bs.hsys[s].present && bnorm[s] > 0.0 && rn > o.tol * bnorm[s] && itc[s] < o.max_iter;
    };
    while (true) {
      bool any = false;
      for (int s = 0; s < nsys; ++s) any = any || running(s);
      if (!any) break;
      batch_run_cycle<T>(c, bs, o.tol, o.max_iter, o.order, graph);
      HIP_CHECK(hipStreamSynchronize(st));
      bool progress = false;
      for (int s = 0; s < nsys; ++s) {
        const double* q = bs.status + 4 * s;
        if (q[1] != itc[s]) progress = true;
        if (q[2] != 0.0) restarts[s] += 1;
        rn2[s] = q[0];
        itc[s] = q[1];
        if (q[3] != 0.0 || !std::isfinite(q[0])) throw Error(STF_ENAN, "non-finite residual in a batched solve");
      }
      if (!progress) throw Error(STF_EDEVICE, "internal: a batched FGMRES cycle made no progress");
    }
    HIP_CHECK(hipEventRecord(bs.ev[3], st));
    // Solutions back to the caller, histories and infos.
    const hipMemcpyKind ok = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int s = 0; s < nsys; ++s) {
      if (!bs.hsys[s].present) continue;
      const int p = s % nprob, r = slot0 + s / nprob;
      const size_t n = (size_t)bs.npts[p];
      HIP_CHECK(hipMemcpyAsync(x_out[p] + 2 * n * r, bs.X.as<double2>() + bs.hsys[s].off,
                               n * sizeof(double2), ok, st));
    }
    std::vector<double> hh((size_t)bs.hcap * nsys);
    HIP_CHECK(hipMemcpyAsync(hh.data(), bs.hist.p, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    float ms = 0.f;
    const double t_solve = hipEventElapsedTime(&ms, bs.ev[2], bs.ev[3]) == hipSuccess ? (double)ms : 0.0;
    for (int s = 0; s < nsys; ++s) {
      if (!bs.hsys[s].present) continue;
      const int p = s % nprob, r = slot0 + s / nprob;
      const double rel = bnorm[s] > 0.0 ? std::sqrt(rn2[s]) / bnorm[s] : 0.0;
      const stf_status sst = (bnorm[s] == 0.0 || rel <= o.tol) ? STF_OK : STF_ENOCONV;
      if (sst != STF_OK && worst == STF_OK) worst = sst;
      if (!info || !info[p]) continue;
      stf_solve_info& inf = info[p][r];
      stf_solve_info loc{};
      loc.iters = (int)itc[s];
      loc.restarts = restarts[s];
      loc.status = sst;
      loc.relres_true = rel;
      loc.relres_x0 = rx0[s];
      loc.used_learned = used[s];
      loc.history = inf.history;
      loc.history_cap = inf.history_cap;
      loc.t_factor_ms = t_fac;
      loc.t_solve_ms = t_solve;
      loc.t_nn_ms = t_nn[s];
      const int len = std::min((int)itc[s] + 1, std::min(inf.history_cap, bs.hcap));
      if (inf.history && len > 0) {
        inf.history[0] = bnorm[s] > 0.0 ? std::sqrt(sch[16 * s + 2]) / bnorm[s] : 0.0;
        for (int i = 1; i < len; ++i) inf.history[i] = hh[(size_t)s * bs.hcap + i];
      }
      loc.history_len = inf.history ? std::max(0, len) : 0;
      inf = loc;
    }
  }
  return worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported entry points
// ---------------------------------------------------------------------------


static stf_status solve_impl(stf_problem pb, int32_t nrhs, const double* b, double* x, int on_device,
                      const stf_solve_opts* opts, stf_solve_info* info, bool refactor) {
  if (!pb) return STF_EINVAL;
  stf_status worst = STF_OK;
  bool perturbed = false;
  stf_status s = guard(pb->ctx, [&] {
    STF_REQUIRE(b && x && opts, "null argument");
    STF_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    STF_REQUIRE(opts->restart >= 1 && opts->restart <= 200, "restart out of range");
    STF_REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
    STF_REQUIRE(std::isfinite(opts->tol) && opts->tol >= 0, "tol must be finite and >= 0");
    STF_REQUIRE(opts->x0_mode == STF_X0_ZERO || opts->x0_mode == STF_X0_USER ||
                    opts->x0_mode == STF_X0_LEARNED,
                "x0_mode invalid");
    STF_REQUIRE(opts->rounds >= 0 && opts->rounds <= 8, "rounds out of range");
    STF_REQUIRE(opts->debug_fault == 0 || opts->debug_fault == 1, "debug_fault must be 0 or 1");
    STF_REQUIRE(opts->order >= STF_ORDER_ADDITIVE && opts->order <= STF_ORDER_CHECKER,
                "unknown source-transfer order");
    STF_REQUIRE(opts->rounds <= 1 || opts->order == STF_ORDER_ADDITIVE,
                "several rounds per application need the additive order");
    if (refactor) {
      if (!pb->assembled) throw Error(STF_ESTATE, "factor before assemble");
      const size_t per = (size_t)pb->N * 2;
      require_finite(pb, b, per * nrhs, on_device, "b");
      stf_ctx c = pb->ctx;
      // The network's guesses on the side stream during the factorisation
      // (device arrays, at most MAX_RHS right-hand sides in one group).
      const bool overlap = opts->x0_mode == STF_X0_LEARNED && on_device && nrhs <= MAX_RHS &&
                           opts->rounds <= 1 && opts->debug_fault == 0;
      if (overlap) {
        STF_REQUIRE(c->nn, "STF_X0_LEARNED needs a network (stf_ctx_set_nn)");
        // The guesses run beside the whole factorisation: its network kernels
        // (memory-bound) share the GPU with the leaf levels (bound by their
        // vector instructions and LDS) and fill what the top levels leave idle.
        SideStream side(c, c->nn->ctx != c ? c->nn->ctx : nullptr);
        side.fork();
        side.run([&] {
          for (int i = 0; i < nrhs; ++i) {
            HIP_CHECK(hipEventRecord(pb->ev[4 + 2 * i], c->stream));
            nn_initial_guess(pb, c->nn, reinterpret_cast<const double2*>(b) + (size_t)i * pb->N,
                             reinterpret_cast<double2*>(x) + (size_t)i * pb->N);
            HIP_CHECK(hipEventRecord(pb->ev[5 + 2 * i], c->stream));
          }
        });
        pb->factored = false;
        perturbed = factor_problem(pb) != 0;
        pb->factored = true;
        side.join();
        const double2* bd[MAX_RHS];
        double2* xd[MAX_RHS];
        for (int i = 0; i < nrhs; ++i) {
          bd[i] = reinterpret_cast<const double2*>(b) + (size_t)i * pb->N;
          xd[i] = reinterpret_cast<double2*>(x) + (size_t)i * pb->N;
        }
        worst = fgmres_multi(pb, nrhs, bd, xd, *opts, info, true);
        HIP_CHECK(hipGetLastError());
        return;
      }
      pb->factored = false;
      perturbed = factor_problem(pb) != 0;
      pb->factored = true;
    }
    if (!pb->factored) throw Error(STF_ESTATE, "solve before factor");
    if (opts->debug_fault == 1) {
      perturbed = factor_problem(pb, true) != 0;
      STF_REQUIRE(perturbed, "internal: the planted fault did not reach the pivot perturbation");
    }
    const size_t per = (size_t)pb->N * 2;
    require_finite(pb, b, per * nrhs, on_device, "b");
    if (opts->x0_mode == STF_X0_USER) require_finite(pb, x, per * nrhs, on_device, "x0");
    hipStream_t st = pb->ctx->stream;
    const size_t vb = (size_t)pb->N * sizeof(double2);
    // Right-hand sides go through in groups of up to MAX_RHS (one with
    // several source-transfer rounds per application: those are not batched).
    const int gmax = (opts->rounds > 1) ? 1 : MAX_RHS;
    for (int r0 = 0; r0 < nrhs; r0 += gmax) {
      const int g = std::min(gmax, nrhs - r0);
      const double2* bd[MAX_RHS];
      double2* xd[MAX_RHS];
      if (!on_device) {
        pb->hb.alloc(vb * g);
        pb->hx.alloc(vb * g);
        HIP_CHECK(hipMemcpyAsync(pb->hb.p, b + r0 * per, vb * g, hipMemcpyHostToDevice, st));
        if (opts->x0_mode == STF_X0_USER)
          HIP_CHECK(hipMemcpyAsync(pb->hx.p, x + r0 * per, vb * g, hipMemcpyHostToDevice, st));
      }
      for (int i = 0; i < g; ++i) {
        if (on_device) {
          bd[i] = reinterpret_cast<const double2*>(b) + (size_t)(r0 + i) * pb->N;
          xd[i] = reinterpret_cast<double2*>(x) + (size_t)(r0 + i) * pb->N;
        } else {
          bd[i] = pb->hb.as<double2>() + (size_t)i * pb->N;
          xd[i] = pb->hx.as<double2>() + (size_t)i * pb->N;
        }
      }
      stf_status r = fgmres_multi(pb, g, bd, xd, *opts, info ? info + r0 : nullptr);
      if (!on_device) {
        HIP_CHECK(hipMemcpyAsync(x + r0 * per, pb->hx.p, vb * g, hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
      }
      if (r != STF_OK && worst == STF_OK) worst = r;
    }
    HIP_CHECK(hipGetLastError());
  });
  if (s != STF_OK) return s;
  if (worst == STF_ENOCONV) pb->ctx->last_error = "FGMRES reached max_iter above tol";
  if (worst == STF_OK && perturbed) {
    pb->ctx->last_error = opts->debug_fault == 1 ? "tiny pivot perturbed during factorisation (planted fault)"
                                                 : "tiny pivot perturbed during factorisation";
    return STF_EPIVOT;
  }
  return worst;
}

extern "C" {

stf_status stf_ctx_create(int device, void* hip_stream, stf_ctx* out) {
  if (!out) return STF_EINVAL;
  *out = nullptr;
  stf_ctx c = nullptr;
  try {
    c = new stf_ctx_s();
  } catch (...) {
    return STF_ENOMEM;
  }
  g_noctx_error.clear();
  stf_status s = guard(c, [&] {
    int n = 0;
    HIP_CHECK(hipGetDeviceCount(&n));
    STF_REQUIRE(device >= 0 && device < n, "device index out of range");
    c->device = device;
    HIP_CHECK(hipSetDevice(device));
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIP_CHECK(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    // Coherent: the Givens kernel writes its estimates here, and the host reads
    // them once the iteration's event has completed.
    HIP_CHECK(hipHostMalloc((void**)&c->pinned, 64 * MAX_RHS * sizeof(double), hipHostMallocCoherent));
    HIP_CHECK(hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0));
    for (int e = 0; e < 2; ++e)
      HIP_CHECK(hipEventCreateWithFlags(&c->iter_ev[e], hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&c->cycle_ev, hipEventDisableTiming));
    c->scratch = scratch_address(device);
    hipDeviceProp_t prop;
    HIP_CHECK(hipGetDeviceProperties(&prop, device));
    c->arch = prop.gcnArchName;
    c->arch = c->arch.substr(0, c->arch.find(':'));     // gfx950, without feature flags
  });
  if (s != STF_OK) {
    g_noctx_error = c->last_error;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return s;
  }
  *out = c;
  return STF_OK;
}

void stf_ctx_destroy(stf_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < STF_K_COUNT; ++k)
    for (auto& pr : c->pending[k]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  for (int e = 0; e < 2; ++e)
    if (c->iter_ev[e]) (void)hipEventDestroy(c->iter_ev[e]);
  if (c->cycle_ev) (void)hipEventDestroy(c->cycle_ev);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (int e = 0; e < 2; ++e)
    if (c->side_ev[e]) (void)hipEventDestroy(c->side_ev[e]);
  if (c->pinned) (void)hipHostFree(c->pinned);
  destroy_batch(c->batch);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* stf_last_error(stf_ctx c) {
  if (!c) return g_noctx_error.empty() ? "null context" : g_noctx_error.c_str();
  return c->last_error.c_str();
}

stf_status stf_ctx_set_timing_mask(stf_ctx c, uint32_t mask) {
  if (!c) return STF_EINVAL;
  return guard(c, [&] {
    c->fold();
    for (int k = 0; k < STF_K_COUNT; ++k) {
      c->total_ms[k] = 0.0;
      c->launches[k] = 0;
    }
    c->timing_mask = mask & ((1u << STF_K_COUNT) - 1u);
    c->timing = c->timing_mask != 0;
  });
}

stf_status stf_ctx_set_timing(stf_ctx c, int enable) {
  return stf_ctx_set_timing_mask(c, enable ? (1u << STF_K_COUNT) - 1u : 0u);
}

stf_status stf_ctx_kernel_stats(stf_ctx c, int cls, double* total_ms, int64_t* launches) {
  if (!c) return STF_EINVAL;
  return guard(c, [&] {
    STF_REQUIRE(cls >= 0 && cls < STF_K_COUNT, "kernel class out of range");
    c->fold();
    if (total_ms) *total_ms = c->total_ms[cls];
    if (launches) *launches = c->launches[cls];
  });
}

stf_status stf_plan_query(const stf_params* prm, stf_plan_info* out) {
  if (!prm || !out) return STF_EINVAL;
  try {
    Plan pl = build_plan(*prm, nullptr);
    *out = plan_info(pl);
    return STF_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return STF_EINVAL;
  }
}

stf_status stf_debug_level_shapes(const stf_params* prm, int32_t nrhs, int32_t* nlevels,
                                  int32_t* ncandidates, int32_t* invalid) {
  if (!prm || nrhs < 1 || nrhs > MAX_RHS) return STF_EINVAL;
  try {
    Plan pl = build_plan(*prm, nullptr);
    std::vector<LevelArgs> lv;
    for (const SubDesc& s : pl.subs)
      for (const SymFront& f : pl.shapes[s.shape]->fronts) {
        if ((int)lv.size() <= f.depth) lv.resize(f.depth + 1, LevelArgs{});
        LevelArgs& a = lv[f.depth];
        a.nlevel += 1;
        a.max_m = std::max(a.max_m, f.p + f.q);
        a.max_p = std::max(a.max_p, f.p);
        a.max_pm = std::max(a.max_pm, f.p * (f.p + f.q));
      }
    int cands = 0, bad = 0;
    const size_t elem = prm->front_prec == STF_C64 ? 8 : 16;
    for (const LevelArgs& a : lv) {
      bad += !factor_shape_ok(a, elem, factor_default(a, elem));
      for (const FactorShape& f : factor_candidates(a, elem)) {
        ++cands;
        bad += !factor_shape_ok(a, elem, f);
      }
      for (int w = 0; w < 2; ++w) {
        bad += !sweep_shape_ok(a, w == 0, elem, nrhs, sweep_default(a, w == 0, elem));
        for (const SweepShape& sh : sweep_candidates(a, w == 0, elem, nrhs)) {
          ++cands;
          bad += !sweep_shape_ok(a, w == 0, elem, nrhs, sh);
        }
      }
    }
    if (nlevels) *nlevels = (int32_t)lv.size();
    if (ncandidates) *ncandidates = cands;
    if (invalid) *invalid = bad;
    return STF_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return STF_EINVAL;
  }
}

stf_status stf_debug_local_axes(const stf_params* prm, int32_t k, int32_t* dims, double* cw,
                                double* ce, double* cs, double* cn) {
  if (!prm) return STF_EINVAL;
  try {
    stf_params p = normalized(*prm);
    validate_params(p);
    GlobalAxes g = build_global_axes(p);
    std::vector<SubDesc> subs = build_partition(p, g);
    if (k < 0 || k >= (int)subs.size()) return STF_EINVAL;
    const SubDesc& s = subs[k];
    if (dims) {
      int32_t d[8] = {s.ox0, s.oy0, s.nxl, s.nyl, s.ix0, s.ix1, s.iy0, s.iy1};
      std::memcpy(dims, d, sizeof(d));
    }
    auto put = [](double* dst, const std::vector<cd>& v) {
      if (!dst) return;
      for (size_t i = 0; i < v.size(); ++i) {
        dst[2 * i] = v[i].real();
        dst[2 * i + 1] = v[i].imag();
      }
    };
    put(cw, s.cx.w);
    put(ce, s.cx.e);
    put(cs, s.cy.w);
    put(cn, s.cy.e);
    return STF_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return STF_EINVAL;
  }
}

stf_status stf_problem_create(stf_ctx c, const stf_params* prm, const double* eps_cells,
                              int on_device, stf_problem* out) {
  if (!c) return STF_EINVAL;
  if (!out || !prm || !eps_cells) {
    c->last_error = "null argument";
    return STF_EINVAL;
  }
  *out = nullptr;
  stf_problem pb = nullptr;
  stf_status s = guard(c, [&] {
    pb = new stf_problem_s();
    pb->ctx = c;
    static std::atomic<uint64_t> next_uid{1};
    pb->uid = next_uid.fetch_add(1);
    pb->plan = build_plan(*prm, &c->shapes);
    pb->prm = pb->plan.prm;
    pb->make_events();
    build_device_state(pb);
    assemble_eps(pb, eps_cells, on_device);
  });
  if (s != STF_OK) {
    delete pb;
    return s;
  }
  *out = pb;
  return STF_OK;
}

stf_status stf_assemble(stf_problem pb, const double* eps_cells, int on_device) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(eps_cells != nullptr, "null eps_cells");
    assemble_eps(pb, eps_cells, on_device);
  });
}

stf_status stf_factor(stf_problem pb) {
  if (!pb) return STF_EINVAL;
  int flagged = 0;
  stf_status s = guard(pb->ctx, [&] {
    if (!pb->assembled) throw Error(STF_ESTATE, "factor before assemble");
    flagged = factor_problem(pb);
    pb->factored = true;
  });
  if (s == STF_OK && flagged) {
    pb->ctx->last_error = "tiny pivot perturbed during factorisation";
    return STF_EPIVOT;
  }
  return s;
}

stf_status stf_apply(stf_problem pb, const double* x, double* y, int on_device) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(x && y, "null argument");
    hipStream_t st = pb->ctx->stream;
    size_t vb = (size_t)pb->N * sizeof(double2);
    if (on_device) {
      apply_A(pb, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y));
      HIP_CHECK(hipGetLastError());
      return;
    }
    pb->hb.alloc(vb);
    pb->hx.alloc(vb);
    HIP_CHECK(hipMemcpyAsync(pb->hb.p, x, vb, hipMemcpyHostToDevice, st));
    apply_A(pb, pb->hb.as<double2>(), pb->hx.as<double2>());
    HIP_CHECK(hipMemcpyAsync(y, pb->hx.p, vb, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

stf_status stf_precond_apply(stf_problem pb, const double* v, double* z, int on_device) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(v && z, "null argument");
    if (!pb->factored) throw Error(STF_ESTATE, "precond before factor");
    hipStream_t st = pb->ctx->stream;
    size_t vb = (size_t)pb->N * sizeof(double2);
    if (on_device) {
      precond(pb, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(z));
      HIP_CHECK(hipGetLastError());
      return;
    }
    pb->hb.alloc(vb);
    pb->hx.alloc(vb);
    HIP_CHECK(hipMemcpyAsync(pb->hb.p, v, vb, hipMemcpyHostToDevice, st));
    precond(pb, pb->hb.as<double2>(), pb->hx.as<double2>());
    HIP_CHECK(hipMemcpyAsync(z, pb->hx.p, vb, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

stf_status stf_precond_apply_noalloc(stf_problem pb, const double* v, double* z) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(v && z, "null argument");
    const size_t need = round_workspace_bytes(pb->plan, pb->prec);
    if (need > SCRATCH_BYTES)
      throw Error(STF_EINVAL, "problem needs " + std::to_string(need) +
                                  " bytes of round workspace; the allocation-free round holds at most " +
                                  std::to_string(SCRATCH_BYTES));
    if (!pb->factored || !pb->mf) throw Error(STF_ESTATE, "precond before factor");
    Mf& mf = *pb->mf;
    int64_t ve = 0, ue = 0;
    round_workspace_elems(pb->plan, ve, ue);
    STF_REQUIRE(ve == mf.vec_elems && ue == mf.u_elems, "internal: workspace size mismatch");
    unsigned char* base = static_cast<unsigned char*>(pb->ctx->scratch);
    const size_t es = pb->prec == STF_C64 ? sizeof(float2) : sizeof(double2);
    const size_t voff = ((size_t)mf.vec_elems * es + 255) & ~size_t(255);
    RhsSet r;
    r.nr = 1;
    r.v[0] = reinterpret_cast<const double2*>(v);
    r.z[0] = reinterpret_cast<double2*>(z);
    if (pb->prec == STF_C64)
      precond_launch<float2>(pb->ctx, mf, r, reinterpret_cast<float2*>(base),
                             reinterpret_cast<float2*>(base + voff), false, nullptr, 1);
    else
      precond_launch<double2>(pb->ctx, mf, r, reinterpret_cast<double2*>(base),
                              reinterpret_cast<double2*>(base + voff), false, nullptr, 1);
    HIP_CHECK(hipGetLastError());
  });
}

stf_status stf_stationary_solve(stf_problem pb, const double* b, double* x, int on_device,
                                double tol, int32_t max_rounds, int32_t stop, double* hist,
                                double* hist_energy, int32_t* rounds_out) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(b && x, "null argument");
    STF_REQUIRE(stop == STF_STOP_RESIDUAL || stop == STF_STOP_OVERLAP, "unknown stop rule");
    STF_REQUIRE(max_rounds >= 0 && max_rounds <= 100000, "max_rounds out of range");
    STF_REQUIRE(std::isfinite(tol) && tol >= 0, "tol must be finite and >= 0");
    if (!pb->factored) throw Error(STF_ESTATE, "solve before factor");
    const long long N = pb->N;
    require_finite(pb, b, 2 * (size_t)N, on_device, "b");
    hipStream_t st = pb->ctx->stream;
    const size_t vb = (size_t)N * sizeof(double2);
    const double2* bd = reinterpret_cast<const double2*>(b);
    double2* xd = reinterpret_cast<double2*>(x);
    if (!on_device) {
      pb->hb.alloc(vb);
      pb->hx.alloc(vb);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, b, vb, hipMemcpyHostToDevice, st));
      bd = pb->hb.as<double2>();
      xd = pb->hx.as<double2>();
    }
    pb->kt.alloc(vb);
    pb->kt2.alloc(vb);
    double2* r = pb->kt.as<double2>();
    double2* z = pb->kt2.as<double2>();
    double* sc = pb->scal.as<double>();          // [0..1] |b|^2 (real part), [2] |r|^2, [4] energy
    Mf& mf = *pb->mf;
    DBuf per_sub;
    per_sub.alloc(sizeof(double) * mf.nsub);
    // Eq. (20): the summed norms of the local fields on the overlapping regions
    // of the round just taken (before the next round overwrites them).
    auto energy = [&] {
      if (pb->prec == STF_C64)
        launch_overlap_norm<float2>(st, mf.u.as<float2>(), mf.subs.as<SubDev>(), mf.nsub,
                                    per_sub.as<double>(), sc + 4);
      else
        launch_overlap_norm<double2>(st, mf.u.as<double2>(), mf.subs.as<SubDev>(), mf.nsub,
                                     per_sub.as<double>(), sc + 4);
    };
    double h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    norm2(pb, bd, reinterpret_cast<double2*>(sc));
    precond(pb, bd, xd);                          // x_0 = B b
    energy();
    residual(pb, xd, bd, r, sc + 2);
    HIP_CHECK(hipMemcpyAsync(h, sc, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    const double bn = std::sqrt(h[0]);
    auto rel = [&](double r2) { return bn > 0.0 ? std::sqrt(r2) / bn : std::sqrt(r2); };
    double rr = rel(h[2]);
    const double e0 = h[4];
    double en = e0;
    if (hist) hist[0] = rr;
    if (hist_energy) hist_energy[0] = e0;
    auto done = [&] { return stop == STF_STOP_RESIDUAL ? rr <= tol : en < tol * e0 || e0 == 0.0; };
    int k = 0;
    while (k < max_rounds && !done()) {
      if (!std::isfinite(rr) || !std::isfinite(en)) throw Error(STF_ENAN, "non-finite residual");
      precond(pb, r, z);                          // B (b - A x): the transferred sources
      energy();
      {
        Timed t(pb->ctx, K_UPDATE);
        launch_axpy(st, xd, z, N);                // x <- x + B (b - A x)
      }
      residual(pb, xd, bd, r, sc + 2);
      HIP_CHECK(hipMemcpyAsync(h + 2, sc + 2, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      rr = rel(h[2]);
      en = h[4];
      ++k;
      if (hist) hist[k] = rr;
      if (hist_energy) hist_energy[k] = en;
    }
    if (!on_device) {
      HIP_CHECK(hipMemcpyAsync(x, xd, vb, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
    if (rounds_out) *rounds_out = k;
    if (!std::isfinite(rr)) throw Error(STF_ENAN, "non-finite residual");
    if (!done()) throw Error(STF_ENOCONV, "tolerance not reached in max_rounds rounds");
  });
}

stf_status stf_line_flux(stf_problem pb, const double* e, int on_device, int32_t axis,
                         int32_t index, int32_t lo, int32_t hi, double* out) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(e && out, "null argument");
    const int nx = pb->prm.nx, ny = pb->prm.ny;
    STF_REQUIRE(axis == 0 || axis == 1, "axis must be 0 or 1");
    const int across = axis == 1 ? ny : nx, along = axis == 1 ? nx : ny;
    STF_REQUIRE(index >= 0 && index + 1 < across, "line index out of range");
    STF_REQUIRE(lo >= 0 && lo <= hi && hi <= along, "line range out of range");
    hipStream_t st = pb->ctx->stream;
    const double2* ed = reinterpret_cast<const double2*>(e);
    if (!on_device) {
      const size_t vb = (size_t)pb->N * sizeof(double2);
      pb->hb.alloc(vb);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, e, vb, hipMemcpyHostToDevice, st));
      ed = pb->hb.as<double2>();
    }
    double* d = pb->scal.as<double>() + 3;
    launch_line_flux(st, ed, nx, axis, index, lo, hi, pb->prm.k0, pb->prm.dx, pb->prm.dy, d);
    HIP_CHECK(hipGetLastError());
    double h = 0.0;
    HIP_CHECK(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    *out = h;
  });
}

stf_status stf_rcs(stf_problem pb, const double* e, int on_device, const int32_t* box, int32_t nang,
                   const double* phis, double* sigma, double* F) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(e && box && phis && sigma, "null argument");
    STF_REQUIRE(nang >= 1 && nang <= 1000000, "nang out of range");
    const int nx = pb->prm.nx, ny = pb->prm.ny;
    const int i0 = box[0], i1 = box[1], j0 = box[2], j1 = box[3];
    STF_REQUIRE(i0 >= 0 && i1 > i0 && i1 + 1 < nx && j0 >= 0 && j1 > j0 && j1 + 1 < ny,
                "contour box out of range");
    for (int a = 0; a < nang; ++a) STF_REQUIRE(std::isfinite(phis[a]), "non-finite angle");
    hipStream_t st = pb->ctx->stream;
    const double2* ed = reinterpret_cast<const double2*>(e);
    if (!on_device) {
      const size_t vb = (size_t)pb->N * sizeof(double2);
      pb->hb.alloc(vb);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, e, vb, hipMemcpyHostToDevice, st));
      ed = pb->hb.as<double2>();
    }
    DBuf dph, dF;
    dph.alloc(sizeof(double) * nang);
    dF.alloc(sizeof(double2) * nang);
    HIP_CHECK(hipMemcpyAsync(dph.p, phis, sizeof(double) * nang, hipMemcpyHostToDevice, st));
    launch_far_field(st, ed, nx, i0, i1, j0, j1, pb->prm.dx, pb->prm.dy, pb->prm.k0,
                     dph.as<double>(), nang, dF.as<double2>());
    HIP_CHECK(hipGetLastError());
    std::vector<double2> hF(nang);
    HIP_CHECK(hipMemcpyAsync(hF.data(), dF.p, sizeof(double2) * nang, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int a = 0; a < nang; ++a) {
      sigma[a] = (hF[a].x * hF[a].x + hF[a].y * hF[a].y) / (4.0 * pb->prm.k0);
      if (F) {
        F[2 * a] = hF[a].x;
        F[2 * a + 1] = hF[a].y;
      }
    }
  });
}

stf_status stf_precond_apply_batch(stf_problem pb, int32_t nrhs, const double* v, double* z,
                                   int on_device) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(v && z, "null argument");
    STF_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    if (!pb->factored) throw Error(STF_ESTATE, "precond before factor");
    hipStream_t st = pb->ctx->stream;
    const size_t vb = (size_t)pb->N * sizeof(double2);
    const double2* vd = reinterpret_cast<const double2*>(v);
    double2* zd = reinterpret_cast<double2*>(z);
    if (!on_device) {
      pb->hb.alloc(vb * nrhs);
      pb->hx.alloc(vb * nrhs);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, v, vb * nrhs, hipMemcpyHostToDevice, st));
      vd = pb->hb.as<double2>();
      zd = pb->hx.as<double2>();
    }
    for (int r0 = 0; r0 < nrhs; r0 += MAX_RHS) {
      RhsSet rs;
      rs.nr = std::min(MAX_RHS, nrhs - r0);
      for (int i = 0; i < rs.nr; ++i) {
        rs.v[i] = vd + (size_t)(r0 + i) * pb->N;
        rs.z[i] = zd + (size_t)(r0 + i) * pb->N;
      }
      precond_set(pb, rs);
    }
    HIP_CHECK(hipGetLastError());
    if (!on_device) {
      HIP_CHECK(hipMemcpyAsync(z, pb->hx.p, vb * nrhs, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
  });
}

stf_status stf_sweep_apply(stf_problem pb, int32_t order, const double* v, double* z,
                           int on_device) {
  if (!pb) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(v && z, "null argument");
    STF_REQUIRE(order >= STF_ORDER_ADDITIVE && order <= STF_ORDER_CHECKER,
                "unknown source-transfer order");
    if (!pb->factored) throw Error(STF_ESTATE, "precond before factor");
    hipStream_t st = pb->ctx->stream;
    const size_t vb = (size_t)pb->N * sizeof(double2);
    RhsSet r;
    r.nr = 1;
    if (on_device) {
      r.v[0] = reinterpret_cast<const double2*>(v);
      r.z[0] = reinterpret_cast<double2*>(z);
    } else {
      pb->hb.alloc(vb);
      pb->hx.alloc(vb);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, v, vb, hipMemcpyHostToDevice, st));
      r.v[0] = pb->hb.as<double2>();
      r.z[0] = pb->hx.as<double2>();
    }
    precond_set(pb, r, order);
    HIP_CHECK(hipGetLastError());
    if (!on_device) {
      HIP_CHECK(hipMemcpyAsync(z, pb->hx.p, vb, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
  });
}

stf_status stf_solve(stf_problem pb, int32_t nrhs, const double* b, double* x, int on_device,
                     const stf_solve_opts* opts, stf_solve_info* info) {
  return solve_impl(pb, nrhs, b, x, on_device, opts, info, false);
}

stf_status stf_factor_solve(stf_problem pb, int32_t nrhs, const double* b, double* x, int on_device,
                            const stf_solve_opts* opts, stf_solve_info* info) {
  return solve_impl(pb, nrhs, b, x, on_device, opts, info, true);
}

stf_status stf_batch_solve(stf_ctx ctx, int32_t nprob, const stf_problem* probs,
                           const int32_t* nrhs, const double* const* b, double* const* x,
                           int on_device, const stf_solve_opts* opts, stf_solve_info* const* info) {
  if (!ctx) return STF_EINVAL;
  stf_status worst = STF_OK;
  bool perturbed = false;
  stf_status s = guard(ctx, [&] {
    STF_REQUIRE(nprob >= 1 && probs && nrhs && b && x && opts, "null argument or empty batch");
    STF_REQUIRE(opts->restart >= 1 && opts->restart <= BATCH_MAX_RESTART,
                "batched restart out of range (1..32)");
    STF_REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
    STF_REQUIRE(std::isfinite(opts->tol) && opts->tol >= 0, "tol must be finite and >= 0");
    STF_REQUIRE(opts->x0_mode == STF_X0_ZERO || opts->x0_mode == STF_X0_USER ||
                    opts->x0_mode == STF_X0_LEARNED,
                "x0_mode invalid");
    STF_REQUIRE(opts->rounds <= 1, "a batched solve takes one source-transfer round per application");
    STF_REQUIRE(opts->debug_fault == 0, "debug_fault is not available in a batched solve");
    STF_REQUIRE(opts->order >= STF_ORDER_ADDITIVE && opts->order <= STF_ORDER_CHECKER,
                "unknown source-transfer order");
    for (int p = 0; p < nprob; ++p) {
      STF_REQUIRE(probs[p] && probs[p]->ctx == ctx, "problem missing or on another context");
      STF_REQUIRE(probs[p]->assembled, "problem not assembled");
      STF_REQUIRE(probs[p]->prec == probs[0]->prec, "all problems of a batch need one front precision");
      STF_REQUIRE(nrhs[p] >= 1, "nrhs must be >= 1");
      STF_REQUIRE(b[p] && x[p], "null right-hand side or solution pointer");
      for (int q = 0; q < p; ++q) STF_REQUIRE(probs[q] != probs[p], "a problem appears twice in the batch");
      const size_t per = (size_t)probs[p]->N * 2 * nrhs[p];
      require_finite(probs[p], b[p], per, on_device, "b");
      if (opts->x0_mode == STF_X0_USER) require_finite(probs[p], x[p], per, on_device, "x0");
    }
    worst = probs[0]->prec == STF_C64
                ? batch_solve_t<float2>(ctx, nprob, probs, nrhs, b, x, on_device, *opts, info, perturbed)
                : batch_solve_t<double2>(ctx, nprob, probs, nrhs, b, x, on_device, *opts, info, perturbed);
    HIP_CHECK(hipGetLastError());
  });
  if (s != STF_OK) return s;
  if (worst == STF_ENOCONV) ctx->last_error = "FGMRES reached max_iter above tol";
  if (worst == STF_OK && perturbed) {
    ctx->last_error = "tiny pivot perturbed during factorisation";
    return STF_EPIVOT;
  }
  return worst;
}

stf_status stf_autotune(stf_ctx ctx, int32_t nprob, const stf_problem* probs, int32_t nrhs,
                        int32_t what, int32_t reps, stf_tune_report* report) {
  if (!ctx) return STF_EINVAL;
  if (report) *report = stf_tune_report{0, 0, 0.0, 0.0, -1, 0.0, 0.0};
  return guard(ctx, [&] {
    STF_REQUIRE(nprob >= 1 && probs, "need at least one problem");
    STF_REQUIRE(nrhs >= 1 && nrhs <= MAX_RHS, "1 to 4 right-hand sides per sweep");
    STF_REQUIRE(what >= 1 && what <= 63, "what: bits 1 factorisation, 2 additive sweeps, 4 / 8 / 16 / 32 staged orders");
    STF_REQUIRE(reps >= 1 && reps <= 100, "reps must be 1..100");
    for (int p = 0; p < nprob; ++p) {
      STF_REQUIRE(probs[p] && probs[p]->ctx == ctx, "problem missing or on another context");
      if (!probs[p]->assembled) throw Error(STF_ESTATE, "autotune before assemble");
      STF_REQUIRE(probs[p]->prec == probs[0]->prec, "all problems need one front precision");
      for (int q = 0; q < p; ++q) STF_REQUIRE(probs[q] != probs[p], "a problem appears twice");
    }
    const bool c64 = probs[0]->prec == STF_C64;
    TuneTally tally;
    auto run = [&](Mf& mf, const double2* keps, const double2* gc, int* flag, long long ntot) {
      if (c64) {
        if (what & 1) tune_factor_mf<float2>(ctx, mf, keps, flag, reps, tally);
        factor_mf<float2>(ctx, mf, keps, flag, false, nullptr, nullptr);
        if (what & 2) tune_sweeps_mf<float2>(ctx, mf, nrhs, ntot, reps, tally);
        for (int order = 1; order <= STF_ORDER_CHECKER; ++order)
          if (what & (2 << order)) tune_staged_mf<float2>(ctx, mf, nrhs, ntot, keps, gc, order, reps, tally);
      } else {
        if (what & 1) tune_factor_mf<double2>(ctx, mf, keps, flag, reps, tally);
        factor_mf<double2>(ctx, mf, keps, flag, false, nullptr, nullptr);
        if (what & 2) tune_sweeps_mf<double2>(ctx, mf, nrhs, ntot, reps, tally);
        for (int order = 1; order <= STF_ORDER_CHECKER; ++order)
          if (what & (2 << order)) tune_staged_mf<double2>(ctx, mf, nrhs, ntot, keps, gc, order, reps, tally);
      }
    };
    if (nprob == 1) {
      stf_problem pb = probs[0];
      run(pb->ensure_mf(), pb->keps.as<double2>(), pb->gcoef.as<double2>(), pb->flag.as<int>(), pb->N);
      pb->factored = true;
      pb->fac_timed = false;
    } else {
      BatchState& bs = batch_state(ctx, nprob, probs);
      run(bs.mf, bs.keps.as<double2>(), bs.gc.as<double2>(), bs.flag.as<int>(), bs.ntot);
    }
    // a captured batch cycle holds the shapes of its capture
    if (ctx->batch) ctx->batch->release_graph();
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (report)
      *report = stf_tune_report{tally.levels,     tally.changed,          tally.ms_default,
                                tally.ms_tuned,   tally.fuse_depth,       tally.ms_round_default,
                                tally.ms_round_tuned};
  });
}


stf_status stf_tune_pick(stf_ctx ctx, int32_t nprob, const stf_problem* probs, int32_t nrhs,
                         int32_t what, int32_t index, int32_t* max_candidates) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    STF_REQUIRE(nprob >= 1 && probs, "need at least one problem");
    STF_REQUIRE(nrhs >= 1 && nrhs <= MAX_RHS, "1 to 4 right-hand sides per sweep");
    STF_REQUIRE(what >= 1 && what <= 63, "what: bits 1 factorisation, 2 additive sweeps, 4 / 8 / 16 / 32 staged orders");
    STF_REQUIRE(index >= 0, "candidate index must be >= 0");
    for (int p = 0; p < nprob; ++p) {
      STF_REQUIRE(probs[p] && probs[p]->ctx == ctx, "problem missing or on another context");
      if (!probs[p]->assembled) throw Error(STF_ESTATE, "tune_pick before assemble");
      STF_REQUIRE(probs[p]->prec == probs[0]->prec, "all problems need one front precision");
    }
    Mf* mf = nullptr;
    const double2* keps = nullptr;
    if (nprob == 1) {
      mf = &probs[0]->ensure_mf();
      keps = probs[0]->keps.as<double2>();
    } else {
      BatchState& bs = batch_state(ctx, nprob, probs);
      mf = &bs.mf;
      keps = bs.keps.as<double2>();
    }
    const int most = probs[0]->prec == STF_C64 ? tune_pick_mf<float2>(ctx, *mf, keps, nrhs, what, index)
                                               : tune_pick_mf<double2>(ctx, *mf, keps, nrhs, what, index);
    if (ctx->batch) ctx->batch->release_graph();
    if (max_candidates) *max_candidates = most;
  });
}

stf_status stf_tune_save(stf_ctx ctx, const char* path) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    STF_REQUIRE(path != nullptr, "null path");
    FILE* f = std::fopen(path, "w");
    STF_REQUIRE(f != nullptr, "cannot open the tune file for writing");
    bool ok = std::fprintf(f, "stfdfd-tune 1 %s %zu\n", ctx->arch.c_str(), ctx->tune.size()) > 0;
    for (const auto& kv : ctx->tune) {
      const TuneKey& k = kv.first;
      const TuneEntry& e = kv.second;
      ok = ok && std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %.9g %.9g\n", k.op, k.elem, k.nr, k.nlevel,
                              k.max_m, k.max_p, e.kind, e.a, e.b, e.c, e.ms, e.ms_default) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    STF_REQUIRE(ok, "writing the tune file failed");
  });
}

stf_status stf_tune_load(stf_ctx ctx, const char* path) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    STF_REQUIRE(path != nullptr, "null path");
    FILE* f = std::fopen(path, "r");
    STF_REQUIRE(f != nullptr, "cannot open the tune file");
    std::map<TuneKey, TuneEntry> got;
    char magic[32] = {0}, arch[128] = {0};
    int version = 0;
    long long count = -1;
    bool ok = std::fscanf(f, "%31s %d %127s %lld", magic, &version, arch, &count) == 4 &&
              std::string(magic) == "stfdfd-tune" && version == 1 && count >= 0 && count <= 1000000;
    std::string why = ok ? "" : "not a tune file (bad header)";
    if (ok && ctx->arch != arch) {
      ok = false;
      why = std::string("tune file is for ") + arch + ", this device is " + ctx->arch;
    }
    for (long long i = 0; ok && i < count; ++i) {
      TuneKey k{};
      TuneEntry e{};
      ok = std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %lf %lf", &k.op, &k.elem, &k.nr, &k.nlevel,
                       &k.max_m, &k.max_p, &e.kind, &e.a, &e.b, &e.c, &e.ms, &e.ms_default) == 12;
      ok = ok && k.op >= 0 && k.op <= 3 + STF_ORDER_CHECKER && (k.elem == 8 || k.elem == 16) &&
           (k.op == 0 ? k.nr == 0 : (k.nr >= 1 && k.nr <= MAX_RHS)) && k.nlevel >= 1 &&
           std::isfinite(e.ms) && std::isfinite(e.ms_default);
      if (k.op <= 2)   // a level: its largest front and separator, a launch shape
        ok = ok && k.max_m >= 1 && k.max_p >= 0 && k.max_p <= k.max_m && e.kind >= 1 && e.kind <= 2;
      else             // subtree sweeps of a set, additive or staged order (max_m: deepest
                       // level, max_p: subdomains)
        ok = ok && k.max_m >= 0 && k.max_p >= 1 && e.kind == 1 && e.a >= -1 && e.a < k.max_m &&
             e.b >= 1 && e.b <= 8;
      if (ok) got[k] = e;
      else why = "malformed tune file entry";
    }
    std::fclose(f);
    STF_REQUIRE(ok, why);
    for (const auto& kv : got) ctx->tune[kv.first] = kv.second;
    if (ctx->batch) ctx->batch->release_graph();
  });
}

stf_status stf_tune_clear(stf_ctx ctx) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    ctx->tune.clear();
    if (ctx->batch) ctx->batch->release_graph();
  });
}

int32_t stf_tune_count(stf_ctx ctx) { return ctx ? (int32_t)ctx->tune.size() : -1; }

stf_status stf_tune_entry(stf_ctx ctx, int32_t i, int32_t* key, int32_t* shape, double* ms) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    STF_REQUIRE(i >= 0 && i < (int32_t)ctx->tune.size(), "tune entry index out of range");
    auto it = ctx->tune.begin();
    std::advance(it, i);
    const TuneKey& k = it->first;
    const TuneEntry& e = it->second;
    if (key) {
      const int32_t v[6] = {k.op, k.elem, k.nr, k.nlevel, k.max_m, k.max_p};
      std::copy(v, v + 6, key);
    }
    if (shape) {
      const int32_t v[4] = {e.kind, e.a, e.b, e.c};
      std::copy(v, v + 4, shape);
    }
    if (ms) {
      ms[0] = e.ms;
      ms[1] = e.ms_default;
    }
  });
}

stf_status stf_problem_info(stf_problem pb, stf_plan_info* out) {
  if (!pb || !out) return STF_EINVAL;
  *out = plan_info(pb->plan);
  out->device_bytes = pb->device_bytes();
  return STF_OK;
}

void stf_problem_destroy(stf_problem pb) {
  if (!pb) return;
  (void)hipSetDevice(pb->ctx->device);
  (void)hipStreamSynchronize(pb->ctx->stream);
  delete pb;
}

// ---- learned warm start ------------------------------------------------

int64_t stf_nn_param_count(const stf_nn_config* cfg) {
  if (!cfg) return -1;
  try {
    nn_validate(*cfg);
  } catch (...) {
    return -1;
  }
  return nn_param_count(*cfg);
}

stf_status stf_nn_create(stf_ctx ctx, const stf_nn_config* cfg, const float* params, stf_nn* out) {
  if (!ctx || !out) return STF_EINVAL;
  *out = nullptr;
  stf_nn nn = nullptr;
  stf_status s = guard(ctx, [&] {
    STF_REQUIRE(cfg && params, "null argument");
    nn_validate(*cfg);
    nn = new stf_nn_s();
    nn->ctx = ctx;
    nn->cfg = *cfg;
    nn_setup(nn);
    const size_t pb = (size_t)nn->np * sizeof(float);
    for (long long i = 0; i < nn->np; ++i)
      STF_REQUIRE(std::isfinite(params[i]), "nn: non-finite parameter");
    HIP_CHECK(hipMemcpyAsync(nn->par.p, params, pb, hipMemcpyHostToDevice, ctx->stream));
    nn_quantize_bf16(ctx->stream, nn->par.as<float>(), nn->wq.as<float>(), nn->np);
    HIP_CHECK(hipMemsetAsync(nn->am.p, 0, pb, ctx->stream));
    HIP_CHECK(hipMemsetAsync(nn->av.p, 0, pb, ctx->stream));
    HIP_CHECK(hipMemsetAsync(nn->grad.p, 0, pb, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  });
  if (s != STF_OK) {
    delete nn;
    return s;
  }
  *out = nn;
  return STF_OK;
}

void stf_nn_destroy(stf_nn nn) {
  if (!nn) return;
  (void)hipSetDevice(nn->ctx->device);
  (void)hipStreamSynchronize(nn->ctx->stream);
  if (nn->ctx->nn == nn) nn->ctx->nn = nullptr;
  delete nn;
}

stf_status stf_nn_get_params(stf_nn nn, float* params) {
  if (!nn) return STF_EINVAL;
  return guard(nn->ctx, [&] {
    STF_REQUIRE(params, "null argument");
    HIP_CHECK(hipMemcpyAsync(params, nn->par.p, (size_t)nn->np * sizeof(float),
                             hipMemcpyDeviceToHost, nn->ctx->stream));
    HIP_CHECK(hipStreamSynchronize(nn->ctx->stream));
  });
}

stf_status stf_nn_set_params(stf_nn nn, const float* params) {
  if (!nn) return STF_EINVAL;
  return guard(nn->ctx, [&] {
    STF_REQUIRE(params, "null argument");
    for (long long i = 0; i < nn->np; ++i)
      STF_REQUIRE(std::isfinite(params[i]), "nn: non-finite parameter");
    const size_t pb = (size_t)nn->np * sizeof(float);
    hipStream_t st = nn->ctx->stream;
    HIP_CHECK(hipMemcpyAsync(nn->par.p, params, pb, hipMemcpyHostToDevice, st));
    nn_quantize_bf16(st, nn->par.as<float>(), nn->wq.as<float>(), nn->np);
    HIP_CHECK(hipMemsetAsync(nn->am.p, 0, pb, st));
    HIP_CHECK(hipMemsetAsync(nn->av.p, 0, pb, st));
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

stf_status stf_nn_forward(stf_nn nn, int32_t batch, const float* f, float* y) {
  if (!nn) return STF_EINVAL;
  return guard(nn->ctx, [&] {
    STF_REQUIRE(f && y, "null argument");
    nn_ensure(nn, batch);
    nn_forward(nn, batch, f, y, false);          // inference: no pre-activations kept
    HIP_CHECK(hipGetLastError());
  });
}

stf_status stf_nn_loss_grad(stf_nn nn, int32_t batch, const float* f, const float* t, double* loss,
                            float* grad) {
  if (!nn) return STF_EINVAL;
  return guard(nn->ctx, [&] {
    STF_REQUIRE(f && t && loss, "null argument");
    *loss = nn_loss_grad(nn, batch, f, t);
    STF_REQUIRE(std::isfinite(*loss), "nn: non-finite loss");
    if (grad) {
      HIP_CHECK(hipMemcpyAsync(grad, nn->grad.p, (size_t)nn->np * sizeof(float),
                               hipMemcpyDeviceToHost, nn->ctx->stream));
      HIP_CHECK(hipStreamSynchronize(nn->ctx->stream));
    }
  });
}

stf_status stf_nn_train_step(stf_nn nn, int32_t batch, const float* f, const float* t, double lr,
                             int32_t step, double* loss) {
  if (!nn) return STF_EINVAL;
  return guard(nn->ctx, [&] {
    STF_REQUIRE(f && t && loss, "null argument");
    STF_REQUIRE(step >= 1, "nn: step counts from 1");
    STF_REQUIRE(std::isfinite(lr) && lr > 0, "nn: learning rate must be positive");
    *loss = nn_loss_grad(nn, batch, f, t);
    STF_REQUIRE(std::isfinite(*loss), "nn: non-finite loss");
    Timed tm(nn->ctx, K_NN);
    nn_adam(nn->ctx->stream, nn->par.as<float>(), nn->grad.as<float>(), nn->am.as<float>(),
            nn->av.as<float>(), nn->np, lr, step, 0.9, 0.999, 1e-8, nn->wq.as<float>());
    HIP_CHECK(hipGetLastError());
  });
}

stf_status stf_ctx_set_nn(stf_ctx ctx, stf_nn nn) {
  if (!ctx) return STF_EINVAL;
  return guard(ctx, [&] {
    STF_REQUIRE(!nn || nn->ctx == ctx, "network created on another context");
    ctx->nn = nn;
  });
}

stf_status stf_nn_tile_data(stf_problem pb, stf_nn nn, const double* b, const double* x, float* f,
                            float* t, int32_t* ntiles) {
  if (!pb || !nn) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(ntiles, "null argument");
    const stf_params& p = pb->prm;
    const int n = nn->cfg.n;
    const int nt = nn_tiling(pb, nn, n);
    *ntiles = nt;
    hipStream_t st = pb->ctx->stream;
    if (f) {
      STF_REQUIRE(b, "b is required with f");
      nn_features(st, pb->keps.as<double2>(), reinterpret_cast<const double2*>(b), p.k0 * p.k0,
                  p.nx, p.pml[0], p.pml[2], nn->org.as<int2>(), nt, n, f);
    }
    if (t) {
      STF_REQUIRE(x, "x is required with t");
      nn_fields(st, reinterpret_cast<const double2*>(x), p.nx, p.pml[0], p.pml[2],
                nn->org.as<int2>(), nt, n, t);
    }
    HIP_CHECK(hipGetLastError());
  });
}

stf_status stf_nn_initial_guess(stf_problem pb, stf_nn nn, const double* b, double* x0,
                                int on_device) {
  if (!pb || !nn) return STF_EINVAL;
  return guard(pb->ctx, [&] {
    STF_REQUIRE(b && x0, "null argument");
    const size_t vb = (size_t)pb->N * sizeof(double2);
    hipStream_t st = pb->ctx->stream;
    require_finite(pb, b, (size_t)pb->N * 2, on_device, "b");
    if (on_device) {
      nn_initial_guess(pb, nn, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x0));
    } else {
      pb->hb.alloc(vb);
      pb->hx.alloc(vb);
      HIP_CHECK(hipMemcpyAsync(pb->hb.p, b, vb, hipMemcpyHostToDevice, st));
      nn_initial_guess(pb, nn, pb->hb.as<double2>(), pb->hx.as<double2>());
      HIP_CHECK(hipMemcpyAsync(x0, pb->hx.p, vb, hipMemcpyDeviceToHost, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

}  // extern "C"
