// hsrq_server.cpp -- the serving loop: continuous batching of solve requests.
//
// One worker thread owns the device work.  Requests (a problem with device H
// and X owned by the caller) wait in a FIFO queue and are admitted while the
// HBM budget (workspace + H + X of every admitted request) allows.  Every
// admitted request advances one tile-column step per tick: a tick is one
// launch of the critical kernel and one of the far-tile kernel covering the
// current step of every active request, whatever step each one is at (the
// step travels with each task).  Requests that arrive while others run join
// at the next tick; a request whose steps are done gets its final kernels and
// leaves.  With precision 1 a request runs the FP32-product pass first; its
// FP64 residual check runs when that pass completes, and the failing shifts
// are re-solved by an FP64 child request whose results are scattered over the
// parent's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hsrq.h"
#include "hsrq_common.h"
#include "hsrq_plan.h"

using namespace hsrq;

namespace {

constexpr int kRing = 4;                         // tick array slots in flight
constexpr size_t kTickBytes = size_t(16) << 20;  // device bytes per tick slot

// size classes for pooled buffers: 1/8 steps between powers of two
size_t size_class(size_t b) {
  if (b <= 4096) return 4096;
  size_t p = 1;
  while (p < b) p <<= 1;
  const size_t step = p >> 4;  // p/2 .. p in steps of p/16
  return ((b + step - 1) / step) * step;
}

struct Pool {  // cached device (or pinned host) buffers by size class
  bool host = false;
  std::multimap<size_t, void*> free_;
  std::vector<std::pair<void*, size_t>> all;
  void* get(size_t want, size_t* cap) {
    const size_t c = size_class(want);
    auto it = free_.lower_bound(c);
    if (it != free_.end() && it->first <= c + c / 4) {
      void* p = it->second;
      *cap = it->first;
      free_.erase(it);
      return p;
    }
    void* p = nullptr;
    const hipError_t e = host ? hipHostMalloc(&p, c, hipHostMallocDefault) : hipMalloc(&p, c);
    if (e != hipSuccess) return nullptr;
    all.emplace_back(p, c);
    *cap = c;
    return p;
  }
  void put(void* p, size_t cap) {
    if (p) free_.emplace(cap, p);
  }
  void release() {
    for (auto& a : all) {
      if (host)
        hipHostFree(a.first);
      else
        hipFree(a.first);
    }
    all.clear();
    free_.clear();
  }
};

enum ReqState { RQ_QUEUED, RQ_ACTIVE, RQ_CHECK, RQ_WAIT_CHILD, RQ_FINISHING, RQ_DONE };

struct Req {
  uint64_t tag = 0;
  hsrq_problem_t prob{};
  std::vector<double> wr, wi;
  int prec = 0;
  size_t charge = 0;  // budget bytes
  double t_submit = 0, t_start = 0, t_done = 0;
  void* work = nullptr;
  size_t work_cap = 0;
  void* head = nullptr;  // pinned head image
  size_t head_cap = 0;
  Plan plan;
  ProbDesc desc{};
  int t = 0;
  ReqState state = RQ_QUEUED;
  hipEvent_t ev = nullptr;  // completion of the last enqueued phase
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
  int status = HSRQ_OK;
  int fallback = 0;
  // mixed precision
  size_t o_keep = 0;           // starting vectors kept in the workspace
  std::vector<int> fail;       // failing shifts (parent)
  Req* parent = nullptr;       // set on a fallback child
  Req* child = nullptr;
  ~Req() {
    if (ready) hipEventDestroy(ready);
  }
  std::vector<int> child_cols;  // parent column of each child column
  std::vector<CopyEnt> scatter;
  void* lists = nullptr;
  size_t lists_cap = 0;
};

}  // namespace

struct hsrq_server_s {
  int device = 0;
  size_t budget = 0, used = 0;
  hsrq_opts_t opts{};
  int nb = 128;
  int fcb = 64;  // columns per far-tile block of the all-FP64 requests
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::deque<std::unique_ptr<Req>> queue;          // submitted, not admitted
  std::vector<std::unique_ptr<Req>> live;          // admitted, not completed
  std::vector<hsrq_completion_t> done;
  std::chrono::steady_clock::time_point t0;
  int init_status = HSRQ_OK;
  bool ready = false;
  // device state, worker thread only
  hipStream_t s = nullptr, a = nullptr;
  Pool dpool, hpool;
  void* tick_dev = nullptr;
  void* tick_host[kRing] = {};
  hipEvent_t tick_ev[kRing] = {};
  hipEvent_t ev_far = nullptr, ev_copy = nullptr;
  int tick_slot = 0;
  std::vector<hipEvent_t> ev_free;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

hipEvent_t get_event(hsrq_server_s* S) {
  if (!S->ev_free.empty()) {
    hipEvent_t e = S->ev_free.back();
    S->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// workspace of one request: the plan, then (precision 1) the kept starting
// vectors and an internal residual array
size_t request_bytes(const hsrq_problem_t& p, int prec, int nb, int fcb, size_t* plan_bytes, size_t* keep_off) {
  Plan P;
  build_plan(P, 1, &p, nb, prec == 0 ? fcb : 64);
  size_t w = align_up(P.total_bytes);
  *keep_off = w;
  const size_t cols = (size_t)count_cols(p.m, p.wi);
  if (prec == 1) w += align_up(sizeof(double) * (size_t)p.n * cols) + align_up(sizeof(double) * (size_t)p.m);
  *plan_bytes = P.total_bytes;
  return w;
}

// admission: workspace, plan, head image; enqueue head copy, prep, init
int admit(hsrq_server_s* S, Req* r) {
  size_t pb = 0, keep = 0;
  const size_t wb = request_bytes(r->prob, r->prec, S->nb, S->fcb, &pb, &keep);
  r->work = S->dpool.get(wb, &r->work_cap);
  if (!r->work) return HSRQ_ERR_ALLOC;
  r->o_keep = keep;
  if (r->prec == 1 && !r->prob.resid) {  // the check needs residuals
    const size_t cols = (size_t)count_cols(r->prob.m, r->prob.wi);
    r->prob.resid = at<double>(r->work, keep + align_up(sizeof(double) * (size_t)r->prob.n * cols));
  }
  build_plan(r->plan, 1, &r->prob, S->nb, r->prec == 0 ? S->fcb : 64);
  r->plan.prec = r->prec;
  r->head = S->hpool.get(r->plan.head_bytes, &r->head_cap);
  if (!r->head) return HSRQ_ERR_ALLOC;
  hsrq_opts_t o = S->opts;
  o.precision = r->prec;
  fill_staging(r->plan, 1, &r->prob, r->work, &o, static_cast<char*>(r->head));
  std::memcpy(&r->desc, static_cast<char*>(r->head) + r->plan.o_desc, sizeof(ProbDesc));
  const Plan& P = r->plan;
  hipStream_t s = S->s;
  // the caller's H and X are complete once its stream reaches the submission
  if (r->ready && hipStreamWaitEvent(s, r->ready, 0) != hipSuccess) return HSRQ_ERR_HIP;
  if (hipMemcpyAsync(r->work, r->head, P.head_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return HSRQ_ERR_HIP;
  const ProbDesc* dd = at<ProbDesc>(r->work, P.o_desc);
  launch_fill(at<double>(r->work, P.o_zero_all), (long long)P.zero_count, 0.0, s);
  launch_prep(dd, at<int4>(r->work, P.o_bprep), (int)P.blk_prep.size(), 1, P.nmax, s);
  launch_init(dd, at<int4>(r->work, P.o_binit), (int)P.blk_init.size(), s);
  if (r->prec == 1 && r->prob.m > 0) {  // keep the starting vectors for the fallback
    const size_t cols = (size_t)count_cols(r->prob.m, r->prob.wi);
    if (hipMemcpy2DAsync(at<double>(r->work, r->o_keep), sizeof(double) * r->prob.n, r->prob.X,
                         sizeof(double) * r->prob.ldx, sizeof(double) * r->prob.n, cols, hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
      return HSRQ_ERR_HIP;
  }
  r->t = 0;
  r->t_start = S->now();
  r->state = RQ_ACTIVE;
  return HSRQ_OK;
}

void release(hsrq_server_s* S, Req* r) {
  S->dpool.put(r->work, r->work_cap);
  S->hpool.put(r->head, r->head_cap);
  S->hpool.put(r->lists, r->lists_cap);
  r->work = r->head = r->lists = nullptr;
  if (r->ev) S->ev_free.push_back(r->ev);
  r->ev = nullptr;
}

// final kernels of a request whose steps are done
int finish_steps(hsrq_server_s* S, Req* r) {
  const Plan& P = r->plan;
  hipStream_t s = S->s;
  const ProbDesc* dd = at<ProbDesc>(r->work, P.o_desc);
  launch_final(dd, at<int2>(r->work, P.o_bcols), (int)P.blk_cols.size(), at<int4>(r->work, P.o_bfin),
               (int)P.blk_fin.size(), s);
  const bool resid = r->prec == 1 || r->parent || (S->opts.residual && r->prob.resid);
  if (resid)
    launch_resid(dd, at<int4>(r->work, P.o_bout), (int)P.blk_out.size(), at<int2>(r->work, P.o_bcols),
                 (int)P.blk_cols.size(), s);
  if (r->prec == 0) launch_output(dd, at<int4>(r->work, P.o_bout), (int)P.blk_out.size(), s);
  if (!r->ev) r->ev = get_event(S);
  if (!r->ev || hipEventRecord(r->ev, s) != hipSuccess) return HSRQ_ERR_HIP;
  r->state = r->prec == 1 ? RQ_CHECK : RQ_FINISHING;
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

// one tick: the current step of every active request
int tick(hsrq_server_s* S) {
  std::vector<Req*> act;
  for (auto& r : S->live)
    if (r->state == RQ_ACTIVE) act.push_back(r.get());
  if (act.empty()) return HSRQ_OK;
  // task lists per precision, descriptors of every active request
  std::vector<ProbDesc> descs;
  std::vector<Task> crit[2], far[2];
  for (Req* r : act) {
    const int p = (int)descs.size();
    descs.push_back(r->desc);
    const ProbDesc& d = r->desc;
    const int t = r->t;
    const int ncrit = (d.ncols + kCrit - 1) / kCrit;
    for (int L = 0; L < ncrit; ++L)
      crit[r->prec].push_back(t == 0 ? Task{p, task_code(TK_CHAIN, 0), d.N - 1, L}
                                     : Task{p, task_code(TK_CRIT, t), d.N - t - 1, L});
    if (t > 0)
      for (int i = 0; i < d.N - t - 1; ++i)
        for (int L = 0; L < d.nfblk; ++L) far[r->prec].push_back(Task{p, task_code(TK_FAR, t), i, L});
  }
  const size_t bd = align_up(sizeof(ProbDesc) * descs.size());
  size_t off[4], tot = bd;
  std::vector<Task>* lists[4] = {&crit[0], &crit[1], &far[0], &far[1]};
  for (int k = 0; k < 4; ++k) {
    off[k] = tot;
    tot = align_up(tot + sizeof(Task) * lists[k]->size());
  }
  if (tot > kTickBytes / kRing) return HSRQ_ERR_WORKSPACE;  // admission keeps ticks below this
  const int sl = S->tick_slot;
  S->tick_slot = (sl + 1) % kRing;
  if (hipEventSynchronize(S->tick_ev[sl]) != hipSuccess) return HSRQ_ERR_HIP;
  char* hb = static_cast<char*>(S->tick_host[sl]);
  std::memcpy(hb, descs.data(), sizeof(ProbDesc) * descs.size());
  for (int k = 0; k < 4; ++k)
    if (!lists[k]->empty()) std::memcpy(hb + off[k], lists[k]->data(), sizeof(Task) * lists[k]->size());
  char* db = static_cast<char*>(S->tick_dev) + (size_t)sl * (kTickBytes / kRing);
  hipStream_t s = S->s, a = S->a;
  // the previous tick's far kernels, then this tick's arrays
  if (hipStreamWaitEvent(s, S->ev_far, 0) != hipSuccess) return HSRQ_ERR_HIP;
  if (hipMemcpyAsync(db, hb, tot, hipMemcpyHostToDevice, s) != hipSuccess) return HSRQ_ERR_HIP;
  hipEventRecord(S->tick_ev[sl], s);
  hipEventRecord(S->ev_copy, s);
  hipStreamWaitEvent(a, S->ev_copy, 0);
  const ProbDesc* dd = reinterpret_cast<const ProbDesc*>(db);
  for (int pr = 0; pr < 2; ++pr) {
    if (!crit[pr].empty())
      launch_crit(S->nb, pr, S->opts.rotations, share_step((int)far[pr].size(), pr == 0 ? S->fcb : 64, share_min(&S->opts)) ? 1 : 0, dd, reinterpret_cast<const Task*>(db + off[pr]), (int)crit[pr].size(), s);
    if (!far[pr].empty())
      launch_far(S->nb, pr, S->opts.rotations, pr == 0 ? S->fcb : 64, dd, reinterpret_cast<const Task*>(db + off[2 + pr]),
                 (int)far[pr].size(), a);
  }
  hipEventRecord(S->ev_far, a);
  // advance; requests whose last step ran get their final kernels
  bool any_end = false;
  for (Req* r : act)
    if (++r->t >= r->desc.N) any_end = true;
  if (any_end) {
    if (hipStreamWaitEvent(s, S->ev_far, 0) != hipSuccess) return HSRQ_ERR_HIP;
    for (Req* r : act)
      if (r->t >= r->desc.N) {
        const int st = finish_steps(S, r);
        if (st) return st;
      }
  }
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

// mixed precision, after the first pass: the check, then the output and the
// fallback child if shifts fail
int check_request(hsrq_server_s* S, Req* r) {
  const int m = r->prob.m;
  std::vector<double> res(std::max(m, 1));
  std::vector<int32_t> inf(std::max(m, 1));
  const double* rp = r->desc.Ru;
  if (hipMemcpy(res.data(), rp, sizeof(double) * m, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(inf.data(), r->prob.info, sizeof(int32_t) * m, hipMemcpyDeviceToHost) != hipSuccess)
    return HSRQ_ERR_HIP;
  const double tol = 10.0 * r->prob.n * std::ldexp(1.0, -52);
  r->fail.clear();
  for (int l = 0; l < m; ++l) {
    const bool final_flag = inf[l] == 2 || inf[l] == 3 || inf[l] == 4;
    if (!final_flag && (inf[l] != 0 || !(res[l] <= tol))) r->fail.push_back(l);
  }
  const Plan& P = r->plan;
  hipStream_t s = S->s;
  launch_output(at<ProbDesc>(r->work, P.o_desc), at<int4>(r->work, P.o_bout), (int)P.blk_out.size(), s);
  r->fallback = (int)r->fail.size();
  if (r->fail.empty()) {
    if (hipEventRecord(r->ev, s) != hipSuccess) return HSRQ_ERR_HIP;
    r->state = RQ_FINISHING;
    return HSRQ_OK;
  }
  // the child: the failing shifts, all FP64, from the kept starting vectors;
  // its X, scale and info arrays live in its own workspace tail
  auto c = std::make_unique<Req>();
  c->tag = r->tag;
  c->prec = 0;
  c->parent = r;
  const hsrq_problem_t& pr = r->prob;
  std::vector<int> firstcol(m);
  for (int l = 0, k = 0; l < m; ++l) {
    firstcol[l] = k;
    k += pr.wi[l] != 0.0 ? 2 : 1;
  }
  for (int l : r->fail) {
    c->wr.push_back(pr.wr[l]);
    c->wi.push_back(pr.wi[l]);
    for (int k = 0; k < (pr.wi[l] != 0.0 ? 2 : 1); ++k) c->child_cols.push_back(firstcol[l] + k);
  }
  hsrq_problem_t q{};
  q.n = pr.n;
  q.H = pr.H;
  q.ldh = pr.ldh;
  q.m = (int)r->fail.size();
  q.wr = c->wr.data();
  q.wi = c->wi.data();
  q.ldx = pr.n;
  c->prob = q;
  size_t pb = 0, keep = 0;
  const size_t wb = request_bytes(q, 0, S->nb, S->fcb, &pb, &keep);
  const size_t nc = c->child_cols.size();
  const size_t tail = align_up(sizeof(double) * pr.n * nc) + align_up(24 * (size_t)q.m + 64);
  c->work = S->dpool.get(wb + tail, &c->work_cap);
  if (!c->work) return HSRQ_ERR_ALLOC;
  char* base = static_cast<char*>(c->work) + align_up(wb);
  double* Xc = reinterpret_cast<double*>(base);
  char* sc = base + align_up(sizeof(double) * pr.n * nc);
  c->prob.X = Xc;
  c->prob.scale_mant = reinterpret_cast<double*>(sc);
  c->prob.resid = reinterpret_cast<double*>(sc + 8 * (size_t)q.m);
  c->prob.scale_exp = reinterpret_cast<int32_t*>(sc + 16 * (size_t)q.m);
  c->prob.info = reinterpret_cast<int32_t*>(sc + 20 * (size_t)q.m);
  const double* keepv = at<double>(r->work, r->o_keep);
  for (size_t g = 0; g < nc; ++g)
    if (hipMemcpyAsync(Xc + g * pr.n, keepv + (size_t)c->child_cols[g] * pr.n, sizeof(double) * pr.n,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return HSRQ_ERR_HIP;
  // admit the child with its preallocated workspace
  void* w = c->work;
  size_t wc = c->work_cap;
  build_plan(c->plan, 1, &c->prob, S->nb, S->fcb);
  c->plan.prec = 0;
  c->head = S->hpool.get(c->plan.head_bytes, &c->head_cap);
  if (!c->head) return HSRQ_ERR_ALLOC;
  hsrq_opts_t o = S->opts;
  o.precision = 0;
  fill_staging(c->plan, 1, &c->prob, w, &o, static_cast<char*>(c->head));
  std::memcpy(&c->desc, static_cast<char*>(c->head) + c->plan.o_desc, sizeof(ProbDesc));
  const Plan& P2 = c->plan;
  if (hipMemcpyAsync(w, c->head, P2.head_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return HSRQ_ERR_HIP;
  const ProbDesc* dd = at<ProbDesc>(w, P2.o_desc);
  launch_fill(at<double>(w, P2.o_zero_all), (long long)P2.zero_count, 0.0, s);
  launch_prep(dd, at<int4>(w, P2.o_bprep), (int)P2.blk_prep.size(), 1, P2.nmax, s);
  launch_init(dd, at<int4>(w, P2.o_binit), (int)P2.blk_init.size(), s);
  c->work_cap = wc;
  c->t = 0;
  c->t_start = S->now();
  c->state = RQ_ACTIVE;
  // the scatter list of the child's results over the parent's outputs
  for (size_t g = 0; g < nc; ++g)
    c->scatter.push_back(CopyEnt{Xc + g * pr.n, pr.X + (size_t)c->child_cols[g] * pr.ldx,
                                 (long long)sizeof(double) * pr.n});
  for (size_t j = 0; j < r->fail.size(); ++j) {
    const int l = r->fail[j];
    c->scatter.push_back(CopyEnt{c->prob.scale_exp + j, pr.scale_exp + l, 4});
    c->scatter.push_back(CopyEnt{c->prob.scale_mant + j, pr.scale_mant + l, 8});
    c->scatter.push_back(CopyEnt{c->prob.info + j, pr.info + l, 4});
    if (pr.resid) c->scatter.push_back(CopyEnt{c->prob.resid + j, pr.resid + l, 8});
  }
  r->child = c.get();
  r->state = RQ_WAIT_CHILD;
  S->live.push_back(std::move(c));
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

void complete(hsrq_server_s* S, Req* r) {
  r->t_done = S->now();
  r->state = RQ_DONE;
  hsrq_completion_t c{};
  c.tag = r->tag;
  c.status = r->status;
  c.fallback = r->fallback;
  c.t_submit = r->t_submit;
  c.t_start = r->t_start;
  c.t_done = r->t_done;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->used -= r->charge;
    S->done.push_back(c);
  }
  S->cv_done.notify_all();
}

// completion events and phase transitions
int progress(hsrq_server_s* S) {
  for (size_t i = 0; i < S->live.size(); ++i) {
    Req* r = S->live[i].get();
    if (r->state == RQ_CHECK || r->state == RQ_FINISHING) {
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return HSRQ_ERR_HIP;
      if (r->state == RQ_CHECK) {
        const int st = check_request(S, r);
        if (st) return st;
        continue;
      }
      if (r->parent) {  // a fallback child: scatter over the parent's results
        Req* p = r->parent;
        const size_t need = sizeof(CopyEnt) * r->scatter.size();
        r->lists = S->hpool.get(need, &r->lists_cap);
        if (!r->lists) return HSRQ_ERR_ALLOC;
        std::memcpy(r->lists, r->scatter.data(), need);
        launch_copy(static_cast<const CopyEnt*>(r->lists), (int)r->scatter.size(), S->s);
        if (hipEventRecord(p->ev, S->s) != hipSuccess) return HSRQ_ERR_HIP;
        p->state = RQ_FINISHING;
        p->child = nullptr;
        r->state = RQ_DONE;
        continue;  // the child's buffers are released with the parent below
      }
      complete(S, r);
    }
  }
  // drop completed requests together with their fallback child (a parent
  // completes only after the child's results were scattered)
  std::vector<char> drop(S->live.size(), 0);
  for (size_t i = 0; i < S->live.size(); ++i) {
    const Req* r = S->live[i].get();
    const Req* top = r->parent ? r->parent : r;
    drop[i] = top->state == RQ_DONE;
  }
  std::vector<std::unique_ptr<Req>> keep;
  for (size_t i = 0; i < S->live.size(); ++i)
    if (drop[i]) release(S, S->live[i].get());
  for (size_t i = 0; i < S->live.size(); ++i)
    if (!drop[i]) keep.push_back(std::move(S->live[i]));
  S->live.swap(keep);
  return HSRQ_OK;
}

int tick_bytes_estimate(const Req* r, int nb, int fcb) {
  const int N = (r->prob.n + nb - 1) / nb;
  const int cols = count_cols(r->prob.m, r->prob.wi);
  const int f = r->prec == 0 ? fcb : 64;
  const int nblk = (cols + f - 1) / f, ncrit = (cols + kCrit - 1) / kCrit;
  return (int)(sizeof(ProbDesc) + sizeof(Task) * ((size_t)ncrit + (size_t)std::max(N - 2, 0) * nblk) + 512);
}

void worker_main(hsrq_server_s* S) {
  int st = hipSetDevice(S->device) == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
  if (!st && crit_smem_init() != 0) st = HSRQ_ERR_HIP;
  if (!st && hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) != hipSuccess) st = HSRQ_ERR_HIP;
  if (!st && hipStreamCreateWithFlags(&S->a, hipStreamNonBlocking) != hipSuccess) st = HSRQ_ERR_HIP;
  if (!st && hipMalloc(&S->tick_dev, kTickBytes) != hipSuccess) st = HSRQ_ERR_ALLOC;
  for (int k = 0; k < kRing && !st; ++k) {
    if (hipHostMalloc(&S->tick_host[k], kTickBytes / kRing, hipHostMallocDefault) != hipSuccess) st = HSRQ_ERR_ALLOC;
    if (!st && hipEventCreateWithFlags(&S->tick_ev[k], hipEventDisableTiming) != hipSuccess) st = HSRQ_ERR_HIP;
  }
  if (!st && (hipEventCreateWithFlags(&S->ev_far, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&S->ev_copy, hipEventDisableTiming) != hipSuccess))
    st = HSRQ_ERR_HIP;
  if (!st) hipEventRecord(S->ev_far, S->a);
  S->hpool.host = true;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->init_status = st;
    S->ready = true;
  }
  S->cv_done.notify_all();
  while (!st) {
    // admit from the queue while the budget and the tick arrays allow
    std::vector<std::unique_ptr<Req>> adm;
    {
      std::unique_lock<std::mutex> g(S->mu);
      int tick_est = 0;
      for (auto& r : S->live) tick_est += tick_bytes_estimate(r.get(), S->nb, S->fcb);
      while (!S->queue.empty()) {
        Req* r = S->queue.front().get();
        const int tb = tick_bytes_estimate(r, S->nb, S->fcb);
        if (S->used + r->charge > S->budget || tick_est + tb > (int)(kTickBytes / kRing) / 2) break;
        S->used += r->charge;
        tick_est += tb;
        adm.push_back(std::move(S->queue.front()));
        S->queue.pop_front();
      }
      const bool idle = S->live.empty() && adm.empty();
      if (idle && S->queue.empty()) {
        if (S->stop) break;
        S->cv_work.wait_for(g, std::chrono::milliseconds(50));
        continue;
      }
    }
    for (auto& r : adm) {
      r->status = admit(S, r.get());
      if (r->status) {
        st = r->status;
        break;
      }
      S->live.push_back(std::move(r));
    }
    if (st) break;
    st = tick(S);
    if (st) break;
    st = progress(S);
    if (st) break;
    // nothing active but requests finishing: wait for the device a little
    bool active = false;
    for (auto& r : S->live) active = active || r->state == RQ_ACTIVE;
    if (!active && !S->live.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  if (st) {  // a device error: fail everything still pending
    std::lock_guard<std::mutex> g(S->mu);
    for (auto& r : S->live)
      if (!r->parent) S->done.push_back(hsrq_completion_t{r->tag, st, 0, r->t_submit, r->t_start, S->now()});
    for (auto& r : S->queue) S->done.push_back(hsrq_completion_t{r->tag, st, 0, r->t_submit, 0.0, S->now()});
    S->queue.clear();
    S->init_status = st;
  }
  S->cv_done.notify_all();
  if (S->s) hipStreamSynchronize(S->s);
  if (S->a) hipStreamSynchronize(S->a);
  for (auto& r : S->live) release(S, r.get());
  S->live.clear();
  S->dpool.release();
  S->hpool.release();
  if (S->tick_dev) hipFree(S->tick_dev);
  for (int k = 0; k < kRing; ++k) {
    if (S->tick_host[k]) hipHostFree(S->tick_host[k]);
    if (S->tick_ev[k]) hipEventDestroy(S->tick_ev[k]);
  }
  for (hipEvent_t e : S->ev_free) hipEventDestroy(e);
  if (S->ev_far) hipEventDestroy(S->ev_far);
  if (S->ev_copy) hipEventDestroy(S->ev_copy);
  if (S->s) hipStreamDestroy(S->s);
  if (S->a) hipStreamDestroy(S->a);
}

}  // namespace

extern "C" {

int hsrq_server_create(hsrq_server_t* out, int device, size_t hbm_budget_bytes, const hsrq_opts_t* opts) {
  if (!out) return -1;
  *out = nullptr;
  if (hbm_budget_bytes == 0) return -3;
  if (opts && opts->nb != 0 && opts->nb != 64 && opts->nb != 128) return -4;
  if (opts && opts->precision != 0 && opts->precision != 1) return -4;
  if (opts && opts->rotations != 0 && opts->rotations != 1) return -4;
  if (opts && !opts_valid(opts)) return -4;
  hsrq_server_s* S = new (std::nothrow) hsrq_server_s();
  if (!S) return HSRQ_ERR_ALLOC;
  S->device = device;
  S->budget = hbm_budget_bytes;
  if (opts) S->opts = *opts;
  S->nb = (opts && opts->nb) ? opts->nb : 128;
  S->fcb = (opts && opts->cols_per_block == 32 && opts->rotations == 1) ? 32 : 64;
  S->t0 = std::chrono::steady_clock::now();
  S->worker = std::thread(worker_main, S);
  std::unique_lock<std::mutex> g(S->mu);
  S->cv_done.wait(g, [&] { return S->ready; });
  const int st = S->init_status;
  g.unlock();
  if (st) {
    S->worker.join();
    delete S;
    return st;
  }
  *out = S;
  return HSRQ_OK;
}

int hsrq_server_submit(hsrq_server_t S, const hsrq_problem_t* problem, uint64_t tag, void* stream) {
  if (!S || !problem) return HSRQ_ERR_ARG;
  const int chk = check_problem(*problem);
  if (chk || problem->m < 1) return HSRQ_ERR_ARG;
  auto r = std::make_unique<Req>();
  r->tag = tag;
  r->prob = *problem;
  r->wr.assign(problem->wr, problem->wr + problem->m);
  r->wi.assign(problem->wi, problem->wi + problem->m);
  r->prob.wr = r->wr.data();
  r->prob.wi = r->wi.data();
  r->prec = S->opts.precision;
  size_t pb = 0, keep = 0;
  const size_t cols = (size_t)count_cols(problem->m, problem->wi);
  r->charge = size_class(request_bytes(r->prob, r->prec, S->nb, S->fcb, &pb, &keep)) +
              sizeof(double) * (size_t)problem->ldh * problem->n + sizeof(double) * (size_t)problem->ldx * cols;
  if (r->prec == 1) r->charge += r->charge / 2;  // room for a fallback child
  if (r->charge > S->budget) return HSRQ_ERR_BUSY;
  if (tick_bytes_estimate(r.get(), S->nb, S->fcb) > (int)(kTickBytes / kRing) / 2) return HSRQ_ERR_BUSY;
  {
    // order the request after the work the caller has enqueued on its
    // stream so far (NULL is the null stream, torch's default stream; the
    // event is created on the server's device)
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(S->device) != hipSuccess) return HSRQ_ERR_HIP;
    hipError_t e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->ready, static_cast<hipStream_t>(stream));
    hipSetDevice(cur);
    if (e != hipSuccess) return HSRQ_ERR_HIP;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop || S->init_status) return HSRQ_ERR_ARG;
    r->t_submit = S->now();
    S->queue.push_back(std::move(r));
  }
  S->cv_work.notify_one();
  return HSRQ_OK;
}

int hsrq_server_poll(hsrq_server_t S, hsrq_completion_t* out, int max, int* count, int wait_ms) {
  if (!S || !count || max < 0 || (max > 0 && !out)) return HSRQ_ERR_ARG;
  std::unique_lock<std::mutex> g(S->mu);
  if (S->done.empty() && wait_ms > 0)
    S->cv_done.wait_for(g, std::chrono::milliseconds(wait_ms), [&] { return !S->done.empty(); });
  const int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *count = k;
  return S->init_status;
}

int hsrq_server_clock(hsrq_server_t S, double* seconds) {
  if (!S || !seconds) return HSRQ_ERR_ARG;
  *seconds = S->now();
  return HSRQ_OK;
}

int hsrq_server_destroy(hsrq_server_t S) {
  if (!S) return HSRQ_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  delete S;
  return HSRQ_OK;
}

}  // extern "C"
