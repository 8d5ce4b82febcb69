// Serving loop of the C ABI: continuous batching of thermal solves.
//
// A request is one XTRG run (a lattice's XXZ Hamiltonian, the series start
// at tau0, n doublings at bond budget D).  The z-shifted grids and other
// independent runs of Sec. II.B (Eq. zshift) share no data, so any set of
// them can advance together: a worker thread owned by the context admits
// queued requests whenever their device-memory estimate fits the budget,
// advances every admitted request by one doubling per batch step through
// the batched doubling (one grouped SVD launch per Jacobi round for all of
// them), accumulates lambda_{n+1} = 2 lambda_n + ln c and the observables of
// Eq. (ThermalQuan) after each doubling, and retires finished requests at
// once.  Requests that arrive while others run join at the next batch step.
// A request whose numbers turn non-finite, or whose memory the budget
// refuses, fails alone with its status; the others continue.  Each result
// is the one the same request gets alone: the batched doubling returns for
// every chain what the single-chain call returns.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "context.h"

namespace xtrg {

namespace {

// ---------------------------------------------------------------------------
// Minimal JSON reader for the request objects (objects, arrays, numbers,
// strings without escapes beyond \" and \\, true / false / null).
// ---------------------------------------------------------------------------
struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0.0;
  bool b = false;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const std::string& k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p;
  }
  [[noreturn]] void fail(const char* what) {
    throw Error(XTRG_EINVAL, std::string("request JSON: ") + what);
  }
  std::string string() {
    if (p >= end || *p != '"') fail("expected a string");
    ++p;
    std::string out;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= end || (*p != '"' && *p != '\\' && *p != '/')) fail("unsupported escape");
      }
      out += *p++;
    }
    if (p >= end) fail("unterminated string");
    ++p;
    return out;
  }
  JVal value(int depth) {
    if (depth > 16) fail("nested too deeply");
    ws();
    if (p >= end) fail("unexpected end");
    JVal v;
    if (*p == '{') {
      v.kind = JVal::OBJ;
      ++p;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return v;
      }
      for (;;) {
        ws();
        std::string k = string();
        ws();
        if (p >= end || *p != ':') fail("expected ':'");
        ++p;
        v.obj.emplace_back(k, value(depth + 1));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') {
          ++p;
          return v;
        }
        fail("expected ',' or '}'");
      }
    }
    if (*p == '[') {
      v.kind = JVal::ARR;
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return v;
      }
      for (;;) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          return v;
        }
        fail("expected ',' or ']'");
      }
    }
    if (*p == '"') {
      v.kind = JVal::STR;
      v.str = string();
      return v;
    }
    auto word = [&](const char* w) {
      const size_t n = std::strlen(w);
      if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) {
        p += n;
        return true;
      }
      return false;
    };
    if (word("true")) {
      v.kind = JVal::BOOL;
      v.b = true;
      return v;
    }
    if (word("false")) {
      v.kind = JVal::BOOL;
      return v;
    }
    if (word("null")) return v;
    if (word("NaN")) {            // accepted so that bad numbers reach the solver as numbers
      v.kind = JVal::NUM;
      v.num = std::nan("");
      return v;
    }
    char* q = nullptr;
    v.num = std::strtod(p, &q);
    if (q == p) fail("expected a value");
    p = q;
    v.kind = JVal::NUM;
    return v;
  }
};

JVal parse_json(const char* text) {
  JParser ps{text, text + std::strlen(text)};
  JVal v = ps.value(0);
  ps.ws();
  if (ps.p != ps.end) ps.fail("trailing characters");
  if (v.kind != JVal::OBJ) ps.fail("a request is an object");
  return v;
}

double num_field(const JVal& o, const char* k, double dflt, bool required = false) {
  const JVal* v = o.get(k);
  if (!v) {
    if (required) throw Error(XTRG_EINVAL, std::string("request: missing field ") + k);
    return dflt;
  }
  if (v->kind != JVal::NUM) throw Error(XTRG_EINVAL, std::string("request: field ") + k + " must be a number");
  return v->num;
}

int int_field(const JVal& o, const char* k, int dflt, bool required = false) {
  const double v = num_field(o, k, dflt, required);
  if (!(v == std::floor(v)) || std::fabs(v) > 1e9)
    throw Error(XTRG_EINVAL, std::string("request: field ") + k + " must be an integer");
  return (int)v;
}

// ---------------------------------------------------------------------------
// Requests and the server
// ---------------------------------------------------------------------------
using Clock = std::chrono::steady_clock;

struct Request {
  unsigned long long id = 0;
  // the solve
  int n_sites = 0;
  std::vector<int> bonds;
  std::vector<double> jxy, jz;
  double tau0 = 0.0, beta_mix = 1.0;
  double series_tol = 0.0;   // > 0: the series start to this expansion error instead of order 1 / 2
  int n_doublings = 0, D = 0, n_sweeps = 2, order = 1, precision = XTRG_FP64;
  bool u1 = false;           // U(1) charge sectors: charge-definite start, C_E factorised by S^z blocks
  // state
  bool done = false;       // visible to poll (set under the server lock)
  bool admitted = false;   // likewise: admitted to the batch
  int progress = 0;        // likewise: doublings completed
  bool finished = false;   // set by the worker when the run ends
  int status = XTRG_OK;
  std::string err;
  std::unique_ptr<xtrg_mpo_s> H, rho;
  double lam = 0.0, tau = 0.0;
  int n_done = 0;
  double flops = 0.0;      // algorithmic flops of its doublings
  size_t footprint = 0;
  std::string records;    // JSON array body
  Clock::time_point t_submit, t_admit, t_finish;
};

// Device bytes of one solve during a doubling at bond budget D (FP64
// estimate, an upper bound for the mixed forms): per-site environment
// blocks 4 D^3 (L - 1), warm-start bases (4D)(4D + 32)(L - 1), sites and
// their copies 16 D^2 L, environments 6 D^3, the two-site tensor and SVD
// workspaces 4 (4D)(4D + 32), those of the QR route of first visits
// 6 (4D)(4D + 32), the Jacobi's closing check (4D + 32)^2, plus 4 MiB for
// the chain's share of the grouped SVD launch (descriptor and Gram
// partials of up to 128 block pairs).
size_t footprint_bytes(int L, int D) {
  const double d = D, m = 4.0 * d, mc = m + 32.0;
  const double elems = 4.0 * d * d * d * (L - 1) + m * mc * (L - 1) + 16.0 * d * d * L + 6.0 * d * d * d +
                       4.0 * m * mc + 6.0 * m * mc + mc * mc;
  return (size_t)(8.0 * elems) + (size_t(4) << 20);
}

// Device bytes the context holds besides the chains' own: 64 MiB (scratch,
// Hamiltonians, small workspaces) plus the split-K partials of the largest
// two-site overlap, 16 (4D)^2 doubles at bond budget D.
size_t shared_bytes(int D_max) {
  const double m = 4.0 * D_max;
  return (size_t(64) << 20) + (size_t)(8.0 * 16.0 * m * m);
}

std::string fmt(const char* f, ...) __attribute__((format(printf, 1, 2)));
std::string fmt(const char* f, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, f);
  std::vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return buf;
}

std::string json_escape(const std::string& s) {
  std::string o;
  for (char ch : s) {
    if (ch == '"' || ch == '\\') o += '\\';
    if (ch == '\n') {
      o += "\\n";
      continue;
    }
    o += ch;
  }
  return o;
}

}  // namespace

// One lane of the server: a worker thread with its own context (and stream)
// that advances its admitted requests in lockstep, one doubling per batch
// step.  Lanes run concurrently on the device: the Jacobi rounds of a
// single batch leave most compute units idle, so a second batch of
// requests of a different size overlaps them instead of waiting behind the
// larger requests' doublings.
struct Lane {
  xtrg_ctx c = nullptr;       // lane 0: the server's context; others owned by the lane
  hipStream_t stream = nullptr;
  bool owned = false;
  std::thread worker;
  bool running = false;       // the worker thread is in its loop
  std::deque<Request*> pending;
  std::vector<Request*> active;
  // Requests finished since the loop last held the lock: they are marked
  // done there, together with the decision to leave the loop, so that a
  // client that sees its last result done also finds the lane idle.
  std::vector<Request*> finished_now;
  size_t used = 0, shared = 0;   // admitted footprints and the lane's shared reserve (under the server lock)
};

struct Server {
  xtrg_ctx c = nullptr;
  std::mutex mu;
  bool stop = false;         // context teardown: finish the batch step, then leave
  unsigned long long next_id = 1;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::map<unsigned long long, std::unique_ptr<Request>> all;
  size_t budget = 0;
  int max_chains = 64;
  double max_cost = 0.0;     // largest per-doubling cost proxy seen
  Clock::time_point t0 = Clock::now();

  double secs(Clock::time_point t) const { return std::chrono::duration<double>(t - t0).count(); }

  // Work of one doubling at saturation, up to a constant: sites x D^4.
  static double cost(const Request& r) { return (double)r.n_sites * std::pow((double)r.D, 4.0); }

  // Lane of a new request: 0 for the largest class, k for requests
  // 8^k times cheaper than the largest seen so far (the last lane takes the rest).
  int route(const Request& r) {
    const double w = cost(r);
    max_cost = std::max(max_cost, w);
    int k = 0;
    while (k + 1 < (int)lanes.size() && w * std::pow(8.0, k + 1) <= max_cost) ++k;
    return k;
  }

  bool any_running() const {
    for (const auto& l : lanes)
      if (l->running) return true;
    return false;
  }

  void record(Lane& ln, Request& r, const xtrg_compress_info* info) {
    xtrg_obs a{}, b{};
    xtrg_impl::observables(ln.c, r.rho.get(), r.lam, r.tau, r.H.get(), r.n_sites, &a, &b, nullptr);
    std::string dims = "[";
    for (size_t i = 0; i < r.rho->dims.size(); ++i) dims += (i ? "," : "") + std::to_string(r.rho->dims[i]);
    dims += "]";
    if (info) r.flops += info->flops;
    if (!r.records.empty()) r.records += ",";
    r.records += fmt("{\"n\":%d,\"tau\":%.17g,\"lam\":%.17g,", r.n_done, r.tau, r.lam) + "\"bond_dims\":" + dims +
                 fmt(",\"f_tau\":%.17g,\"u_tau\":%.17g,\"c_tau\":%.17g,\"f_2tau\":%.17g,\"u_2tau\":%.17g,"
                     "\"c_2tau\":%.17g,\"herm_resid\":%.17g,\"sz_tot\":%.17g,\"su2_resid\":%.17g,\"trunc_err\":%.17g,"
                     "\"flops\":%.17g}",
                     a.f, a.u, a.c, b.f, b.u, b.c, b.herm_resid, b.sz_tot, b.su2_resid,
                     info ? info->trunc_err_max : 0.0, info ? info->flops : 0.0);
  }

  void finish(Lane& ln, Request& r, int status, const std::string& err) {
    r.finished = true;
    r.status = status;
    r.err = err;
    r.t_finish = Clock::now();
    r.rho.reset();
    r.H.reset();
    ln.finished_now.push_back(&r);
  }

  // Build H and rho(tau0) of an admitted request, with its first record.
  void admit(Lane& ln, Request& r) {
    r.t_admit = Clock::now();
    try {
      r.H = xtrg_impl::hamiltonian(ln.c, r.n_sites, (int)r.jxy.size(), r.bonds.data(), r.jxy.data(), r.jz.data());
      if (r.series_tol > 0) {
        int nt = 0;
        r.rho = xtrg_impl::settn_init(ln.c, r.H.get(), r.tau0, r.D, 2, r.series_tol, &r.lam, &nt);
      } else {
        r.rho = xtrg_impl::init_rho(ln.c, r.H.get(), r.tau0, r.order, 0, &r.lam, r.u1);
      }
      r.tau = r.tau0;
      record(ln, r, nullptr);
    } catch (const Error& e) {
      if (e.code == XTRG_EDEVICE) throw;
      finish(ln, r, e.code, e.what());
    }
  }

  // One batch step of a lane: every active request advances by one doubling.
  void step(Lane& ln) {
    const int n = (int)ln.active.size();
    std::vector<xtrg_mpo> ins(n), outs(n, nullptr);
    std::vector<xtrg_compress_opts> opts(n);
    std::vector<xtrg_compress_info> infos(n);
    for (int q = 0; q < n; ++q) {
      Request& r = *ln.active[q];
      ins[q] = r.rho.get();
      xtrg_compress_opts o{};
      o.D_max = r.D;
      o.n_sweeps = r.n_sweeps;
      // the doubling reaches beta = 2 tau_{n+1} = 4 tau_n: mixed contractions
      // only from beta_mix on (the high-temperature doublings stay FP64)
      o.precision = 4.0 * r.tau >= r.beta_mix ? r.precision : XTRG_FP64;
      o.degen_rtol = 1e-6;
      o.sv_floor = 1e-14;
      o.u1 = r.u1 ? 1 : 0;
      opts[q] = o;
      infos[q] = xtrg_compress_info{};
    }
    std::string err;
    xtrg_impl::square_compress(ln.c, n, ins.data(), opts.data(), outs.data(), infos.data(), &err);
    std::vector<Request*> still;
    for (int q = 0; q < n; ++q) {
      Request& r = *ln.active[q];
      if (!outs[q]) {
        finish(ln, r, infos[q].status, "doubling " + std::to_string(r.n_done + 1) + ": " +
                                           (infos[q].status == XTRG_ENOMEM ? "device memory refused by the budget"
                                                                           : "non-finite numbers in the compression"));
        continue;
      }
      r.rho.reset(outs[q]);
      r.lam = 2.0 * r.lam + infos[q].dlog_norm;
      r.tau *= 2.0;
      r.n_done += 1;
      try {
        record(ln, r, &infos[q]);
      } catch (const Error& e) {
        if (e.code == XTRG_EDEVICE) throw;
        finish(ln, r, e.code, e.what());
        continue;
      }
      if (r.n_done >= r.n_doublings) finish(ln, r, XTRG_OK, "");
      else still.push_back(&r);
    }
    if ((int)still.size() < n) xtrg_impl::trim(ln.c);   // workspaces sized for the chains that left
    ln.active = still;
  }

  // Memory the other lanes hold (footprints and shared reserves), under the lock.
  size_t used_elsewhere(const Lane& ln) const {
    size_t u = 0;
    for (const auto& l : lanes)
      if (l.get() != &ln) u += l->used + l->shared;
    return u;
  }

  void loop(Lane& ln) {
    (void)hipSetDevice(c->device);
    for (;;) {
      std::vector<Request*> admit_now;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (Request* r : ln.finished_now) r->done = true;
        ln.finished_now.clear();
        for (Request* r : ln.active) {
          r->admitted = true;
          r->progress = r->n_done;
        }
        if (stop || (ln.pending.empty() && ln.active.empty())) {
          ln.running = false;
          ln.used = ln.shared = 0;
          if (!any_running()) c->serving.store(false);
          return;
        }
        // admission in arrival order while the estimate fits the budget left
        // by the other lanes (this lane's shared workspaces for its largest
        // bond budget first)
        const size_t other = used_elsewhere(ln);
        size_t used = 0;
        int dmax = 0;
        for (Request* r : ln.active) {
          used += r->footprint;
          dmax = std::max(dmax, r->D);
        }
        while (!ln.pending.empty() && (int)(ln.active.size() + admit_now.size()) < max_chains) {
          Request* r = ln.pending.front();
          const size_t shared = shared_bytes(std::max(dmax, r->D));
          if (r->footprint + shared > budget) {   // would never fit: fail now
            ln.pending.pop_front();
            r->status = XTRG_ENOMEM;
            r->err = "device-memory estimate " + std::to_string(r->footprint) + " B exceeds the serving budget " +
                     std::to_string(budget) + " B";
            r->t_admit = r->t_finish = Clock::now();
            r->done = true;
            continue;
          }
          if (other + used + r->footprint + shared > budget) break;   // wait for memory to free up
          used += r->footprint;
          dmax = std::max(dmax, r->D);
          ln.pending.pop_front();
          admit_now.push_back(r);
        }
        ln.used = used;
        ln.shared = (ln.active.empty() && admit_now.empty()) ? 0 : shared_bytes(dmax);
      }
      try {
        for (Request* r : admit_now) {
          admit(ln, *r);
          if (r->rho) ln.active.push_back(r);   // else it failed at its start and is finished
        }
        if (!ln.active.empty()) step(ln);
        else if (admit_now.empty()) {
          // nothing admitted and nothing running: the pending front waits for
          // memory that other lanes hold; look again shortly
          std::this_thread::sleep_for(std::chrono::milliseconds(20));
        }
      } catch (const std::exception& e) {
        // a runtime error ends every request in flight on this lane
        const int code = dynamic_cast<const Error*>(&e) ? static_cast<const Error&>(e).code : XTRG_EDEVICE;
        for (Request* r : ln.active) finish(ln, *r, code, e.what());
        for (Request* r : admit_now)
          if (!r->finished) finish(ln, *r, code, e.what());
        ln.active.clear();
      }
    }
  }

  // Lanes are set up at the first request: lane 0 on the server's context,
  // the others on contexts of their own (same device and budget, each with
  // a stream of its own at the default priority).
  void make_lanes(int n) {
    for (int k = 0; k < n; ++k) {
      auto ln = std::make_unique<Lane>();
      if (k == 0) {
        ln->c = c;
      } else {
        XTRG_HIP(hipSetDevice(c->device));
        XTRG_HIP(hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking));
        const int rc = xtrg_ctx_create(c->device, ln->stream, c->budget, &ln->c);
        if (rc != XTRG_OK) {
          (void)hipStreamDestroy(ln->stream);
          throw Error(rc, "serving lane: context creation failed");
        }
        ln->owned = true;
      }
      lanes.push_back(std::move(ln));
    }
  }

  // Replace the lanes (none running; under the lock).  The requests and
  // their results stay.
  void relane(int n) {
    for (auto& ln : lanes) {
      if (ln->worker.joinable()) ln->worker.join();
      if (ln->owned) {
        (void)xtrg_ctx_destroy(ln->c);
        (void)hipStreamDestroy(ln->stream);
      }
    }
    lanes.clear();
    max_cost = 0.0;
    make_lanes(n);
  }

  void start(Lane& ln) {
    if (ln.running) return;
    if (ln.worker.joinable()) ln.worker.join();   // the previous worker has left its loop
    ln.running = true;
    c->serving.store(true);
    Lane* lp = &ln;
    ln.worker = std::thread([this, lp] { loop(*lp); });
  }
};

void server_shutdown(xtrg_ctx c) {
  Server* S = c->server;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  for (auto& ln : S->lanes)
    if (ln->worker.joinable()) ln->worker.join();
  for (auto& ln : S->lanes) {
    for (Request* r : ln->active) {
      r->rho.reset();
      r->H.reset();
    }
    if (ln->owned) {
      (void)xtrg_ctx_destroy(ln->c);
      (void)hipStreamDestroy(ln->stream);
    }
  }
  delete S;
  c->server = nullptr;
  c->serving.store(false);
}

}  // namespace xtrg

using xtrg::Error;

extern "C" {

int xtrg_serve_submit(xtrg_ctx c, const char* request_json, unsigned long long* id) {
  if (!c || !request_json || !id) return XTRG_EINVAL;
  try {
    auto r = std::make_unique<xtrg::Request>();
    const xtrg::JVal v = xtrg::parse_json(request_json);
    r->n_sites = xtrg::int_field(v, "n_sites", 0, true);
    r->tau0 = xtrg::num_field(v, "tau0", 0.0, true);
    r->n_doublings = xtrg::int_field(v, "n_doublings", 0, true);
    r->D = xtrg::int_field(v, "D", 0, true);
    r->n_sweeps = xtrg::int_field(v, "n_sweeps", 2);
    r->order = xtrg::int_field(v, "order", 1);
    r->beta_mix = xtrg::num_field(v, "beta_mix", 1.0);
    r->series_tol = xtrg::num_field(v, "series_tol", 0.0);
    if (const xtrg::JVal* pv = v.get("precision")) {
      if (pv->kind != xtrg::JVal::STR) throw Error(XTRG_EINVAL, "request: precision is fp64, fp32 or bf16x3");
      if (pv->str == "fp64") r->precision = XTRG_FP64;
      else if (pv->str == "fp32") r->precision = XTRG_FP32;
      else if (pv->str == "bf16x3") r->precision = XTRG_BF16X3;
      else throw Error(XTRG_EINVAL, "request: precision is fp64, fp32 or bf16x3");
    }
    if (const xtrg::JVal* uv = v.get("u1")) {
      if (uv->kind != xtrg::JVal::BOOL) throw Error(XTRG_EINVAL, "request: u1 is true or false");
      r->u1 = uv->b;
    }
    if (r->u1 && r->series_tol > 0) throw Error(XTRG_EINVAL, "request: u1 takes the order-1/2 start (series_tol 0)");
    const xtrg::JVal* bv = v.get("bonds");
    if (!bv || bv->kind != xtrg::JVal::ARR) throw Error(XTRG_EINVAL, "request: bonds is a list of [i, j] pairs");
    for (const auto& b : bv->arr) {
      if (b.kind != xtrg::JVal::ARR || b.arr.size() != 2 || b.arr[0].kind != xtrg::JVal::NUM ||
          b.arr[1].kind != xtrg::JVal::NUM)
        throw Error(XTRG_EINVAL, "request: bonds is a list of [i, j] pairs");
      r->bonds.push_back((int)b.arr[0].num);
      r->bonds.push_back((int)b.arr[1].num);
    }
    const size_t nb = bv->arr.size();
    auto couplings = [&](const char* k, std::vector<double>& out) {
      const xtrg::JVal* cv = v.get(k);
      if (!cv) throw Error(XTRG_EINVAL, std::string("request: missing field ") + k);
      if (cv->kind == xtrg::JVal::NUM) out.assign(nb, cv->num);
      else if (cv->kind == xtrg::JVal::ARR && cv->arr.size() == nb) {
        for (const auto& x : cv->arr) {
          if (x.kind != xtrg::JVal::NUM) throw Error(XTRG_EINVAL, std::string("request: ") + k + " entries are numbers");
          out.push_back(x.num);
        }
      } else {
        throw Error(XTRG_EINVAL, std::string("request: ") + k + " is a number or one number per bond");
      }
    };
    couplings("jxy", r->jxy);
    couplings("jz", r->jz);
    if (r->n_sites < 2 || !(r->tau0 > 0) || r->n_doublings < 0 || r->D < 1 || r->n_sweeps < 1 || r->order < 1 ||
        r->order > 2 || !(r->series_tol >= 0))
      throw Error(XTRG_EINVAL, "request: n_sites >= 2, tau0 > 0, n_doublings >= 0, D >= 1, n_sweeps >= 1, order 1 or 2");
    for (int b : r->bonds)
      if (b < 0 || b >= r->n_sites) throw Error(XTRG_EINVAL, "request: bond index out of range");
    r->footprint = xtrg::footprint_bytes(r->n_sites, r->D);
    r->t_submit = xtrg::Clock::now();

    if (!c->server) {
      auto S0 = std::make_unique<xtrg::Server>();
      S0->c = c;
      S0->make_lanes(c->serve_lanes);
      c->server = S0.release();
    }
    xtrg::Server* S = c->server;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) throw Error(XTRG_EINVAL, "context is being destroyed");
    if (S->budget == 0) {
      size_t fr = 0, tot = 0;
      if (c->budget) S->budget = c->budget;
      else if (hipSetDevice(c->device) == hipSuccess && hipMemGetInfo(&fr, &tot) == hipSuccess)
        S->budget = (size_t)(0.85 * (double)fr);
      else
        throw Error(XTRG_EDEVICE, "hipMemGetInfo failed");
    }
    r->id = S->next_id++;
    *id = r->id;
    xtrg::Lane& ln = *S->lanes[S->route(*r)];
    ln.pending.push_back(r.get());
    S->all[r->id] = std::move(r);
    S->start(ln);
    c->err.clear();
    return XTRG_OK;
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return XTRG_EINVAL;
  }
}

int xtrg_serve_set_lanes(xtrg_ctx c, int n_lanes) {
  if (!c || n_lanes < 1 || n_lanes > 4) return XTRG_EINVAL;
  try {
    xtrg::Server* S = c->server;
    if (!S) {
      c->serve_lanes = n_lanes;
      return XTRG_OK;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->any_running()) return XTRG_EBUSY;
    c->serve_lanes = n_lanes;
    S->relane(n_lanes);
    return XTRG_OK;
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  }
}

int xtrg_serve_poll(xtrg_ctx c, unsigned long long id, char* result_json, size_t cap) {
  if (!c || !result_json || cap == 0) return XTRG_EINVAL;
  xtrg::Server* S = c->server;
  if (!S) return XTRG_EINVAL;
  std::string out;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) return XTRG_EINVAL;
    const xtrg::Request& r = *it->second;
    if (!r.done) {   // progress: the state and the doublings completed so far
      out = xtrg::fmt("{\"id\":%llu,\"state\":\"%s\",\"doublings\":%d}", r.id,
                      r.admitted ? "running" : "queued", r.progress);
      if (out.size() + 1 <= cap) std::memcpy(result_json, out.c_str(), out.size() + 1);
      return XTRG_EBUSY;
    }
    const double sub = S->secs(r.t_submit), adm = S->secs(r.t_admit), fin = S->secs(r.t_finish);
    out = xtrg::fmt("{\"id\":%llu,\"status\":%d,\"error\":\"", r.id, r.status) + xtrg::json_escape(r.err) +
          xtrg::fmt("\",\"submitted_s\":%.9g,\"admitted_s\":%.9g,\"finished_s\":%.9g,\"latency_s\":%.9g,"
                    "\"doublings\":%d,\"flops\":%.17g,\"records\":[",
                    sub, adm, fin, fin - sub, r.n_done, r.flops) +
          r.records + "]}";
  }
  if (out.size() + 1 > cap) return XTRG_EINVAL;
  std::memcpy(result_json, out.c_str(), out.size() + 1);
  return XTRG_OK;
}

}  // extern "C"
