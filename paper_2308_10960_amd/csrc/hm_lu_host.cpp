// Host driver of the H-LU factorisation with accumulated updates
// (include/hm_lu.h): walks the recursion of the block LU over the block tree
// and enqueues the kernels of hm_lu.hip on one stream.  All numbers stay on
// the device: the ranks of low-rank blocks are device integers that the
// kernels read, and the host sizes every buffer by capacities (upper bounds
// of the ranks), so nothing is read back until the factorisation ends.
//
// Device memory comes from one arena allocated at creation, handed out by a
// first-fit allocator.  Independent branches of the recursion (the two
// triangular solves of an LU step, the two column or row halves of a solve)
// run on streams of their own, forked from and joined back into the
// caller's stream with events; so that no buffer is reused while another
// stream may still read it, buffers and rank slots freed during the
// factorisation return to the allocator only at its end.  The solve runs on
// one stream and frees at once (a later kernel on that stream runs after
// every earlier one).
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/hm_lu.h"
#include "hm_internal.hpp"
#include "hm_lu_internal.hpp"

namespace {

using hm::fail;
using hm::lu::Dim;
using hm::lu::Part;

constexpr size_t kAlign = 256;
constexpr int kForkStreams = 8;    // streams the forked branches of a factorisation take turns on

struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;               // offset -> length
  std::unordered_map<size_t, size_t> live_;     // offset -> length
  void init(char* b, size_t s) {
    base = b;
    size = s / kAlign * kAlign;
    free_.clear();
    free_[0] = size;
  }
  void* alloc(size_t bytes) {
    bytes = std::max<size_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      live_[off] = bytes;
      used += bytes;
      peak = std::max(peak, used);
      return base + off;
    }
    return nullptr;
  }
  // While defer is set, released buffers are only collected (their memory
  // may still be in use by kernels of another stream) and return to the
  // free list at flush(), after every stream has finished.
  bool defer = false;
  std::vector<void*> deferred;
  void flush() {
    defer = false;
    for (void* p : deferred) release(p);
    deferred.clear();
  }
  void release(void* p) {
    if (!p) return;
    if (defer) {
      deferred.push_back(p);
      return;
    }
    const size_t off = (size_t)((char*)p - base);
    auto lv = live_.find(off);
    if (lv == live_.end()) return;
    size_t len = lv->second;
    live_.erase(lv);
    used -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }
};

struct OutOfMemory {};
struct DeviceError { hipError_t e; };

// A matrix over a target t x s (m x n): zero, dense, or a low-rank term
// U V^T at row offsets (see Part).  `own` lists the arena buffers and
// `slot` the rank slot that die with it (empty for a view).
struct Term {
  int kind = 0;                  // 0 zero, 1 dense, 2 low-rank
  int64_t m = 0, n = 0;
  double* D = nullptr;
  int64_t ldd = 0;
  Part p;
  int64_t kcap = 0;
  std::vector<void*> own;
  int32_t slot = -1;
};

struct Leaf {
  int32_t tau = 0, sigma = 0, kind = 0;
  int64_t m = 0, n = 0;
  double* D = nullptr;           // dense: m x n, ld m
  double* U = nullptr;           // low-rank: U (m x cap, ld m), V (n x cap, ld n)
  double* V = nullptr;
  int64_t cap = 0;
  int32_t slot = -1;
  void* blk = nullptr;           // arena buffer holding the leaf's data
};

}  // namespace

struct hm_lu {
  int device = 0;
  int64_t n = 0;
  std::vector<int64_t> beg, end;
  std::vector<int32_t> son0, son1;
  std::vector<Leaf> leaves;
  std::unordered_map<uint64_t, int32_t> at;      // (tau, sigma) -> leaf
  void* mem = nullptr;
  Arena arena;
  int32_t* d_slots = nullptr;                    // rank slots; the last one is the error flag
  int32_t n_slots = 0;
  std::vector<int32_t> free_slots, deferred_slots;
  hipStream_t s = nullptr;                       // the stream work is enqueued on now
  std::vector<hipStream_t> pool;                 // streams for forked branches
  size_t next_stream = 0;
  std::vector<hipEvent_t> fj;                    // fork / join events
  size_t fj_used = 0;
  double eps = 0;
  int dtype = HM_F64;
  int mbits = 52;
  bool factored = false, broken = false;
  int64_t kernels = 0, truncations = 0;
  int32_t max_rank = 0;
  double factor_doubles = 0, stored_bytes = 0;
  // profiling of the truncation kernels (hm_lu_profile)
  bool prof = false;
  std::vector<hipEvent_t> events;
  double* d_flog = nullptr;
  int64_t flog_cap = 0;
  double trunc_ms = 0, trunc_flops = 0;

  // ------------------------------------------------------------ resources
  static uint64_t key(int32_t t, int32_t s2) { return ((uint64_t)(uint32_t)t << 32) | (uint32_t)s2; }
  const Leaf* leaf(int32_t t, int32_t s2) const {
    auto it = at.find(key(t, s2));
    return it == at.end() ? nullptr : &leaves[it->second];
  }
  Leaf* leaf(int32_t t, int32_t s2) {
    auto it = at.find(key(t, s2));
    return it == at.end() ? nullptr : &leaves[it->second];
  }
  int64_t size(int32_t c) const { return end[c] - beg[c]; }
  int64_t rel(int32_t c, int32_t parent) const { return beg[c] - beg[parent]; }
  double* dalloc(int64_t count) {
    void* p = arena.alloc((size_t)std::max<int64_t>(count, 1) * sizeof(double));
    if (!p) throw OutOfMemory{};
    return (double*)p;
  }
  int32_t slot_alloc() {
    if (free_slots.empty()) throw OutOfMemory{};
    const int32_t q = free_slots.back();
    free_slots.pop_back();
    return q;
  }
  void chk(hipError_t e) {             // a kernel launch
    ++kernels;
    if (e != hipSuccess) throw DeviceError{e};
  }
  static void chk_api(hipError_t e) {   // any other enqueued call
    if (e != hipSuccess) throw DeviceError{e};
  }
  void drop(Term& T) {
    for (void* p : T.own) arena.release(p);
    T.own.clear();
    if (T.slot >= 0) release_slot(T.slot);
    T.slot = -1;
    T.kind = 0;
  }
  void release_slot(int32_t q) {
    if (arena.defer) deferred_slots.push_back(q);
    else free_slots.push_back(q);
  }

  // ------------------------------------------------------------ streams
  hipEvent_t event() {
    if (fj_used == fj.size()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) throw DeviceError{hipErrorOutOfMemory};
      fj.push_back(e);
    }
    return fj[fj_used++];
  }
  // A stream for a branch that may run beside the rest of the current
  // stream's work: it starts after everything enqueued so far.
  hipStream_t fork() {
    if (pool.empty()) return s;
    hipStream_t c = pool[next_stream++ % pool.size()];
    if (c == s) c = pool[next_stream++ % pool.size()];
    hipEvent_t e = event();
    chk_api(hipEventRecord(e, s));
    chk_api(hipStreamWaitEvent(c, e, 0));
    return c;
  }
  // The current stream continues after everything enqueued on c so far.
  void join(hipStream_t c) {
    if (c == s) return;
    hipEvent_t e = event();
    chk_api(hipEventRecord(e, c));
    chk_api(hipStreamWaitEvent(s, e, 0));
  }

  // ------------------------------------------------- block times dense panel
  // out (rows of t, ldo) += alpha block(t, s) Z (rows of s, ldz, nc columns)
  void mul(int32_t t, int32_t s2, const double* Z, int64_t ldz, Dim nc, int64_t nccap, double* out, int64_t ldo,
           double alpha) {
    const Leaf* L = leaf(t, s2);
    if (L) {
      if (L->kind == HM_DENSE) {
        chk(hm::lu::gemm(Dim{L->m}, nc, Dim{L->n}, L->m, nccap, alpha, L->D, L->m, 0, Z, ldz, 0, 1.0, out, ldo, s));
      } else {
        double* tmp = dalloc(L->cap * nccap);
        const Dim k{0, d_slots + L->slot, L->cap};
        chk(hm::lu::gemm(k, nc, Dim{L->n}, L->cap, nccap, 1.0, L->V, L->n, 1, Z, ldz, 0, 0.0, tmp, L->cap, s));
        chk(hm::lu::gemm(Dim{L->m}, nc, k, L->m, nccap, alpha, L->U, L->m, 0, tmp, L->cap, 0, 1.0, out, ldo, s));
        arena.release(tmp);
      }
      return;
    }
    for (int32_t ti : {son0[t], son1[t]})
      for (int32_t sj : {son0[s2], son1[s2]})
        mul(ti, sj, Z + rel(sj, s2), ldz, nc, nccap, out + rel(ti, t), ldo, alpha);
  }

  // out (rows of s, ldo) += alpha block(t, s)^T Z (rows of t)
  void mul_t(int32_t t, int32_t s2, const double* Z, int64_t ldz, Dim nc, int64_t nccap, double* out, int64_t ldo,
             double alpha) {
    const Leaf* L = leaf(t, s2);
    if (L) {
      if (L->kind == HM_DENSE) {
        chk(hm::lu::gemm(Dim{L->n}, nc, Dim{L->m}, L->n, nccap, alpha, L->D, L->m, 1, Z, ldz, 0, 1.0, out, ldo, s));
      } else {
        double* tmp = dalloc(L->cap * nccap);
        const Dim k{0, d_slots + L->slot, L->cap};
        chk(hm::lu::gemm(k, nc, Dim{L->m}, L->cap, nccap, 1.0, L->U, L->m, 1, Z, ldz, 0, 0.0, tmp, L->cap, s));
        chk(hm::lu::gemm(Dim{L->n}, nc, k, L->n, nccap, alpha, L->V, L->n, 0, tmp, L->cap, 0, 1.0, out, ldo, s));
        arena.release(tmp);
      }
      return;
    }
    for (int32_t ti : {son0[t], son1[t]})
      for (int32_t sj : {son0[s2], son1[s2]})
        mul_t(ti, sj, Z + rel(ti, t), ldz, nc, nccap, out + rel(sj, s2), ldo, alpha);
  }

  // ------------------------------------------------- H-triangular solves
  void solve_lower(int32_t t, double* Z, int64_t ldz, Dim nc, int64_t nccap) {       // Z := L_tt^-1 Z
    const Leaf* L = leaf(t, t);
    if (L) {
      chk(hm::lu::trsm(L->D, L->m, (int)L->m, 0, Z, ldz, nc, nccap, s));
      return;
    }
    const int32_t t0 = son0[t], t1 = son1[t];
    double* Z0 = Z + rel(t0, t);
    double* Z1 = Z + rel(t1, t);
    solve_lower(t0, Z0, ldz, nc, nccap);
    mul(t1, t0, Z0, ldz, nc, nccap, Z1, ldz, -1.0);
    solve_lower(t1, Z1, ldz, nc, nccap);
  }

  void solve_upper_t(int32_t t, double* Z, int64_t ldz, Dim nc, int64_t nccap) {     // Z := U_tt^-T Z
    const Leaf* L = leaf(t, t);
    if (L) {
      chk(hm::lu::trsm(L->D, L->m, (int)L->m, 1, Z, ldz, nc, nccap, s));
      return;
    }
    const int32_t t0 = son0[t], t1 = son1[t];
    double* Z0 = Z + rel(t0, t);
    double* Z1 = Z + rel(t1, t);
    solve_upper_t(t0, Z0, ldz, nc, nccap);
    mul_t(t0, t1, Z0, ldz, nc, nccap, Z1, ldz, -1.0);
    solve_upper_t(t1, Z1, ldz, nc, nccap);
  }

  void solve_upper(int32_t t, double* Z, int64_t ldz, Dim nc, int64_t nccap) {       // Z := U_tt^-1 Z
    const Leaf* L = leaf(t, t);
    if (L) {
      chk(hm::lu::trsm(L->D, L->m, (int)L->m, 2, Z, ldz, nc, nccap, s));
      return;
    }
    const int32_t t0 = son0[t], t1 = son1[t];
    double* Z0 = Z + rel(t0, t);
    double* Z1 = Z + rel(t1, t);
    solve_upper(t1, Z1, ldz, nc, nccap);
    mul(t0, t1, Z1, ldz, nc, nccap, Z0, ldz, -1.0);
    solve_upper(t0, Z0, ldz, nc, nccap);
  }

  // ------------------------------------------------------------ terms
  Term lowrank_term(int64_t m, int64_t n) {
    Term T;
    T.kind = 2;
    T.m = m;
    T.n = n;
    T.p.urows = m;
    T.p.vrows = n;
    return T;
  }

  // block(t, r) block(r, s) as a low-rank term over t x s
  Term product(int32_t t, int32_t r, int32_t s2) {
    const Leaf* X = leaf(t, r);
    const Leaf* Y = leaf(r, s2);
    const int64_t m = size(t), n = size(s2), nr = size(r);
    Term T = lowrank_term(m, n);
    if (X && X->kind == HM_LOWRANK) {                 // U (Y^T V)^T
      double* Z = dalloc(n * X->cap);
      T.own.push_back(Z);
      chk(hm::lu::fill(Z, n, n, X->cap, 0.0, s));
      const Dim k{0, d_slots + X->slot, X->cap};
      mul_t(r, s2, X->V, nr, k, X->cap, Z, n, 1.0);
      T.p.U = X->U;
      T.p.ldu = m;
      T.p.V = Z;
      T.p.ldv = n;
      T.p.k = k;
      T.kcap = X->cap;
      return T;
    }
    if (Y && Y->kind == HM_LOWRANK) {                 // (X U) V^T
      double* Z = dalloc(m * Y->cap);
      T.own.push_back(Z);
      chk(hm::lu::fill(Z, m, m, Y->cap, 0.0, s));
      const Dim k{0, d_slots + Y->slot, Y->cap};
      mul(t, r, Y->U, nr, k, Y->cap, Z, m, 1.0);
      T.p.U = Z;
      T.p.ldu = m;
      T.p.V = Y->V;
      T.p.ldv = n;
      T.p.k = k;
      T.kcap = Y->cap;
      return T;
    }
    if (X && Y) {                                     // dense X, dense Y: X (Y^T)^T, rank |r|
      T.p.U = X->D;
      T.p.ldu = m;
      T.p.V = Y->D;
      T.p.ldv = nr;
      T.p.vtrans = 1;
      T.p.k = Dim{nr};
      T.kcap = nr;
      return T;
    }
    if (X) {                                          // dense X, t a leaf cluster: I (Y^T X^T)^T
      double* XT = dalloc(nr * m);
      chk(hm::lu::transpose(X->D, m, m, nr, XT, nr, s));
      double* Z = dalloc(n * m);
      T.own.push_back(Z);
      chk(hm::lu::fill(Z, n, n, m, 0.0, s));
      mul_t(r, s2, XT, nr, Dim{m}, m, Z, n, 1.0);
      arena.release(XT);
      T.p.U = nullptr;
      T.p.V = Z;
      T.p.ldv = n;
      T.p.k = Dim{m};
      T.kcap = m;
      return T;
    }
    if (Y) {                                          // dense Y, s a leaf cluster: (X Y) I
      double* Z = dalloc(m * n);
      T.own.push_back(Z);
      chk(hm::lu::fill(Z, m, m, n, 0.0, s));
      mul(t, r, Y->D, nr, Dim{n}, n, Z, m, 1.0);
      T.p.U = Z;
      T.p.ldu = m;
      T.p.V = nullptr;
      T.p.k = Dim{n};
      T.kcap = n;
      return T;
    }
    // no leaf factor: the sons' products placed at their offsets, each added with truncation
    Term acc;
    acc.m = m;
    acc.n = n;
    for (int32_t ti : {son0[t], son1[t]})
      for (int32_t sj : {son0[s2], son1[s2]})
        for (int32_t rl : {son0[r], son1[r]}) {
          Term sub = product(ti, rl, sj);
          sub.m = m;
          sub.n = n;
          sub.p.uoff += rel(ti, t);
          sub.p.voff += rel(sj, s2);
          acc = add(acc, sub, false);
        }
    return acc;
  }

  // one truncation kernel; with profiling, HIP events around it and its
  // arithmetic in the flop log
  void run_trunc(const Part& p0, const Part& p1, int64_t m, int64_t n, double* scr, double* W, double* X,
                 int32_t* rank_out) {
    double* flog = nullptr;
    if (prof && d_flog && truncations < flog_cap) flog = d_flog + truncations;
    const bool timed = prof && truncations < flog_cap;
    if (timed) {
      while ((size_t)(2 * truncations + 2) > events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) throw DeviceError{hipErrorOutOfMemory};
        events.push_back(e);
      }
      chk_api(hipEventRecord(events[2 * truncations], s));
    }
    chk(hm::lu::trunc(p0, p1, m, n, eps, scr, W, X, rank_out, d_slots + n_slots, flog, s));
    if (timed) chk_api(hipEventRecord(events[2 * truncations + 1], s));
    ++truncations;
  }

  Part part_of(const Term& T, double sign) const {
    Part p = T.p;
    p.sign = sign;
    if (T.kind == 0) {
      p = Part{};
      p.k = Dim{0};
    }
    return p;
  }

  // acc + term (both over the same m x n target); consumes both
  Term add(Term& acc, Term& term, bool dense) {
    const int64_t m = acc.m, n = acc.n;
    Term out;
    out.m = m;
    out.n = n;
    if (dense) {
      if (acc.kind == 1) {
        out = acc;
        acc.own.clear();
        acc.kind = 0;
      } else {
        out.kind = 1;
        out.D = dalloc(m * n);
        out.ldd = m;
        out.own.push_back(out.D);
        chk(hm::lu::fill(out.D, m, m, n, 0.0, s));
      }
      add_dense(out, term);
      drop(term);
      return out;
    }
    const int64_t capsum = (acc.kind == 2 ? acc.kcap : 0) + term.kcap;
    const int64_t capo = std::min<int64_t>({(int64_t)hm::lu::kMaxTrunc, m, n, capsum});
    double* scr = dalloc(hm::lu::trunc_scratch(m, n, capsum));
    double* W = dalloc((m + n) * std::max<int64_t>(capo, 1));
    out.kind = 2;
    out.p.U = W;
    out.p.ldu = m;
    out.p.urows = m;
    out.p.V = W + m * std::max<int64_t>(capo, 1);
    out.p.ldv = n;
    out.p.vrows = n;
    out.slot = slot_alloc();
    out.p.k = Dim{0, d_slots + out.slot, capo};
    out.kcap = capo;
    out.own.push_back(W);
    run_trunc(part_of(acc, 1.0), part_of(term, 1.0), m, n, scr, W, W + m * std::max<int64_t>(capo, 1),
              d_slots + out.slot);
    arena.release(scr);
    drop(acc);
    drop(term);
    return out;
  }

  // dense D (over the target) += alpha U V^T of a low-rank term
  void add_dense(Term& D, const Term& T, double alpha = 1.0) {
    if (T.kind != 2) return;
    double* dst = D.D + T.p.voff * D.ldd + T.p.uoff;
    const Part& p = T.p;
    double* eye = nullptr;
    const double* U = p.U;
    const double* V = p.V;
    int64_t ldu = p.ldu, ldv = p.ldv;
    if (!U) {
      eye = dalloc(p.urows * p.urows);
      chk(hm::lu::eye(eye, p.urows, p.urows, s));
      U = eye;
      ldu = p.urows;
    } else if (!V) {
      eye = dalloc(p.vrows * p.vrows);
      chk(hm::lu::eye(eye, p.vrows, p.vrows, s));
      V = eye;
      ldv = p.vrows;
    }
    chk(hm::lu::gemm(Dim{p.urows}, Dim{p.vrows}, p.k, p.urows, p.vrows, alpha, U, ldu, 0, V, ldv, p.vtrans ? 0 : 1,
                     1.0, dst, D.ldd, s));
    arena.release(eye);
  }

  bool dense_target(int32_t t, int32_t s2) const {
    const Leaf* L = leaf(t, s2);
    return L && L->kind == HM_DENSE;
  }

  using Pend = std::vector<std::array<int32_t, 3>>;

  void gather(int32_t t, int32_t s2, Term& acc, Pend& pend) {
    const bool at_leaf = leaf(t, s2) != nullptr;
    const bool dense = dense_target(t, s2);
    Pend rest;
    for (const auto& q : pend) {
      if (at_leaf || leaf(q[0], q[1]) || leaf(q[1], q[2])) {
        Term term = product(q[0], q[1], q[2]);
        term.m = acc.m;
        term.n = acc.n;
        acc = add(acc, term, dense);
      } else {
        rest.push_back(q);
      }
    }
    pend.swap(rest);
  }

  struct Sub {
    Term acc;
    Pend pend;
  };

  void split(int32_t t, int32_t s2, const Term& acc, const Pend& pend, Sub sub[2][2]) {
    const int32_t ts[2] = {son0[t], son1[t]}, ss[2] = {son0[s2], son1[s2]};
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        Sub& q = sub[i][j];
        const int32_t ti = ts[i], sj = ss[j];
        q.acc = Term{};
        q.acc.m = size(ti);
        q.acc.n = size(sj);
        if (acc.kind == 2) {                          // a view of the parent's accumulator
          Term v = lowrank_term(size(ti), size(sj));
          v.p.U = acc.p.U + rel(ti, t);
          v.p.ldu = acc.p.ldu;
          v.p.V = acc.p.V + rel(sj, s2);
          v.p.ldv = acc.p.ldv;
          v.p.k = acc.p.k;
          v.kcap = acc.kcap;
          if (dense_target(ti, sj)) {
            Term d;
            d.m = size(ti);
            d.n = size(sj);
            d.kind = 1;
            d.D = dalloc(d.m * d.n);
            d.ldd = d.m;
            d.own.push_back(d.D);
            chk(hm::lu::fill(d.D, d.m, d.m, d.n, 0.0, s));
            add_dense(d, v);
            q.acc = d;
          } else {
            q.acc = v;
          }
        }
        q.pend.clear();
        for (const auto& p : pend)
          for (int32_t rl : {son0[p[1]], son1[p[1]]}) q.pend.push_back({ti, rl, sj});
      }
  }

  // leaf (t, s) -= acc
  void apply(Leaf& B, Term& acc) {
    if (acc.kind == 0) return;
    if (B.kind == HM_DENSE) {
      if (acc.kind == 1) {
        chk(hm::lu::axpy(B.m, B.n, -1.0, acc.D, acc.ldd, B.D, B.m, s));
      } else {
        Term d;
        d.kind = 1;
        d.D = B.D;
        d.ldd = B.m;
        add_dense(d, acc, -1.0);
      }
      drop(acc);
      return;
    }
    if (acc.kind == 1) throw DeviceError{hipErrorInvalidValue};   // never: low-rank leaves get low-rank sums
    Term cur = lowrank_term(B.m, B.n);
    cur.p.U = B.U;
    cur.p.ldu = B.m;
    cur.p.V = B.V;
    cur.p.ldv = B.n;
    cur.p.k = Dim{0, d_slots + B.slot, B.cap};
    cur.kcap = B.cap;
    Term a2 = acc;
    const int64_t capsum = B.cap + acc.kcap;
    const int64_t capo = std::min<int64_t>({(int64_t)hm::lu::kMaxTrunc, B.m, B.n, capsum});
    double* scr = dalloc(hm::lu::trunc_scratch(B.m, B.n, capsum));
    double* W = dalloc((B.m + B.n) * std::max<int64_t>(capo, 1));
    const int32_t slot = slot_alloc();
    run_trunc(part_of(cur, 1.0), part_of(a2, -1.0), B.m, B.n, scr, W, W + B.m * std::max<int64_t>(capo, 1),
              d_slots + slot);
    arena.release(scr);
    arena.release(B.blk);
    release_slot(B.slot);
    B.blk = W;
    B.U = W;
    B.V = W + B.m * std::max<int64_t>(capo, 1);
    B.cap = capo;
    B.slot = slot;
    drop(acc);
  }

  void finalize(Leaf& B) {
    if (dtype == HM_F64) return;
    if (B.kind == HM_DENSE) {
      chk(hm::lu::round_dfl(B.D, B.m, B.m, Dim{B.n}, B.n, mbits, s));
    } else {
      const Dim k{0, d_slots + B.slot, B.cap};
      chk(hm::lu::round_dfl(B.U, B.m, B.m, k, B.cap, mbits, s));
      chk(hm::lu::round_dfl(B.V, B.n, B.n, k, B.cap, mbits, s));
    }
  }

  // ------------------------------------------------------------ recursion
  void lu(int32_t t, Term acc, Pend pend) {
    gather(t, t, acc, pend);
    Leaf* B = leaf(t, t);
    if (B) {
      apply(*B, acc);
      chk(hm::lu::getrf(B->D, B->m, (int)B->m, s));
      finalize(*B);
      return;
    }
    Sub sub[2][2];
    split(t, t, acc, pend, sub);
    const int32_t t0 = son0[t], t1 = son1[t];
    lu(t0, std::move(sub[0][0].acc), std::move(sub[0][0].pend));
    // the two solves are independent: U01 here, L10 on a forked stream
    const hipStream_t here = s, c = fork();
    solve_l(t0, t1, std::move(sub[0][1].acc), std::move(sub[0][1].pend));
    s = c;
    solve_u(t1, t0, std::move(sub[1][0].acc), std::move(sub[1][0].pend));
    s = here;
    join(c);
    sub[1][1].pend.push_back({t1, t0, t1});
    lu(t1, std::move(sub[1][1].acc), std::move(sub[1][1].pend));
    drop(acc);
  }

  void solve_l(int32_t t, int32_t s2, Term acc, Pend pend) {    // block(t, s) := L_tt^-1 (block - updates)
    gather(t, s2, acc, pend);
    Leaf* B = leaf(t, s2);
    if (B) {
      apply(*B, acc);
      if (B->kind == HM_DENSE) solve_lower(t, B->D, B->m, Dim{B->n}, B->n);
      else solve_lower(t, B->U, B->m, Dim{0, d_slots + B->slot, B->cap}, B->cap);
      finalize(*B);
      return;
    }
    Sub sub[2][2];
    split(t, s2, acc, pend, sub);
    const int32_t t0 = son0[t], t1 = son1[t];
    const int32_t ss[2] = {son0[s2], son1[s2]};
    // the two column halves are independent: the second on a forked stream
    const hipStream_t here = s, c = fork();
    for (int j = 0; j < 2; ++j) {
      s = j == 0 ? here : c;
      solve_l(t0, ss[j], std::move(sub[0][j].acc), std::move(sub[0][j].pend));
      sub[1][j].pend.push_back({t1, t0, ss[j]});
      solve_l(t1, ss[j], std::move(sub[1][j].acc), std::move(sub[1][j].pend));
    }
    s = here;
    join(c);
    drop(acc);
  }

  void solve_u(int32_t t, int32_t s2, Term acc, Pend pend) {    // block(t, s) := (block - updates) U_ss^-1
    gather(t, s2, acc, pend);
    Leaf* B = leaf(t, s2);
    if (B) {
      apply(*B, acc);
      if (B->kind == HM_DENSE) {
        double* DT = dalloc(B->n * B->m);
        chk(hm::lu::transpose(B->D, B->m, B->m, B->n, DT, B->n, s));
        solve_upper_t(s2, DT, B->n, Dim{B->m}, B->m);
        chk(hm::lu::transpose(DT, B->n, B->n, B->m, B->D, B->m, s));
        arena.release(DT);
      } else {
        solve_upper_t(s2, B->V, B->n, Dim{0, d_slots + B->slot, B->cap}, B->cap);
      }
      finalize(*B);
      return;
    }
    Sub sub[2][2];
    split(t, s2, acc, pend, sub);
    const int32_t s0 = son0[s2], s1 = son1[s2];
    const int32_t ts[2] = {son0[t], son1[t]};
    // the two row halves are independent: the second on a forked stream
    const hipStream_t here = s, c = fork();
    for (int i = 0; i < 2; ++i) {
      s = i == 0 ? here : c;
      solve_u(ts[i], s0, std::move(sub[i][0].acc), std::move(sub[i][0].pend));
      sub[i][1].pend.push_back({ts[i], s0, s1});
      solve_u(ts[i], s1, std::move(sub[i][1].acc), std::move(sub[i][1].pend));
    }
    s = here;
    join(c);
    drop(acc);
  }
};

namespace {

// Checks that the leaves tile the block tree of the cluster tree: every
// recursion path from (0, 0) ends in exactly one leaf, and no leaf is left.
bool tiles(const hm_lu* F, int32_t t, int32_t s2, int64_t& seen) {
  if (F->leaf(t, s2)) {
    ++seen;
    return true;
  }
  if (F->son0[t] < 0 || F->son0[s2] < 0) return false;
  for (int32_t ti : {F->son0[t], F->son1[t]})
    for (int32_t sj : {F->son0[s2], F->son1[s2]})
      if (!tiles(F, ti, sj, seen)) return false;
  return true;
}

int dfl_mbits(int32_t dt) {
  switch (dt) {
    case HM_DFL16: return 4;
    case HM_DFL24: return 12;
    case HM_DFL32: return 20;
    case HM_DFL40: return 28;
    case HM_DFL48: return 36;
    default: return -1;
  }
}

}  // namespace

extern "C" {

hm_status hm_lu_create(const hm_lu_tree* tree, int64_t n_leaves, const int32_t* tau, const int32_t* sigma,
                       const int32_t* kind, const int32_t* rank, const double* const* h_a,
                       const double* const* h_b, size_t arena_bytes, hm_lu** out) {
  if (!out) return fail(HM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tree || !tree->begin || !tree->end || !tree->son0 || !tree->son1 || tree->n_clusters < 1)
    return fail(HM_EINVAL, "bad cluster tree");
  if (n_leaves < 1 || !tau || !sigma || !kind || !rank || !h_a || !h_b) return fail(HM_EINVAL, "bad leaves");
  std::unique_ptr<hm_lu> F(new hm_lu());
  const int64_t nc = tree->n_clusters;
  F->beg.assign(tree->begin, tree->begin + nc);
  F->end.assign(tree->end, tree->end + nc);
  F->son0.assign(tree->son0, tree->son0 + nc);
  F->son1.assign(tree->son1, tree->son1 + nc);
  F->n = F->end[0] - F->beg[0];
  if (F->beg[0] != 0 || F->n <= 0) return fail(HM_EINVAL, "the root must span [0, n)");
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t a = F->son0[c], b = F->son1[c];
    if ((a < 0) != (b < 0)) return fail(HM_EINVAL, "cluster %lld: one son", (long long)c);
    if (a < 0) continue;
    if (a >= nc || b >= nc || F->beg[a] != F->beg[c] || F->end[a] != F->beg[b] || F->end[b] != F->end[c] ||
        F->beg[a] >= F->end[a] || F->beg[b] >= F->end[b])
      return fail(HM_EINVAL, "cluster %lld: sons do not split it", (long long)c);
  }
  F->leaves.resize((size_t)n_leaves);
  size_t need = 0;
  for (int64_t i = 0; i < n_leaves; ++i) {
    Leaf& L = F->leaves[i];
    L.tau = tau[i];
    L.sigma = sigma[i];
    if (L.tau < 0 || L.tau >= nc || L.sigma < 0 || L.sigma >= nc) return fail(HM_EINVAL, "leaf %lld: cluster", (long long)i);
    L.kind = kind[i];
    L.m = F->size(L.tau);
    L.n = F->size(L.sigma);
    if (L.kind != HM_DENSE && L.kind != HM_LOWRANK) return fail(HM_EINVAL, "leaf %lld: kind", (long long)i);
    if (L.tau == L.sigma && (L.kind != HM_DENSE || L.m > HM_LU_MAX_LEAF))
      return fail(HM_ESHAPE, "diagonal leaf %lld must be dense with at most %d rows", (long long)i, HM_LU_MAX_LEAF);
    if (L.kind == HM_LOWRANK && (rank[i] < 0 || rank[i] > std::min(L.m, L.n)))
      return fail(HM_ESHAPE, "leaf %lld: rank %d", (long long)i, rank[i]);
    if (!h_a[i] || (L.kind == HM_LOWRANK && rank[i] > 0 && !h_b[i])) return fail(HM_EINVAL, "leaf %lld: data", (long long)i);
    if (!F->at.emplace(hm_lu::key(L.tau, L.sigma), (int32_t)i).second)
      return fail(HM_EPARTITION, "leaf %lld repeats a block", (long long)i);
    need += (L.kind == HM_DENSE ? L.m * L.n : (L.m + L.n) * std::max(rank[i], 1)) * sizeof(double);
  }
  int64_t seen = 0;
  if (!tiles(F.get(), 0, 0, seen) || seen != n_leaves)
    return fail(HM_EPARTITION, "the leaves do not tile the block tree");
  if (hipGetDevice(&F->device) != hipSuccess) return fail(HM_EDEVICE, "hipGetDevice");
  if (hm::lu::trunc_lds_limit() < hm::lu::kMaxTrunc)
    return fail(HM_EDEVICE, "the device's LDS holds no %d-wide truncation", hm::lu::kMaxTrunc);
  if (hipError_t e = hm::lu::prepare_trunc(); e != hipSuccess) return fail(HM_EDEVICE, "%s", hipGetErrorString(e));
  F->n_slots = (int32_t)std::min<int64_t>(4 * n_leaves + (1 << 20), (int64_t)1 << 28);
  if (arena_bytes < need + ((size_t)F->n_slots + 1) * 4 + (1 << 20))
    return fail(HM_ENOMEM, "arena of %zu bytes below the %zu bytes of the leaves", arena_bytes, need);
  if (hipMalloc(&F->mem, arena_bytes) != hipSuccess) return fail(HM_ENOMEM, "hipMalloc(%zu)", arena_bytes);
  const size_t slot_bytes = (((size_t)F->n_slots + 1) * 4 + kAlign - 1) / kAlign * kAlign;
  F->d_slots = (int32_t*)F->mem;
  F->arena.init((char*)F->mem + slot_bytes, arena_bytes - slot_bytes);
  F->free_slots.reserve(F->n_slots);
  for (int32_t q = F->n_slots - 1; q >= 0; --q) F->free_slots.push_back(q);
  std::vector<int32_t> init_rank((size_t)F->n_slots + 1, 0);
  try {
    for (int64_t i = 0; i < n_leaves; ++i) {
      Leaf& L = F->leaves[i];
      if (L.kind == HM_DENSE) {
        L.D = F->dalloc(L.m * L.n);
        L.blk = L.D;
        if (hipMemcpy(L.D, h_a[i], sizeof(double) * L.m * L.n, hipMemcpyHostToDevice) != hipSuccess)
          throw DeviceError{hipErrorInvalidValue};
      } else {
        L.cap = std::max(rank[i], 1);
        L.U = F->dalloc((L.m + L.n) * L.cap);
        L.blk = L.U;
        L.V = L.U + L.m * L.cap;
        L.slot = F->slot_alloc();
        init_rank[L.slot] = rank[i];
        if (rank[i] > 0 &&
            (hipMemcpy(L.U, h_a[i], sizeof(double) * L.m * rank[i], hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(L.V, h_b[i], sizeof(double) * L.n * rank[i], hipMemcpyHostToDevice) != hipSuccess))
          throw DeviceError{hipErrorInvalidValue};
      }
    }
  } catch (const OutOfMemory&) {
    (void)hipFree(F->mem);
    return fail(HM_ENOMEM, "arena too small for the leaves");
  } catch (const DeviceError& e) {
    (void)hipFree(F->mem);
    return fail(HM_EDEVICE, "upload: %s", hipGetErrorString(e.e));
  }
  if (hipMemcpy(F->d_slots, init_rank.data(), init_rank.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(F->mem);
    return fail(HM_EDEVICE, "upload of the ranks");
  }
  *out = F.release();
  return HM_OK;
}

hm_status hm_lu_factor(hm_lu* F, double eps, int32_t dtype, void* stream) {
  if (!F) return fail(HM_EINVAL, "F is NULL");
  if (F->factored || F->broken) return fail(HM_ESTATE, "already factorised (or failed)");
  if (!(eps > 0)) return fail(HM_EINVAL, "eps must be > 0");
  if (dtype != HM_F64 && dfl_mbits(dtype) < 0) return fail(HM_EDTYPE, "dtype %d: HM_F64 or a DFL format", dtype);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != F->device) return fail(HM_EDEVICE, "not the object's device");
  F->eps = eps;
  F->dtype = dtype;
  F->mbits = dtype == HM_F64 ? 52 : dfl_mbits(dtype);
  F->s = (hipStream_t)stream;
  F->kernels = F->truncations = 0;
  F->trunc_ms = F->trunc_flops = 0;
  if (F->prof) {                          // a flop log of up to 2^21 truncations, if the arena has room
    F->flog_cap = (int64_t)1 << 21;
    F->d_flog = (double*)F->arena.alloc((size_t)F->flog_cap * sizeof(double));
    if (!F->d_flog) F->flog_cap = 0;
  }
  // streams for the forked branches (default priority), and deferred frees
  F->pool.clear();
  for (int q = 0; q < kForkStreams; ++q) {
    hipStream_t c;
    if (hipStreamCreateWithFlags(&c, hipStreamNonBlocking) != hipSuccess) break;
    F->pool.push_back(c);
  }
  F->next_stream = 0;
  F->fj_used = 0;
  F->arena.defer = true;
  auto finish = [&]() {                   // every stream done; frees and streams released
    for (hipStream_t c : F->pool) (void)hipStreamSynchronize(c);
    (void)hipStreamSynchronize(F->s);
    for (hipStream_t c : F->pool) (void)hipStreamDestroy(c);
    F->pool.clear();
    F->arena.flush();
    for (int32_t q : F->deferred_slots) F->free_slots.push_back(q);
    F->deferred_slots.clear();
  };
  try {
    F->lu(0, Term{0, F->n, F->n}, {});
  } catch (const OutOfMemory&) {
    F->broken = true;
    finish();
    return fail(HM_ENOMEM, "arena exhausted (peak %zu of %zu bytes)", F->arena.peak, F->arena.size);
  } catch (const DeviceError& e) {
    F->broken = true;
    finish();
    return fail(HM_EDEVICE, "launch: %s", hipGetErrorString(e.e));
  }
  int32_t err = 0;
  const hipError_t ce = hipMemcpyAsync(&err, F->d_slots + F->n_slots, 4, hipMemcpyDeviceToHost, F->s);
  finish();
  if (ce != hipSuccess || hipGetLastError() != hipSuccess) {
    F->broken = true;
    return fail(HM_EDEVICE, "factorisation: %s", hipGetErrorString(ce));
  }
  if (err) {
    F->broken = true;
    return fail(HM_ERANK, "a truncation needed more than %d columns", HM_LU_MAX_RANK);
  }
  if (F->prof) {
    const int64_t nt = std::min(F->truncations, F->flog_cap);
    for (int64_t q = 0; q < nt; ++q) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, F->events[2 * q], F->events[2 * q + 1]) == hipSuccess) F->trunc_ms += ms;
    }
    std::vector<double> fl((size_t)nt);
    if (nt > 0 && hipMemcpy(fl.data(), F->d_flog, nt * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess)
      for (double v : fl) F->trunc_flops += v;
    F->arena.release(F->d_flog);
    F->d_flog = nullptr;
  }
  // statistics: ranks of the low-rank leaves
  std::vector<int32_t> rk((size_t)F->n_slots);
  if (hipMemcpy(rk.data(), F->d_slots, rk.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(HM_EDEVICE, "ranks");
  F->max_rank = 0;
  F->factor_doubles = 0;
  for (const Leaf& L : F->leaves) {
    if (L.kind == HM_DENSE) {
      F->factor_doubles += (double)L.m * L.n;
    } else {
      F->max_rank = std::max(F->max_rank, rk[L.slot]);
      F->factor_doubles += (double)(L.m + L.n) * rk[L.slot];
    }
  }
  F->stored_bytes = F->factor_doubles * (dtype == HM_F64 ? 8.0 : (F->mbits + 12) / 8.0);
  F->factored = true;
  return HM_OK;
}

hm_status hm_lu_solve(hm_lu* F, double* d_x, int64_t ld, int64_t nrhs, void* stream) {
  if (!F || !d_x) return fail(HM_EINVAL, "NULL argument");
  if (!F->factored) return fail(HM_ESTATE, "not factorised");
  if (nrhs < 0 || ld < F->n) return fail(HM_EINVAL, "nrhs %lld, ld %lld", (long long)nrhs, (long long)ld);
  if (nrhs == 0) return HM_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != F->device) return fail(HM_EDEVICE, "not the object's device");
  F->s = (hipStream_t)stream;
  try {
    F->solve_lower(0, d_x, ld, Dim{nrhs}, nrhs);
    F->solve_upper(0, d_x, ld, Dim{nrhs}, nrhs);
  } catch (const OutOfMemory&) {
    return fail(HM_ENOMEM, "arena exhausted");
  } catch (const DeviceError& e) {
    return fail(HM_EDEVICE, "launch: %s", hipGetErrorString(e.e));
  }
  return HM_OK;
}

hm_status hm_lu_leaf(hm_lu* F, int64_t i, int32_t* rank, double* h_a, size_t a_doubles, double* h_b,
                     size_t b_doubles) {
  if (!F || !rank) return fail(HM_EINVAL, "NULL argument");
  if (i < 0 || i >= (int64_t)F->leaves.size()) return fail(HM_EINVAL, "leaf %lld", (long long)i);
  const Leaf& L = F->leaves[i];
  if (hipDeviceSynchronize() != hipSuccess) return fail(HM_EDEVICE, "synchronize");
  if (L.kind == HM_DENSE) {
    *rank = 0;
    if (a_doubles < (size_t)(L.m * L.n) || !h_a) return fail(HM_ENOMEM, "room for %lld doubles", (long long)(L.m * L.n));
    if (hipMemcpy(h_a, L.D, sizeof(double) * L.m * L.n, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(HM_EDEVICE, "copy");
    return HM_OK;
  }
  int32_t k = 0;
  if (hipMemcpy(&k, F->d_slots + L.slot, 4, hipMemcpyDeviceToHost) != hipSuccess) return fail(HM_EDEVICE, "rank");
  *rank = k;
  if (a_doubles < (size_t)(L.m * k) || b_doubles < (size_t)(L.n * k) || (k > 0 && (!h_a || !h_b)))
    return fail(HM_ENOMEM, "room for %lld + %lld doubles", (long long)(L.m * k), (long long)(L.n * k));
  if (k > 0 && (hipMemcpy(h_a, L.U, sizeof(double) * L.m * k, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(h_b, L.V, sizeof(double) * L.n * k, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(HM_EDEVICE, "copy");
  return HM_OK;
}

hm_status hm_lu_stats_get(const hm_lu* F, hm_lu_stats* st) {
  if (!F || !st) return fail(HM_EINVAL, "NULL argument");
  std::memset(st, 0, sizeof(*st));
  st->kernels = F->kernels;
  st->truncations = F->truncations;
  st->max_rank = F->max_rank;
  st->factor_doubles = F->factor_doubles;
  st->stored_bytes = F->stored_bytes;
  st->arena_peak = F->arena.peak;
  st->trunc_ms = F->trunc_ms;
  st->trunc_flops = F->trunc_flops;
  st->timed_truncations = F->prof ? std::min(F->truncations, F->flog_cap) : 0;
  return HM_OK;
}

hm_status hm_lu_profile(hm_lu* F, int32_t on) {
  if (!F) return fail(HM_EINVAL, "F is NULL");
  F->prof = on != 0;
  return HM_OK;
}

void hm_lu_destroy(hm_lu* F) {
  if (!F) return;
  for (hipEvent_t e : F->events) (void)hipEventDestroy(e);
  for (hipEvent_t e : F->fj) (void)hipEventDestroy(e);
  if (F->mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(F->mem);
  }
  delete F;
}

}  // extern "C"
