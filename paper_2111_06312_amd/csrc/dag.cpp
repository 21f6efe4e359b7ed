// Evaluator of symbolic design matrices (Section 4 and the appendix on
// symbolic representation).
//
// A product M G is computed by flattening M into a chain of factors applied
// to G from the right: products are inlined, transposes pushed down to the
// leaves ((AB)^T = B^T A^T, sums and concatenations transposed termwise),
// scalars collected into one coefficient.  A chain atom is a leaf (sparse,
// dense, diagonal), a row selection (the gather), a row slice of the block
// below it (a part of a column concatenation), or a sum / concatenation whose
// terms are chains of their own, continued by the rest of the enclosing
// chain.  A diagonal next to a sparse leaf becomes the row or column scale
// of that leaf's sparse pass (groups formed from the right end of the chain,
// so that equal suffixes are grouped alike).  With the lazy cache, the result of every
// chain suffix times G is kept until the product is done and looked up by
// the ordered list of its factors (the appendix's cache key), so shared
// suffixes (t, t@t, t@t@t; the terms of a sum that end alike) are
// multiplied once.
#include "dag.h"

#include <algorithm>
#include <map>
#include <tuple>

namespace isvd {

namespace {

struct Atom {
  enum Kind { Node, Select, Slice } kind = Node;
  int64_t node = 0;
  bool t = false;
  int part = 0;  // Slice: index of the concatenation part
  bool operator<(const Atom& o) const {
    return std::tie(kind, node, t, part) < std::tie(o.kind, o.node, o.t, o.part);
  }
};
using Chain = std::vector<Atom>;

}  // namespace

struct DagEval {
  std::shared_ptr<const std::vector<std::unique_ptr<DagNode>>> nodes;  // shared with the DAG
  int64_t root = 0;
  bool cache_on = true;
  // block pool (grown on demand, kept between products)
  std::vector<std::unique_ptr<DevBuf>> pool;
  std::vector<char> busy;
  DevBuf gram_c, gram_work;
};

namespace {

template <typename T>
struct View {
  T* p = nullptr;
  int64_t ld = 0, rows = 0;
  int owner = -1;  // pool slot the caller must release, -1: borrowed (input or cache)
};

const DagNode& node_of(const DagEval& ev, int64_t id) { return *(*ev.nodes)[static_cast<size_t>(id)]; }

// Rows of the result of applying an atom (a factor of the chain).
int64_t out_rows(const DagEval& ev, const Atom& a) {
  const DagNode& n = node_of(ev, a.node);
  if (a.kind == Atom::Select) return a.t ? node_of(ev, n.kids[0]).rows : n.nsub;
  if (a.kind == Atom::Slice) return node_of(ev, n.kids[static_cast<size_t>(a.part)]).cols;
  return a.t ? n.cols : n.rows;
}

void flatten(const DagEval& ev, int64_t id, bool t, Chain& out, double& coef) {
  const DagNode& n = node_of(ev, id);
  switch (n.kind) {
    case DagKind::Transpose: flatten(ev, n.kids[0], !t, out, coef); return;
    case DagKind::Product:
      if (!t) {
        for (int64_t k : n.kids) flatten(ev, k, false, out, coef);
      } else {
        for (auto it = n.kids.rbegin(); it != n.kids.rend(); ++it) flatten(ev, *it, true, out, coef);
      }
      return;
    case DagKind::Sum:
      if (n.kids.size() == 1) {
        coef *= n.w[0];
        flatten(ev, n.kids[0], t, out, coef);
        return;
      }
      out.push_back({Atom::Node, id, t, 0});
      return;
    case DagKind::Gather:
      // M[rows, :] G = S (M G) with the row selector S; (S M)^T = M^T S^T
      if (!t) {
        out.push_back({Atom::Select, id, false, 0});
        flatten(ev, n.kids[0], false, out, coef);
      } else {
        flatten(ev, n.kids[0], true, out, coef);
        out.push_back({Atom::Select, id, true, 0});
      }
      return;
    case DagKind::Diag: out.push_back({Atom::Node, id, false, 0}); return;  // symmetric
    default: out.push_back({Atom::Node, id, t, 0}); return;
  }
}

template <typename T>
class Evaluator {
 public:
  Evaluator(DagEval& ev, const T* G, int64_t ldg, int64_t g_rows, int l, hipStream_t s)
      : ev_(ev), G_(G), ldg_(ldg), g_rows_(g_rows), l_(l), ldb_(round_up(l, 8)), s_(s) {}

  ~Evaluator() {
    // every slot is free again once the product is done (cached ones included)
    std::fill(ev_.busy.begin(), ev_.busy.end(), 0);
  }

  View<T> eval(const Chain& chain, size_t pos) {
    if (pos == chain.size()) return View<T>{const_cast<T*>(G_), ldg_, g_rows_, -1};
    Chain key;
    if (ev_.cache_on) {
      key.assign(chain.begin() + static_cast<std::ptrdiff_t>(pos), chain.end());
      auto it = cache_.find(key);
      if (it != cache_.end()) return it->second;
    }
    View<T> r = compute(chain, pos);
    if (ev_.cache_on) {
      // the slot stays busy until the product is done; callers see a borrowed view
      View<T> held = r;
      held.owner = -1;
      cache_.emplace(std::move(key), held);
      return held;
    }
    return r;
  }

  void release(const View<T>& v) {
    if (v.owner >= 0) ev_.busy[static_cast<size_t>(v.owner)] = 0;
  }

  View<T> acquire(int64_t rows) {
    const size_t bytes = static_cast<size_t>(std::max<int64_t>(rows, 1)) * ldb_ * sizeof(T);
    int pick = -1;
    for (size_t i = 0; i < ev_.pool.size(); ++i) {
      if (ev_.busy[i]) continue;
      if (ev_.pool[i]->bytes >= bytes) {
        pick = static_cast<int>(i);
        break;
      }
      if (pick < 0) pick = static_cast<int>(i);  // a free slot to grow
    }
    if (pick < 0) {
      ev_.pool.push_back(std::make_unique<DevBuf>());
      ev_.busy.push_back(0);
      pick = static_cast<int>(ev_.pool.size() - 1);
    }
    ev_.pool[static_cast<size_t>(pick)]->ensure(bytes);
    ev_.busy[static_cast<size_t>(pick)] = 1;
    return View<T>{ev_.pool[static_cast<size_t>(pick)]->template as<T>(), ldb_, rows, pick};
  }

 private:
  using C = typename ComputeOf<T>::type;

  bool is_kind(const Chain& c, size_t i, DagKind k) const {
    return i < c.size() && c[i].kind == Atom::Node && node_of(ev_, c[i].node).kind == k;
  }

  // Length of the factor group that starts at `pos`.  Groups are formed from
  // the right end of the chain, so a suffix is grouped the same way whatever
  // precedes it and cached suffix results are found again: a sparse leaf
  // takes the diagonal on its left as its row scale; a diagonal with a
  // sparse leaf on its left becomes that leaf's column scale, and the group
  // also takes a diagonal further left as row scale unless that one sits
  // right of another sparse leaf (D A D A: (D A)(D A); A D A D: (A D)(A D);
  // R A R R A R: (R A R)(R A R)).  Everything else is a group of one.
  size_t unit_length(const Chain& c, size_t pos) const {
    std::vector<size_t> len(c.size(), 0);
    auto diag = [&](std::ptrdiff_t i) { return i >= 0 && is_kind(c, static_cast<size_t>(i), DagKind::Diag); };
    auto sparse = [&](std::ptrdiff_t i) { return i >= 0 && is_kind(c, static_cast<size_t>(i), DagKind::Sparse); };
    std::ptrdiff_t i = static_cast<std::ptrdiff_t>(c.size()) - 1;
    while (i >= 0) {
      std::ptrdiff_t st = i;
      if (diag(i) && sparse(i - 1)) {
        st = i - 1;
        if (diag(st - 1) && !sparse(st - 2)) st -= 1;
      } else if (sparse(i)) {
        if (diag(i - 1)) st = i - 1;
      }
      len[static_cast<size_t>(st)] = static_cast<size_t>(i - st + 1);
      i = st - 1;
    }
    ISVD_CHECK(len[pos] > 0, ISVD_E_INVALID, "dag: evaluation inside a factor group");
    return len[pos];
  }

  const C* diag_vals(const DagNode& n) const {
    if constexpr (sizeof(C) == 8) return n.d64.as<double>();
    else return n.d32.as<float>();
  }

  // The pass acc = A [diag(g)] X; the caller sets the epilogue (out, scales).
  SpmmPass pass_for(const DagNode& a, bool t, const DagNode* cs, const View<T>& X) const {
    const Csr& csr = t ? a.bwd : a.fwd;
    SpmmPass p;
    p.n_rows = t ? a.cols : a.rows;
    p.nnz = csr.nnz;
    p.indptr = csr.indptr;
    p.indices = csr.indices;
    p.values = csr.values;
    p.ncols = l_;
    p.heavy_threshold = csr.n_heavy > 0 ? kHeavyThreshold : 0;
    p.heavy_rows = csr.heavy.as<int32_t>();
    p.n_heavy = csr.n_heavy;
    p.src = X.p;
    p.ld_src = X.ld;
    if (cs) {
      p.colscale = diag_vals(*cs);
      p.cs_a = 1.0;
      p.cs_b = 0.0;
    }
    return p;
  }

  // One sparse pass: out = [diag(r)] A [diag(g)] X
  View<T> sparse_pass(const DagNode& a, bool t, const DagNode* rs, const DagNode* cs, const View<T>& X) {
    SpmmPass p = pass_for(a, t, cs, X);
    View<T> out = acquire(p.n_rows);
    if (rs) {
      p.rowscale = diag_vals(*rs);
      p.a0 = 0.0;
      p.a1 = 1.0;
    }
    p.out = out.p;
    p.ld_out = out.ld;
    launch_spmm_pass<T>(p, s_);
    return out;
  }

  struct Group {
    const DagNode* rs = nullptr;
    const DagNode* cs = nullptr;
    const Atom* sparse = nullptr;
    size_t len = 1;
  };

  // The factor group at `pos` if it is a sparse pass (a sparse leaf with its scales).
  bool sparse_group(const Chain& c, size_t pos, Group& g) const {
    const Atom& a = c[pos];
    if (a.kind != Atom::Node) return false;
    const DagKind k = node_of(ev_, a.node).kind;
    if (k != DagKind::Sparse && k != DagKind::Diag) return false;
    g.len = unit_length(c, pos);
    if (k == DagKind::Diag && g.len == 1) return false;
    size_t i = pos;
    if (is_kind(c, i, DagKind::Diag)) g.rs = &node_of(ev_, c[i++].node);
    g.sparse = &c[i++];
    if (i < pos + g.len) g.cs = &node_of(ev_, c[i].node);
    return true;
  }

  // out (+)= coef * (chain times the input).  When the chain starts with a
  // sparse pass, that pass adds into `out` in its epilogue and, with the
  // cache on, also writes the chain's own result for later lookups (second
  // output), so no separate accumulation pass is needed.
  void accumulate(const Chain& c, double coef, const View<T>& out, bool first) {
    Chain key;
    if (ev_.cache_on) {
      key = c;
      auto it = cache_.find(key);
      if (it != cache_.end()) {
        launch_axpby<T>(out.rows, l_, coef, it->second.p, it->second.ld, first ? 0.0 : 1.0, out.p, out.ld, s_);
        return;
      }
    }
    Group g;
    if (!sparse_group(c, 0, g)) {
      View<T> Y = eval(c, 0);
      launch_axpby<T>(out.rows, l_, coef, Y.p, Y.ld, first ? 0.0 : 1.0, out.p, out.ld, s_);
      release(Y);
      return;
    }
    View<T> X = eval(c, g.len);
    SpmmPass p = pass_for(node_of(ev_, g.sparse->node), g.sparse->t, g.cs, X);
    if (g.rs) {
      p.rowscale = diag_vals(*g.rs);
      p.a0 = 0.0;
      p.a1 = coef;
    } else {
      p.a0 = coef;
      p.a1 = 0.0;
    }
    if (!first) {
      p.add = out.p;  // row-local read before the write of the same row
      p.ld_add = out.ld;
      p.b0 = 1.0;
    }
    p.out = out.p;
    p.ld_out = out.ld;
    if (ev_.cache_on) {
      View<T> held = acquire(p.n_rows);
      p.out2 = held.p;
      p.ld_out2 = held.ld;
      p.c0 = g.rs ? 0.0 : 1.0;
      p.c1 = g.rs ? 1.0 : 0.0;
      held.owner = -1;
      cache_.emplace(std::move(key), held);
    }
    launch_spmm_pass<T>(p, s_);
    release(X);
  }

 public:
  // out = coef * (chain times the input), accumulating a leading sum or
  // column concatenation straight into `out`.
  void eval_into(const Chain& chain, double coef, const View<T>& out) {
    const Atom& a = chain[0];
    if (chain.size() == 1 && a.kind == Atom::Node) {
      const DagNode& n = node_of(ev_, a.node);
      if (n.kind == DagKind::Sum || (n.kind == DagKind::Concat && !a.t)) {
        sum_terms(chain, 0, coef, out);
        return;
      }
    }
    View<T> v = eval(chain, 0);
    launch_axpby<T>(out.rows, l_, coef, v.p, v.ld, 0.0, out.p, out.ld, s_);
    release(v);
  }

 private:
  // The terms of the sum or column concatenation at chain[pos], each
  // continued by the rest of the chain, accumulated into out with `scale`.
  // A term that is itself a sum or column concatenation (and not already in
  // the cache) is expanded in place, so nested sums add straight into `out`.
  void sum_terms(const Chain& chain, size_t pos, double scale, const View<T>& out) {
    bool first = true;
    sum_terms(chain, pos, scale, out, first);
  }
  void sum_terms(const Chain& chain, size_t pos, double scale, const View<T>& out, bool& first) {
    const Atom& a = chain[pos];
    const DagNode& n = node_of(ev_, a.node);
    for (size_t k = 0; k < n.kids.size(); ++k) {
      Chain c;
      double coef = scale * (n.kind == DagKind::Sum ? n.w[k] : 1.0);
      flatten(ev_, n.kids[k], a.t, c, coef);
      if (n.kind == DagKind::Concat) c.push_back({Atom::Slice, a.node, false, static_cast<int>(k)});
      c.insert(c.end(), chain.begin() + static_cast<std::ptrdiff_t>(pos) + 1, chain.end());
      if (c[0].kind == Atom::Node && !(ev_.cache_on && cache_.count(c))) {
        const DagNode& h = node_of(ev_, c[0].node);
        if (h.kind == DagKind::Sum || (h.kind == DagKind::Concat && !c[0].t)) {
          sum_terms(c, 0, coef, out, first);
          continue;
        }
      }
      accumulate(c, coef, out, first);
      first = false;
    }
  }

  View<T> compute(const Chain& chain, size_t pos) {
    const Atom& a = chain[pos];
    const DagNode& n = node_of(ev_, a.node);
    if (a.kind == Atom::Slice) {
      // rows [off, off + cols of the part) of the block below
      View<T> X = eval(chain, pos + 1);
      int64_t off = 0;
      for (int i = 0; i < a.part; ++i) off += node_of(ev_, n.kids[static_cast<size_t>(i)]).cols;
      View<T> v = X;
      v.p = X.p + off * X.ld;
      v.rows = node_of(ev_, n.kids[static_cast<size_t>(a.part)]).cols;
      return v;  // the slot of X (if any) travels with the slice
    }
    if (a.kind == Atom::Select) {
      View<T> X = eval(chain, pos + 1);
      View<T> out = acquire(out_rows(ev_, a));
      if (!a.t)
        launch_gather_block<T>(n.nsub, l_, n.sel.as<int64_t>(), X.p, X.ld, out.p, out.ld, s_);
      else
        launch_scatter_block<T>(out.rows, l_, n.pos.as<int32_t>(), X.p, X.ld, out.p, out.ld, s_);
      release(X);
      return out;
    }
    switch (n.kind) {
      case DagKind::Sparse:
      case DagKind::Diag: {
        // the pass unit starting here (grouped from the right end of the chain)
        const size_t len = unit_length(chain, pos);
        size_t i = pos;
        const DagNode* rs = nullptr;
        const DagNode* cs = nullptr;
        if (len == 1 && n.kind == DagKind::Diag) {
          View<T> X = eval(chain, pos + 1);
          View<T> out = acquire(n.rows);
          launch_diag_scale<T>(n.rows, l_, n.d64.as<double>(), X.p, X.ld, out.p, out.ld, s_);
          release(X);
          return out;
        }
        if (is_kind(chain, i, DagKind::Diag)) rs = &node_of(ev_, chain[i++].node);
        const Atom& sa = chain[i++];
        if (i < pos + len) cs = &node_of(ev_, chain[i++].node);
        View<T> X = eval(chain, pos + len);
        View<T> out = sparse_pass(node_of(ev_, sa.node), sa.t, rs, cs, X);
        release(X);
        return out;
      }
      case DagKind::Dense: {
        View<T> X = eval(chain, pos + 1);
        const T* Xl = static_cast<const T*>(n.X);
        View<T> out = acquire(a.t ? n.cols : n.rows);
        if (!a.t) {
          launch_gemm_tall<T>(n.rows, l_, static_cast<int>(n.cols), Xl, n.ldx, 0, nullptr, 0,
                              reinterpret_cast<const C*>(X.p), X.ld, out.p, out.ld, 1.0, 0.0, GemmEpi::Store,
                              nullptr, nullptr, s_);
        } else {
          const int m = static_cast<int>(n.cols);
          ISVD_CHECK(m + l_ <= 2048, ISVD_E_INVALID, "dag dense: columns + block width above 2048");
          ev_.gram_c.ensure(static_cast<size_t>(m) * l_ * sizeof(double));
          ev_.gram_work.ensure(gram_workspace_doubles(n.rows, m, l_) * sizeof(double));
          launch_gram2<T, T>(n.rows, m, l_, Xl, n.ldx, X.p, X.ld, ev_.gram_c.as<double>(), l_,
                             ev_.gram_work.as<double>(), s_);
          launch_convert<T, double>(m, l_, ev_.gram_c.as<double>(), l_, out.p, out.ld, s_);
        }
        release(X);
        return out;
      }
      case DagKind::Sum: {
        View<T> out = acquire(out_rows(ev_, a));
        sum_terms(chain, pos, 1.0, out);
        return out;
      }
      case DagKind::Concat: {
        View<T> out = acquire(out_rows(ev_, a));
        if (!a.t) {
          // [M_1 .. M_m] X = sum_k M_k X_k
          sum_terms(chain, pos, 1.0, out);
          return out;
        }
        // [M_1 .. M_m]^T X stacks M_k^T X
        int64_t off = 0;
        for (size_t k = 0; k < n.kids.size(); ++k) {
          Chain c;
          double coef = 1.0;
          flatten(ev_, n.kids[k], true, c, coef);
          c.insert(c.end(), chain.begin() + static_cast<std::ptrdiff_t>(pos) + 1, chain.end());
          View<T> Y = eval(c, 0);
          launch_axpby<T>(Y.rows, l_, coef, Y.p, Y.ld, 0.0, out.p + off * out.ld, out.ld, s_);
          off += Y.rows;
          release(Y);
        }
        return out;
      }
      default: break;
    }
    throw Error{ISVD_E_INVALID, "dag: node kind cannot be a factor"};
  }

  static constexpr int64_t kHeavyThreshold = 256;

  DagEval& ev_;
  const T* G_;
  int64_t ldg_, g_rows_;
  int l_;
  int64_t ldb_;
  hipStream_t s_;
  std::map<Chain, View<T>> cache_;
};

}  // namespace

std::shared_ptr<DagEval> make_dag_eval(const isvd_dag* dag, int64_t root, bool lazy_cache) {
  auto ev = std::make_shared<DagEval>();
  ev->nodes = dag->store;
  ev->root = root;
  ev->cache_on = lazy_cache;
  return ev;
}

template <typename T>
void dag_apply(DagEval& ev, bool transpose, const T* Y, int64_t ldy, int ncols, T* out, int64_t ldo,
               hipStream_t stream) {
  const DagNode& r = node_of(ev, ev.root);
  Chain chain;
  double coef = 1.0;
  flatten(ev, ev.root, transpose, chain, coef);
  Evaluator<T> e(ev, Y, ldy, transpose ? r.rows : r.cols, ncols, stream);
  e.eval_into(chain, coef, View<T>{out, ldo, transpose ? r.cols : r.rows, -1});
}
template void dag_apply<float>(DagEval&, bool, const float*, int64_t, int, float*, int64_t, hipStream_t);
template void dag_apply<double>(DagEval&, bool, const double*, int64_t, int, double*, int64_t, hipStream_t);

}  // namespace isvd
