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
// of that leaf's sparse pass.  With the lazy cache, the result of every
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
  const isvd_dag* dag = nullptr;
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

const DagNode& node_of(const DagEval& ev, int64_t id) { return *ev.dag->nodes[static_cast<size_t>(id)]; }

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

  const C* diag_vals(const DagNode& n) const {
    if constexpr (sizeof(C) == 8) return n.d64.as<double>();
    else return n.d32.as<float>();
  }

  // One sparse pass: out = [diag(r)] A [diag(g)] X
  View<T> sparse_pass(const DagNode& a, bool t, const DagNode* rs, const DagNode* cs, const View<T>& X) {
    const Csr& csr = t ? a.bwd : a.fwd;
    View<T> out = acquire(t ? a.cols : a.rows);
    SpmmPass p;
    p.n_rows = out.rows;
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
      case DagKind::Sparse: {
        const DagNode* cs = nullptr;
        size_t next = pos + 1;
        if (is_kind(chain, next, DagKind::Diag)) {
          cs = &node_of(ev_, chain[next].node);
          ++next;
        }
        View<T> X = eval(chain, next);
        View<T> out = sparse_pass(n, a.t, nullptr, cs, X);
        release(X);
        return out;
      }
      case DagKind::Diag: {
        if (is_kind(chain, pos + 1, DagKind::Sparse)) {
          const Atom& sa = chain[pos + 1];
          const DagNode* cs = nullptr;
          size_t next = pos + 2;
          if (is_kind(chain, next, DagKind::Diag)) {
            cs = &node_of(ev_, chain[next].node);
            ++next;
          }
          View<T> X = eval(chain, next);
          View<T> out = sparse_pass(node_of(ev_, sa.node), sa.t, &n, cs, X);
          release(X);
          return out;
        }
        View<T> X = eval(chain, pos + 1);
        View<T> out = acquire(n.rows);
        launch_diag_scale<T>(n.rows, l_, n.d64.as<double>(), X.p, X.ld, out.p, out.ld, s_);
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
        for (size_t k = 0; k < n.kids.size(); ++k) {
          Chain c;
          double coef = n.w[k];
          flatten(ev_, n.kids[k], a.t, c, coef);
          c.insert(c.end(), chain.begin() + static_cast<std::ptrdiff_t>(pos) + 1, chain.end());
          View<T> Y = eval(c, 0);
          launch_axpby<T>(out.rows, l_, coef, Y.p, Y.ld, k == 0 ? 0.0 : 1.0, out.p, out.ld, s_);
          release(Y);
        }
        return out;
      }
      case DagKind::Concat: {
        View<T> out = acquire(out_rows(ev_, a));
        int64_t off = 0;
        for (size_t k = 0; k < n.kids.size(); ++k) {
          Chain c;
          double coef = 1.0;
          flatten(ev_, n.kids[k], a.t, c, coef);
          if (!a.t) c.push_back({Atom::Slice, a.node, false, static_cast<int>(k)});
          c.insert(c.end(), chain.begin() + static_cast<std::ptrdiff_t>(pos) + 1, chain.end());
          View<T> Y = eval(c, 0);
          if (!a.t) {
            // [M_1 .. M_m] X = sum_k M_k X_k
            launch_axpby<T>(out.rows, l_, coef, Y.p, Y.ld, k == 0 ? 0.0 : 1.0, out.p, out.ld, s_);
          } else {
            // [M_1 .. M_m]^T X stacks M_k^T X
            launch_axpby<T>(Y.rows, l_, coef, Y.p, Y.ld, 0.0, out.p + off * out.ld, out.ld, s_);
            off += Y.rows;
          }
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
  ev->dag = dag;
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
  View<T> v = e.eval(chain, 0);
  launch_axpby<T>(transpose ? r.cols : r.rows, ncols, coef, v.p, v.ld, 0.0, out, ldo, stream);
  e.release(v);
}
template void dag_apply<float>(DagEval&, bool, const float*, int64_t, int, float*, int64_t, hipStream_t);
template void dag_apply<double>(DagEval&, bool, const double*, int64_t, int, double*, int64_t, hipStream_t);

}  // namespace isvd
