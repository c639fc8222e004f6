// Host setup and V-cycle driver of the FP32 smoothed-aggregation AMG
// preconditioner built on the compact-stencil approximate Jacobian J_tilde
// (Section 3.1, coefficients after Eq. SegSys; used as the preconditioning
// matrix in Section 3.2).
//
// J_tilde = -A (x) I_dim with A the scalar symmetric, diagonally dominant
// M-matrix sum_f alpha K_bar |Delta||Gamma|/|d| (neighbour differences) plus
// the displacement-face terms on the diagonal.  The preconditioner returns
// z ~ J_tilde^{-1} r = -A^{-1} r by one V-cycle on A applied to every
// displacement component at once:
//   setup (FP64, once per mesh): greedy aggregation on the strength graph
//   |a_ij| >= theta sqrt(a_ii a_jj) (theta = 0.08, which keeps the weak
//   direction of stretched cells out of the aggregates), smoothed prolongator
//   P = (I - omega D^{-1} A) P_tent with omega = 4/(3 lambda_max(D^{-1}A)),
//   Galerkin coarse operators R A P with R = P^T, a dense inverse on the
//   coarsest level; everything is stored on the device in FP32;
//   apply (FP32 kernels): Chebyshev(k) pre-smoothing from zero on the interval
//   [lambda_max/30, 1.1 lambda_max] of D^{-1} A, restriction, recursion,
//   prolongation, Chebyshev(k) post-smoothing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <numeric>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "amg.h"
#include "solver.h"

namespace jfnk {

namespace {

constexpr double kTheta = 0.08;
// Coarsening stops at kHostDenseMax rows, whose dense inverse is formed on
// the host; on a single mesh of at least kDeviceDenseMinRows rows it stops
// at kDenseMax rows instead, the inverse formed on the device (rocSOLVER
// Cholesky factor and inverse): the coarse levels in between cost a launch
// chain per V-cycle that such a solve repeats thousands of times, while on
// small meshes and batches the set-up time of the larger inverse would not
// be repaid.
constexpr int64_t kDenseMax = 5000;
constexpr int64_t kHostDenseMax = 200;
constexpr int64_t kDeviceDenseMinRows = 262144;
constexpr int kMaxLevels = 16;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Setup passes over matrix rows run in chunks of kRowChunk rows on host
// threads; outputs are assembled in chunk order, so matrices equal the
// serial build, and sums over rows add per-chunk partials in chunk order.
// Passes that only build rows use shorter chunks (kBuildChunk), which
// balance the coarse levels' few long rows over the threads; their results
// do not depend on the chunk length.
constexpr int64_t kRowChunk = 8192;
constexpr int64_t kBuildChunk = 256;

inline int64_t n_chunks(int64_t n, int64_t len = kRowChunk) { return (n + len - 1) / len; }

// Row output buffers of the setup passes, handed back after each pass and
// reused by the next one (at most kKeptScratch kept): a pass appends to
// memory that earlier passes already mapped instead of growing fresh vectors.
struct RowScratch {
  std::vector<int32_t> col;
  std::vector<double> val;
};

constexpr size_t kKeptScratch = 16;

class ScratchStore {
 public:
  std::unique_ptr<RowScratch> take() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) return std::unique_ptr<RowScratch>(new RowScratch());
    std::unique_ptr<RowScratch> s = std::move(free_.back());
    free_.pop_back();
    return s;
  }
  void give(std::unique_ptr<RowScratch> s) {
    s->col.clear();
    s->val.clear();
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.size() < kKeptScratch) free_.push_back(std::move(s));
  }

 private:
  std::mutex mu_;
  std::vector<std::unique_ptr<RowScratch>> free_;
};

ScratchStore& scratch_store() {
  static ScratchStore* store = new ScratchStore();  // lives until the process ends
  return *store;
}

// A CSR matrix whose row i is appended by row(i, cols, vals, t) (t: the
// calling thread's number, for scratch).  Each thread appends the rows of its
// chunks to a buffer of its own; once all row lengths are known the chunks
// are copied into place in parallel.
template <class RowFn>
HostCsr build_rows(int64_t n, int64_t m, RowFn&& row) {
  const int64_t nc = n_chunks(n, kBuildChunk);
  std::vector<std::unique_ptr<RowScratch>> sp(size_t(host_threads(nc)));
  std::vector<int32_t> owner(static_cast<size_t>(nc));
  std::vector<int64_t> beg(static_cast<size_t>(nc)), len(static_cast<size_t>(nc));
  HostCsr M;
  M.n = n;
  M.m = m;
  M.ptr.resize(size_t(n) + 1);
  M.ptr[0] = 0;
  parallel_for(nc, [&](int64_t c, int t) {
    if (!sp[size_t(t)]) sp[size_t(t)] = scratch_store().take();
    RowScratch& sc = *sp[size_t(t)];
    const int64_t lo = c * kBuildChunk, hi = std::min(n, lo + kBuildChunk);
    owner[size_t(c)] = t;
    beg[size_t(c)] = int64_t(sc.col.size());
    for (int64_t i = lo; i < hi; ++i) {
      const size_t before = sc.col.size();
      row(i, sc.col, sc.val, t);
      M.ptr[size_t(i) + 1] = int32_t(sc.col.size() - before);  // row length for now
    }
    len[size_t(c)] = int64_t(sc.col.size()) - beg[size_t(c)];
  });
  // chunk offsets, then every chunk writes its row ends and entries in place
  std::vector<int64_t> off(size_t(nc) + 1, 0);
  for (int64_t c = 0; c < nc; ++c) off[c + 1] = off[c] + len[c];
  JFNK_REQUIRE(off[nc] < (int64_t(1) << 31), JFNK_E_ARG, "amg: operator too large for 32-bit row offsets");
  M.col.resize(size_t(off[nc]));
  M.val.resize(size_t(off[nc]));
  parallel_for(nc, [&](int64_t c, int) {
    const int64_t lo = c * kBuildChunk, hi = std::min(n, lo + kBuildChunk);
    int64_t p = off[c];
    for (int64_t i = lo; i < hi; ++i) {
      p += M.ptr[size_t(i) + 1];
      M.ptr[size_t(i) + 1] = int32_t(p);
    }
    const RowScratch& sc = *sp[size_t(owner[size_t(c)])];
    std::copy_n(sc.col.data() + beg[c], len[c], M.col.data() + off[c]);
    std::copy_n(sc.val.data() + beg[c], len[c], M.val.data() + off[c]);
  });
  for (auto& b : sp)
    if (b) scratch_store().give(std::move(b));
  return M;
}

// Sparse accumulator of one thread: acc/mark over the output columns.
struct RowAcc {
  std::vector<double> acc;
  std::vector<int32_t> mark, cols;
  void init(int64_t m) {
    if (int64_t(acc.size()) == m) return;
    acc.assign(size_t(m), 0.0);
    mark.assign(size_t(m), -1);
  }
  void add(int64_t i, int32_t c, double v) {
    if (mark[c] != i) {
      mark[c] = int32_t(i);
      acc[c] = 0.0;
      cols.push_back(c);
    }
    acc[c] += v;
  }
};

// The scalar approximate Jacobian (negated: positive diagonal), rows sorted
// by column.  Faces go to host threads, which claim slots in their two rows
// with atomic cursors; the per-row sort of (column, value) pairs then gives
// the same rows whatever order the slots were claimed in.
HostCsr fine_operator(const HostMesh& h, const std::vector<double>& pc_diag) {
  HostCsr A;
  const int64_t n = h.n_cells, nf = h.n_int;
  A.n = A.m = n;
  const int64_t face_chunks = (nf + kRowChunk - 1) / kRowChunk;
  std::vector<int32_t> cnt(n, 1);
  parallel_for(face_chunks, [&](int64_t c, int) {
    for (int64_t j = c * kRowChunk; j < std::min(nf, (c + 1) * kRowChunk); ++j) {
      __atomic_fetch_add(&cnt[h.fown[j]], 1, __ATOMIC_RELAXED);
      __atomic_fetch_add(&cnt[h.fnb[j]], 1, __ATOMIC_RELAXED);
    }
  });
  A.ptr.resize(size_t(n) + 1);
  A.ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) A.ptr[i + 1] = A.ptr[i] + cnt[i];
  A.col.resize(A.ptr[n]);
  A.val.resize(A.ptr[n]);
  std::vector<int32_t>& pos = cnt;  // next free slot of each row
  parallel_for(n_chunks(n), [&](int64_t c, int) {
    for (int64_t i = c * kRowChunk; i < std::min(n, (c + 1) * kRowChunk); ++i) {
      A.col[A.ptr[i]] = int32_t(i);
      A.val[A.ptr[i]] = -pc_diag[i];
      pos[i] = A.ptr[i] + 1;
    }
  });
  parallel_for(face_chunks, [&](int64_t c, int) {
    for (int64_t j = c * kRowChunk; j < std::min(nf, (c + 1) * kRowChunk); ++j) {
      const int32_t a = h.fown[j], b = h.fnb[j];
      const int32_t pa = __atomic_fetch_add(&pos[a], 1, __ATOMIC_RELAXED);
      A.col[pa] = b;
      A.val[pa] = -h.pc_off[j];
      const int32_t pb = __atomic_fetch_add(&pos[b], 1, __ATOMIC_RELAXED);
      A.col[pb] = a;
      A.val[pb] = -h.pc_off[j];
    }
  });
  // sort each row by column (then value, for equal columns)
  parallel_for(n_chunks(n), [&](int64_t c, int) {
    std::vector<std::pair<int32_t, double>> tmp;
    const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
    for (int64_t i = lo; i < hi; ++i) {
      tmp.clear();
      for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) tmp.emplace_back(A.col[k], A.val[k]);
      std::sort(tmp.begin(), tmp.end());
      for (size_t k = 0; k < tmp.size(); ++k) {
        A.col[A.ptr[i] + k] = tmp[k].first;
        A.val[A.ptr[i] + k] = tmp[k].second;
      }
    }
  });
  return A;
}

std::vector<double> diagonal(const HostCsr& A) {
  std::vector<double> d(A.n, 0.0);
  parallel_for(n_chunks(A.n), [&](int64_t c, int) {
    const int64_t lo = c * kRowChunk, hi = std::min(A.n, lo + kRowChunk);
    for (int64_t i = lo; i < hi; ++i)
      for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        if (A.col[k] == i) d[i] = A.val[k];
  });
  return d;
}

// lambda_max of D^{-1} A by power iteration from a fixed start vector.  The
// pass that forms y = D^{-1} A x also sums y*y per chunk, which is the next
// iteration's |x|^2 in the same order.
double lambda_max(const HostCsr& A, const std::vector<double>& d) {
  const int64_t n = A.n, nc = n_chunks(n);
  std::vector<double> x(n), y(n), sq(nc), num(nc);
  parallel_for(nc, [&](int64_t c, int) {
    const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
    for (int64_t i = lo; i < hi; ++i) x[i] = 1.0 + 0.5 * std::sin(0.7 * double(i) + 0.3);
  });
  auto chunk_sum = [&](const std::vector<double>& part) {
    double t = 0;
    for (int64_t c = 0; c < nc; ++c) t += part[c];
    return t;
  };
  parallel_for(nc, [&](int64_t c, int) {
    const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
    double t = 0;
    for (int64_t i = lo; i < hi; ++i) t += x[i] * x[i];
    sq[c] = t;
  });
  double lam = 1.0;
  for (int it = 0; it < 20; ++it) {
    const double nrm = std::sqrt(chunk_sum(sq));
    parallel_for(nc, [&](int64_t c, int) {
      const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
      for (int64_t i = lo; i < hi; ++i) x[i] /= nrm;
    });
    parallel_for(nc, [&](int64_t c, int) {
      const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
      double t = 0, q = 0;
      for (int64_t i = lo; i < hi; ++i) {
        double s = 0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * x[A.col[k]];
        y[i] = s / d[i];
        t += y[i] * x[i];
        q += y[i] * y[i];
      }
      num[c] = t;
      sq[c] = q;
    });
    lam = chunk_sum(num);
    x.swap(y);
  }
  return lam;
}

// Greedy aggregation of rows [lo, hi), which no entry of A connects with
// other rows.  agg[lo, hi) holds -1 on entry; on return it holds local
// numbers: the n1 pass-1 aggregates 0..n1-1 and the n3 pass-3 ones after
// them, each numbered in the order it is formed.
void aggregate_rows(const HostCsr& A, const std::vector<double>& d, int64_t lo, int64_t hi,
                    std::vector<int32_t>& agg, int64_t& n1, int64_t& n3) {
  auto strong = [&](int64_t i, int32_t k) {
    const int32_t j = A.col[k];
    return j != i && std::fabs(A.val[k]) >= kTheta * std::sqrt(std::fabs(d[i] * d[j]));
  };
  int64_t na = 0;
  // pass 1: seed aggregates whose strong neighbourhood is still free
  for (int64_t i = lo; i < hi; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true, any = false;
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k)) {
        any = true;
        if (agg[A.col[k]] >= 0) {
          free = false;
          break;
        }
      }
    if (!free || !any) continue;
    agg[i] = int32_t(na);
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k)) agg[A.col[k]] = int32_t(na);
    ++na;
  }
  n1 = na;
  // pass 2: attach leftovers to the most strongly connected pass-1 aggregate
  const std::vector<int32_t> agg1(agg.begin() + lo, agg.begin() + hi);
  for (int64_t i = lo; i < hi; ++i) {
    if (agg1[i - lo] >= 0) continue;
    double best = 0;
    int32_t ba = -1;
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k) && agg1[A.col[k] - lo] >= 0 && std::fabs(A.val[k]) > best) {
        best = std::fabs(A.val[k]);
        ba = agg1[A.col[k] - lo];
      }
    if (ba >= 0) agg[i] = ba;
  }
  // pass 3: remaining nodes with their free strong neighbours, or singletons.
  // Nodes without any strong neighbour (padding rows of a batch, a mesh that
  // has already been reduced to one coarse unknown) stay out of the coarse
  // space: the smoother alone treats them.
  for (int64_t i = lo; i < hi; ++i) {
    if (agg[i] >= 0) continue;
    bool any = false;
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1] && !any; ++k) any = strong(i, k);
    if (!any) continue;
    agg[i] = int32_t(na);
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k) && agg[A.col[k]] < 0) agg[A.col[k]] = int32_t(na);
    ++na;
  }
  n3 = na - n1;
}

// Ends of consecutive row ranges that no entry of A connects with each other
// (the meshes of a batch, and on coarser levels their aggregates), merged
// into ranges of at least min_len rows.  One range when there is no cut.
std::vector<int64_t> independent_ranges(const HostCsr& A, int64_t min_len) {
  const int64_t n = A.n;
  std::vector<int32_t> lo_col(static_cast<size_t>(n)), hi_col(static_cast<size_t>(n));
  parallel_for(n_chunks(n), [&](int64_t c, int) {
    const int64_t lo = c * kRowChunk, hi = std::min(n, lo + kRowChunk);
    for (int64_t i = lo; i < hi; ++i) {
      int32_t a = int32_t(i), b = int32_t(i);
      for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        a = std::min(a, A.col[k]);
        b = std::max(b, A.col[k]);
      }
      lo_col[i] = a;
      hi_col[i] = b;
    }
  });
  // a cut before row p is valid when no row above reaches p or beyond and no
  // row from p on reaches above p
  std::vector<int32_t> below_min(static_cast<size_t>(n) + 1);
  below_min[n] = std::numeric_limits<int32_t>::max();
  for (int64_t i = n - 1; i >= 0; --i) below_min[i] = std::min(below_min[i + 1], lo_col[i]);
  std::vector<int64_t> ends;
  int64_t start = 0, reach = -1;
  for (int64_t p = 1; p <= n; ++p) {
    reach = std::max<int64_t>(reach, hi_col[p - 1]);
    if (p == n || (reach < p && below_min[p] >= p && p - start >= min_len)) {
      ends.push_back(p);
      start = p;
    }
  }
  return ends;
}

// Aggregates of A (-1: row left out of the coarse space).  Ranges of rows
// that A does not connect are aggregated in parallel; the numbering is that
// of one pass over all rows: pass-1 aggregates in row order, then the
// pass-3 ones in row order.
std::vector<int32_t> aggregate(const HostCsr& A, const std::vector<double>& d, int64_t& nagg) {
  const int64_t n = A.n;
  std::vector<int32_t> agg(n, -1);
  const std::vector<int64_t> ends =
      n > 0 ? independent_ranges(A, std::max<int64_t>(kBuildChunk, n / 64)) : std::vector<int64_t>();
  const int64_t nr = int64_t(ends.size());
  std::vector<int64_t> n1(static_cast<size_t>(nr)), n3(static_cast<size_t>(nr));
  parallel_for(nr, [&](int64_t r, int) {
    aggregate_rows(A, d, r > 0 ? ends[r - 1] : 0, ends[r], agg, n1[r], n3[r]);
  });
  std::vector<int64_t> off1(static_cast<size_t>(nr) + 1, 0), off3(static_cast<size_t>(nr) + 1, 0);
  for (int64_t r = 0; r < nr; ++r) off1[r + 1] = off1[r] + n1[r];
  off3[0] = off1[nr];
  for (int64_t r = 0; r < nr; ++r) off3[r + 1] = off3[r] + n3[r];
  nagg = off3[nr];
  JFNK_REQUIRE(nagg < (int64_t(1) << 31), JFNK_E_ARG, "amg: too many aggregates");
  parallel_for(nr, [&](int64_t r, int) {
    for (int64_t i = r > 0 ? ends[r - 1] : 0; i < ends[r]; ++i) {
      const int32_t a = agg[i];
      if (a >= 0) agg[i] = int32_t(a < n1[r] ? off1[r] + a : off3[r] + (a - n1[r]));
    }
  });
  return agg;
}

// P = (I - omega D^{-1} A) P_tent
HostCsr smoothed_prolongator(const HostCsr& A, const std::vector<double>& d,
                             const std::vector<int32_t>& agg, int64_t nagg, double omega) {
  std::vector<RowAcc> ra(size_t(host_threads(n_chunks(A.n, kBuildChunk))));
  return build_rows(A.n, nagg, [&](int64_t i, std::vector<int32_t>& col, std::vector<double>& val, int t) {
    RowAcc& r = ra[size_t(t)];
    r.init(nagg);
    r.cols.clear();
    if (agg[i] >= 0) r.add(i, agg[i], 1.0);
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (agg[A.col[k]] >= 0) r.add(i, agg[A.col[k]], -omega * A.val[k] / d[i]);
    std::sort(r.cols.begin(), r.cols.end());
    for (int32_t c : r.cols) {
      if (r.acc[c] == 0.0) continue;
      col.push_back(c);
      val.push_back(r.acc[c]);
    }
  });
}

// Transpose.  The rows of M are cut into one piece per thread; each piece
// counts its entries per column and takes, inside every column, the slots
// after those of the pieces above it, so every row of the transpose lists
// its entries in increasing row of M, as one pass over M would.
HostCsr transpose(const HostCsr& M) {
  HostCsr T;
  T.n = M.m;
  T.m = M.n;
  const int np = host_threads(n_chunks(M.n, kBuildChunk));
  std::vector<std::vector<int32_t>> cnt(static_cast<size_t>(np));
  auto piece = [&](int64_t p, int64_t& lo, int64_t& hi) {
    lo = M.n * p / np;
    hi = M.n * (p + 1) / np;
  };
  parallel_for(np, [&](int64_t p, int) {
    cnt[p].assign(size_t(M.m), 0);
    int64_t lo, hi;
    piece(p, lo, hi);
    for (int32_t k = M.ptr[lo]; k < M.ptr[hi]; ++k) cnt[p][M.col[k]]++;
  });
  // per column: the pieces' start offsets inside it, and its length
  T.ptr.resize(size_t(M.m) + 1);
  T.ptr[0] = 0;
  parallel_for(n_chunks(M.m), [&](int64_t c, int) {
    const int64_t lo = c * kRowChunk, hi = std::min(M.m, lo + kRowChunk);
    for (int64_t j = lo; j < hi; ++j) {
      int32_t s = 0;
      for (int p = 0; p < np; ++p) {
        const int32_t t = cnt[p][j];
        cnt[p][j] = s;
        s += t;
      }
      T.ptr[j + 1] = s;
    }
  });
  for (int64_t j = 0; j < M.m; ++j) T.ptr[j + 1] += T.ptr[j];
  T.col.resize(M.col.size());
  T.val.resize(M.val.size());
  parallel_for(np, [&](int64_t p, int) {
    int64_t lo, hi;
    piece(p, lo, hi);
    std::vector<int32_t>& pos = cnt[p];
    for (int64_t i = lo; i < hi; ++i)
      for (int32_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
        const int32_t c = M.col[k];
        const int64_t q = int64_t(T.ptr[c]) + pos[c]++;
        T.col[q] = int32_t(i);
        T.val[q] = M.val[k];
      }
  });
  return T;
}

// Z = X Y.  Rows come out with sorted columns unless sorted = false (the
// intermediate A P: R (A P) adds into each output column in the order of
// R's columns, whatever the order inside a row of A P).
HostCsr multiply(const HostCsr& X, const HostCsr& Y, bool sorted = true) {
  std::vector<RowAcc> ra(size_t(host_threads(n_chunks(X.n, kBuildChunk))));
  return build_rows(X.n, Y.m, [&](int64_t i, std::vector<int32_t>& col, std::vector<double>& val, int t) {
    RowAcc& r = ra[size_t(t)];
    r.init(Y.m);
    r.cols.clear();
    for (int32_t a = X.ptr[i]; a < X.ptr[i + 1]; ++a) {
      const int32_t j = X.col[a];
      const double xv = X.val[a];
      for (int32_t b = Y.ptr[j]; b < Y.ptr[j + 1]; ++b) r.add(i, Y.col[b], xv * Y.val[b]);
    }
    if (sorted) std::sort(r.cols.begin(), r.cols.end());
    for (int32_t c : r.cols) {
      col.push_back(c);
      val.push_back(r.acc[c]);
    }
  });
}

// Inverse of a small SPD matrix by Cholesky (FP64), returned column-major.
std::vector<double> dense_inverse(const HostCsr& A) {
  const int64_t n = A.n;
  std::vector<double> L(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) L[i * n + A.col[k]] = A.val[k];
  double shift = 0;
  for (int64_t i = 0; i < n; ++i) shift = std::max(shift, std::fabs(L[i * n + i]));
  shift *= 1e-12;
  for (int64_t j = 0; j < n; ++j) {
    double s = L[j * n + j] + shift;
    for (int64_t k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    JFNK_REQUIRE(s > 0, JFNK_E_MESH, "amg: coarse operator not positive definite");
    const double ljj = std::sqrt(s);
    L[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = L[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / ljj;
    }
  }
  std::vector<double> inv(n * n);
  std::vector<double> x(n);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) t -= L[i * n + k] * x[k];
      x[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double t = x[i];
      for (int64_t k = i + 1; k < n; ++k) t -= L[k * n + i] * x[k];
      x[i] = t / L[i * n + i];
    }
    for (int64_t i = 0; i < n; ++i) inv[c * n + i] = x[i];   // column-major
  }
  return inv;
}

struct ChebCoef {
  double inv_theta;
  std::vector<double> c1, c2;
};

ChebCoef cheb_coefficients(double lmax, int degree) {
  const double hi = 1.1 * lmax, lo = hi / 30.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  ChebCoef c;
  c.inv_theta = 1.0 / theta;
  double rho_old = 1.0 / sigma;
  for (int k = 1; k < degree; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    c.c1.push_back(rho * rho_old);
    c.c2.push_back(2.0 * rho / delta);
    rho_old = rho;
  }
  return c;
}

// Uploads FP64 host values in the hierarchy's precision.
void upload_values(DevBuf& buf, const double* v, size_t count, bool fp64, hipStream_t s) {
  buf.alloc(std::max<size_t>(count * (fp64 ? 8 : 4), 256));
  if (count == 0) return;
  if (fp64) {
    JFNK_HIP(hipMemcpyAsync(buf.p, v, count * 8, hipMemcpyHostToDevice, s));
  } else {
    std::vector<float> f(v, v + count);
    JFNK_HIP(hipMemcpyAsync(buf.p, f.data(), count * 4, hipMemcpyHostToDevice, s));
    JFNK_HIP(hipStreamSynchronize(s));   // f goes out of scope
    return;
  }
  JFNK_HIP(hipStreamSynchronize(s));
}

void check_rocblas(rocblas_status st, const char* what) {
  JFNK_REQUIRE(st == rocblas_status_success, JFNK_E_HIP, std::string("amg: ") + what + " failed");
}

// Inverse of the SPD coarse operator A on the device: the dense matrix (with
// the host path's diagonal shift) to the device, its Cholesky factor and
// inverse by rocSOLVER in FP64, then both triangles in the hierarchy's
// precision, column-major.  Returns false (out released) when the Cholesky
// factorisation finds the shifted operator not positive definite.
bool dense_inverse_device(const HostCsr& A, bool fp64, hipStream_t s, DevBuf& out) {
  const int64_t n = A.n;
  std::vector<double> M(size_t(n) * size_t(n), 0.0);
  double shift = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      M[size_t(A.col[k]) * n + i] = A.val[k];
      if (A.col[k] == i) shift = std::max(shift, std::fabs(A.val[k]));
    }
  shift *= 1e-12;
  for (int64_t i = 0; i < n; ++i) M[size_t(i) * n + i] += shift;
  // every buffer is allocated before the library section below holds the
  // capture lock (DevBuf allocation and release take it themselves) and
  // released after it
  DevBuf dm, dinfo;
  dm.alloc(M.size() * sizeof(double));
  dinfo.alloc(256);
  out.alloc(M.size() * (fp64 ? 8 : 4));
  JFNK_HIP(hipMemcpyAsync(dm.p, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
  bool pd = true;
  {
    // rocBLAS and rocSOLVER make device-wide calls of their own (handle and
    // workspace set-up, work on the legacy stream) that the runtime rejects
    // while another thread of the process captures a graph on a blocking
    // stream: like allocations, the whole section holds the capture lock
    // shared, from handle creation to its destruction
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    rocblas_handle h = nullptr;
    check_rocblas(rocblas_create_handle(&h), "rocblas_create_handle");
    struct Handle {
      rocblas_handle h;
      ~Handle() { (void)rocblas_destroy_handle(h); }
    } guard{h};
    check_rocblas(rocblas_set_stream(h, s), "rocblas_set_stream");
    rocblas_int info = 0;
    check_rocblas(rocsolver_dpotrf(h, rocblas_fill_lower, rocblas_int(n), dm.as<double>(), rocblas_int(n),
                                   dinfo.as<rocblas_int>()),
                  "Cholesky factorisation");
    JFNK_HIP(hipMemcpyAsync(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipStreamSynchronize(s));
    pd = info == 0;
    if (pd) {
      check_rocblas(rocsolver_dpotri(h, rocblas_fill_lower, rocblas_int(n), dm.as<double>(), rocblas_int(n),
                                     dinfo.as<rocblas_int>()),
                    "inverse from the Cholesky factor");
      JFNK_HIP(hipMemcpyAsync(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipStreamSynchronize(s));
      JFNK_REQUIRE(info == 0, JFNK_E_MESH, "amg: coarse operator singular");
    }
  }
  if (!pd) {
    out.release();
    return false;
  }
  if (fp64)
    amg_sym_from_lower<double>(dm.as<double>(), out.as<double>(), int(n), s);
  else
    amg_sym_from_lower<float>(dm.as<double>(), out.as<float>(), int(n), s);
  JFNK_HIP(hipStreamSynchronize(s));
  return true;
}

}  // namespace

void DevCsr::upload(const HostCsr& h, bool fp64, hipStream_t s) {
  n = int32_t(h.n);
  m = int32_t(h.m);
  nnz = int64_t(h.col.size());
  // each row is shared by the fewest lanes (a power of two) that leave at most
  // three nonzeros to a lane: a short chain of dependent gathers per lane pays
  // on the short fine-level rows as much as on the dense coarse ones
  const double avg = h.n > 0 ? double(h.col.size()) / double(h.n) : 0.0;
  lanes = 1;
  while (lanes < 64 && avg > 3.0 * lanes) lanes *= 2;
  ptr.alloc(std::max<size_t>(h.ptr.size() * 4, 256));
  col.alloc(std::max<size_t>(h.col.size() * 4, 256));
  JFNK_HIP(hipMemcpyAsync(ptr.p, h.ptr.data(), h.ptr.size() * 4, hipMemcpyHostToDevice, s));
  if (!h.col.empty()) JFNK_HIP(hipMemcpyAsync(col.p, h.col.data(), h.col.size() * 4, hipMemcpyHostToDevice, s));
  upload_values(val, h.val.data(), h.val.size(), fp64, s);
}

size_t amg_work_floats(int64_t n, int dim) {
  // upper bound before setup, in elements of the hierarchy's precision: five
  // work vectors per level with a geometric level-size bound (each level at
  // most 3/4 of the previous one)
  return size_t(5) * dim * size_t(4 * n + 64 * kMaxLevels) +
         size_t(2 + n_chunks(kDenseMax, kDenseChunk)) * kDenseMax * dim;
}

size_t amg_work_floats(const jfnk_mesh* m) { return amg_work_floats(m->host.n_cells, m->host.dim); }

void amg_setup(jfnk_mesh* m, bool fp64, hipStream_t s) {
  AmgHierarchy*& slot = fp64 ? m->amg64 : m->amg;
  if (slot) return;
  const double t0 = now_ms();
  auto H = new AmgHierarchy();
  try {
    H->dim = m->host.dim;
    H->fp64 = fp64;
    // With symmetry faces the hierarchy is built from the component mean of
    // the diagonal; the finest level adds back each component's deviation.
    const std::vector<double>& diag0 = m->pc_diag_eff.empty() ? m->host.pc_diag : m->pc_diag_eff;
    const std::vector<double>& sym = m->host.pc_sym;
    std::vector<double> diag_mean;
    if (!sym.empty()) {
      diag_mean = diag0;
      for (size_t c = 0; c < diag_mean.size(); ++c) {
        double t = 0.0;
        for (int q = 0; q < H->dim; ++q) t += sym[c * H->dim + q];
        diag_mean[c] += t / H->dim;
      }
    }
    HostCsr A = fine_operator(m->host, sym.empty() ? diag0 : diag_mean);
    int64_t dense_max = (m->n_seg() == 1 && A.n >= kDeviceDenseMinRows) ? kDenseMax : kHostDenseMax;
    const double nnz0 = double(A.nnz());
    size_t off = 0;
    auto take = [&](int64_t count) {
      size_t o = off;
      off += size_t(count) * H->dim;
      off = (off + 63) & ~size_t(63);
      return o;
    };
    while (true) {
      AmgLevel L;
      L.n = A.n;
      std::vector<double> d = diagonal(A);
      bool last = A.n <= dense_max || int(H->levels.size()) + 1 >= kMaxLevels;
      H->op_complexity += double(A.nnz()) / nnz0;
      if (last && A.n > kHostDenseMax && !dense_inverse_device(A, fp64, s, H->coarse_inv)) {
        // not positive definite in FP64 at this size (the Galerkin products
        // of a nonsymmetric or nearly singular fine operator): coarsen on to
        // the host limit, as a batch or a small mesh does
        JFNK_REQUIRE(int(H->levels.size()) + 1 < kMaxLevels, JFNK_E_MESH,
                     "amg: coarse operator not positive definite");
        dense_max = kHostDenseMax;
        last = false;
      }
      if (last) {
        L.off_x = take(A.n);
        L.off_b = take(A.n);
        if (A.n <= kHostDenseMax) {
          std::vector<double> inv = dense_inverse(A);
          upload_values(H->coarse_inv, inv.data(), inv.size(), fp64, s);
        } else {
          H->off_part = take(n_chunks(A.n, kDenseChunk) * A.n);
        }
        H->n_coarse = A.n;
        H->levels.push_back(std::move(L));
        break;
      }
      int64_t nagg = 0;
      std::vector<int32_t> agg = aggregate(A, d, nagg);
      if (nagg == 0) {
        // No row has a strong neighbour (every mesh of a batch already
        // reduced to uncoupled unknowns): the diagonal inverse solves this
        // level exactly up to the weak couplings, which the smoothers of the
        // finer levels treat.
        L.off_x = take(A.n);
        L.off_b = take(A.n);
        std::vector<double> dinv(A.n);
        for (int64_t i = 0; i < A.n; ++i) dinv[i] = 1.0 / d[i];
        upload_values(H->coarse_inv, dinv.data(), dinv.size(), fp64, s);
        H->coarse_diag = true;
        H->n_coarse = A.n;
        H->levels.push_back(std::move(L));
        break;
      }
      L.lmax = lambda_max(A, d);
      HostCsr P = smoothed_prolongator(A, d, agg, nagg, 4.0 / (3.0 * L.lmax));
      HostCsr R = transpose(P);
      HostCsr Ac = multiply(R, multiply(A, P, false));
      L.A.upload(A, fp64, s);
      L.P.upload(P, fp64, s);
      L.R.upload(R, fp64, s);
      if (H->levels.empty() && !sym.empty()) {
        // finest level: A_q = A + diag(e_q), e_q = -(sym_q - mean), and the
        // inverse of its diagonal per component (A = -J_tilde)
        const int D = H->dim;
        std::vector<double> e(size_t(D) * A.n), dinv(size_t(D) * A.n);
        for (int q = 0; q < D; ++q)
          for (int64_t i = 0; i < A.n; ++i) {
            const double eq = -(diag0[i] + sym[size_t(i) * D + q]) - d[i];
            e[size_t(q) * A.n + i] = eq;
            dinv[size_t(q) * A.n + i] = 1.0 / (d[i] + eq);
          }
        upload_values(L.ecorr, e.data(), e.size(), fp64, s);
        upload_values(L.dinv, dinv.data(), dinv.size(), fp64, s);
      } else {
        std::vector<double> dinv(A.n);
        for (int64_t i = 0; i < A.n; ++i) dinv[i] = 1.0 / d[i];
        upload_values(L.dinv, dinv.data(), dinv.size(), fp64, s);
      }
      L.off_x = take(A.n);
      L.off_b = take(A.n);
      L.off_r = take(A.n);
      L.off_d0 = take(A.n);
      L.off_d1 = take(A.n);
      H->levels.push_back(std::move(L));
      JFNK_REQUIRE(nagg < A.n, JFNK_E_MESH, "amg: aggregation stalled on a large level");
      A = std::move(Ac);
    }
    H->work_floats = off;
    JFNK_REQUIRE(H->work_floats <= amg_work_floats(m->host.n_cells, m->host.dim), JFNK_E_ARG,
                 "amg: hierarchy larger than the workspace bound");
    H->setup_ms = now_ms() - t0;
  } catch (...) {
    delete H;
    throw;
  }
  slot = H;
}

namespace {

// r64 / z64 (finest level only): the FP64 right-hand side, rounded into b
// by the first smoothing launch, and the FP64 output z = -x, written by the
// last one (the casts need no launches of their own).
template <class T>
void vcycle(const AmgHierarchy& H, size_t l, int degree, T* w, hipStream_t s, const int32_t* gate,
            const double* r64 = nullptr, double* z64 = nullptr) {
  const AmgLevel& L = H.levels[l];
  const int dim = H.dim;
  T* x = w + L.off_x;
  T* b = w + L.off_b;
  if (l + 1 == H.levels.size()) {
    if (r64) amg_cast_in<T>(r64, b, L.n, dim, s, gate);
    if (H.coarse_diag)
      amg_diag_solve<T>(H.coarse_inv.as<T>(), b, x, int(H.n_coarse), dim, s, gate);
    else if (H.n_coarse > kHostDenseMax)
      amg_dense_chunked<T>(H.coarse_inv.as<T>(), b, x, w + H.off_part, int(H.n_coarse), dim, s, gate);
    else
      amg_dense<T>(H.coarse_inv.as<T>(), b, x, int(H.n_coarse), dim, s, gate);
    if (z64) amg_cast_out<T>(x, z64, L.n, dim, s, gate);
    return;
  }
  T* r = w + L.off_r;
  T* d0 = w + L.off_d0;
  T* d1 = w + L.off_d1;
  AmgDiag<T> dinv;
  dinv.dinv = L.dinv.as<T>();
  if (L.ecorr.p != nullptr) {
    dinv.dstride = int(L.n);
    dinv.ecorr = L.ecorr.as<T>();
  }
  ChebCoef cc = cheb_coefficients(L.lmax, degree);
  // pre-smoothing from x = 0
  amg_cheb_start0<T>(L.A, dinv, b, x, r, d0, T(cc.inv_theta), dim, s, gate, r64);
  for (int k = 0; k + 1 < degree; ++k) {
    amg_cheb_step<T>(L.A, dinv, d0, d1, r, x, T(cc.c1[k]), T(cc.c2[k]), dim, s, gate);
    std::swap(d0, d1);
  }
  // coarse-grid correction
  amg_residual<T>(L.A, dinv, b, x, r, dim, s, gate);
  const AmgLevel& C = H.levels[l + 1];
  amg_spmv<T>(L.R, r, w + C.off_b, false, dim, s, gate);
  vcycle<T>(H, l + 1, degree, w, s, gate);
  amg_spmv<T>(L.P, w + C.off_x, x, true, dim, s, gate);
  // post-smoothing; the start's x += d rides on the first step's launch
  d0 = w + L.off_d0;
  d1 = w + L.off_d1;
  const bool steps = degree > 1;
  amg_cheb_start<T>(L.A, dinv, b, x, r, d0, T(cc.inv_theta), dim, s, gate, steps, steps ? nullptr : z64);
  for (int k = 0; k + 1 < degree; ++k) {
    amg_cheb_step<T>(L.A, dinv, d0, d1, r, x, T(cc.c1[k]), T(cc.c2[k]), dim, s, gate, k == 0,
                     k + 2 == degree ? z64 : nullptr);
    std::swap(d0, d1);
  }
}

}  // namespace

// work: the preconditioner region of the solve workspace, holding
// H.work_floats elements of the hierarchy's precision.
void amg_apply(jfnk_mesh* m, bool fp64, int cheb_degree, const double* r, double* z, void* work,
               hipStream_t s, const int32_t* gate) {
  const AmgHierarchy* H = fp64 ? m->amg64 : m->amg;
  JFNK_REQUIRE(H != nullptr, JFNK_E_ARG, "amg: not set up");
  JFNK_REQUIRE(work != nullptr, JFNK_E_ARG, "amg: no workspace");
  Profiler& p = m->prof;
  const int t = p.on ? p.begin(3, s) : -1;
  if (fp64)
    vcycle<double>(*H, 0, cheb_degree, static_cast<double*>(work), s, gate, r, z);
  else
    vcycle<float>(*H, 0, cheb_degree, static_cast<float*>(work), s, gate, r, z);
  if (t >= 0) p.end(t, s);
}

void amg_destroy(AmgHierarchy* a) { delete a; }

void amg_describe(const AmgHierarchy& H, jfnk_amg_info& info) {
  info = jfnk_amg_info{};
  info.n_levels = int32_t(H.levels.size());
  info.coarse_dense = H.coarse_diag ? 0 : 1;
  for (size_t l = 0; l < H.levels.size() && l < 16; ++l) {
    const AmgLevel& L = H.levels[l];
    info.rows[l] = L.n;
    const bool last = l + 1 == H.levels.size();
    info.nnz[l] = last ? 0 : L.A.nnz;
    info.lanes[l] = last ? 0 : L.A.lanes;
  }
  info.operator_complexity = H.op_complexity;
  info.setup_ms = H.setup_ms;
  info.device_bytes = int64_t(amg_device_bytes(&H));
}

size_t amg_device_bytes(const AmgHierarchy* a) {
  if (a == nullptr) return 0;
  size_t b = a->coarse_inv.bytes;
  for (const AmgLevel& L : a->levels)
    b += L.dinv.bytes + L.ecorr.bytes + L.A.ptr.bytes + L.A.col.bytes + L.A.val.bytes + L.P.ptr.bytes + L.P.col.bytes +
         L.P.val.bytes + L.R.ptr.bytes + L.R.col.bytes + L.R.val.bytes;
  return b;
}

}  // namespace jfnk
