// Seeded synthetic H-matrix construction: cluster tree, block tree, kernel
// evaluation, ACA with SVD recompression, and per-block storage-precision
// selection.  This is an input generator shared by the GPU path and by the
// CPU oracle: it holds none of the matrix-vector product arithmetic.
//
// Paper references (Kriemann, "Hierarchical Lowrank Arithmetic with Binary
// Compression"):
//   cluster tree            Sec. 2.1, Definition "Cluster Tree"
//   block tree / leaves     Sec. 2.1, Definition "Block Tree"
//   standard admissibility  Sec. 5.1 (min(diam) <= eta * dist)
//   fixed-accuracy blocks   Sec. 2.1, Eq. (1)
//   ACA                     Sec. 5.1 (low-rank blocks approximated by ACA)
//   SVD truncation          Sec. 2.2, Algorithm 1
//   mixed-precision groups  Sec. 3.3 (W Sigma X^H with per-format column groups)
//   block-relative accuracy Sec. 3 (compression accuracy equals the low-rank eps)
//
// Built with g++ -fopenmp into libhmgen.so and driven from hmgen/build.py.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#include <omp.h>

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Cluster {
  int64_t begin, end;     // half-open range in cluster order
  int32_t son0, son1;     // -1 for leaves
  int32_t level;
  double lo[3], hi[3];    // tight bounding box of the cluster's points
};

struct Block {
  int64_t rb, re, cb, ce;
  int32_t tau, sigma;
  int32_t adm;            // 1: admissible (low rank), 0: dense
  int32_t rank;           // low rank after truncation; 0 for dense
  std::vector<double> a;  // dense D (m x n col-major) or U / W (m x k col-major)
  std::vector<double> b;  // V / X (n x k col-major), low rank only
  std::vector<double> s;  // singular values (k), only when sigma is kept
};

enum Kernel : int32_t {
  K_LAPLACE = 0,   // 1/(4 pi r), diagonal 1/(4 pi h); params[0] = h
  K_EXP = 1,       // exp(-r/l), diagonal 1 + d; params[0] = l, params[1] = d
  K_SEPARABLE = 2, // (1 + p_x) * exp(q_y): exact rank one everywhere
};

}  // namespace

struct hmg_tree {
  int64_t n = 0;
  int32_t leaf = 0;
  double eta = 0;
  std::vector<double> pts;       // original order, n x 3
  std::vector<double> pc;        // cluster order, n x 3
  std::vector<int64_t> perm;     // cluster position -> original index
  std::vector<Cluster> cl;
  std::vector<Block> blocks;
  int32_t kernel = 0;
  double kp[4] = {0, 0, 0, 0};
  int32_t keep_sigma = 0;
  bool filled = false;
};

namespace {

// ---------------------------------------------------------------- geometry

void bbox(const hmg_tree& t, int64_t b, int64_t e, double* lo, double* hi) {
  for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
  for (int64_t i = b; i < e; ++i) {
    const double* p = &t.pts[3 * t.perm[i]];
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
}

double diam(const Cluster& c) {
  double s = 0;
  for (int a = 0; a < 3; ++a) s += (c.hi[a] - c.lo[a]) * (c.hi[a] - c.lo[a]);
  return std::sqrt(s);
}

double dist(const Cluster& x, const Cluster& y) {
  double s = 0;
  for (int a = 0; a < 3; ++a) {
    double d = std::max({0.0, y.lo[a] - x.hi[a], x.lo[a] - y.hi[a]});
    s += d * d;
  }
  return std::sqrt(s);
}

// Binary geometric bisection: split the longest bounding-box edge (lowest
// axis on ties) at its midpoint, points <= mid to the first son.  A split
// that leaves one side empty (coincident points) falls back to the median.
int32_t build_cluster(hmg_tree& t, int64_t b, int64_t e, int32_t level) {
  Cluster c{};
  c.begin = b; c.end = e; c.son0 = c.son1 = -1; c.level = level;
  bbox(t, b, e, c.lo, c.hi);
  int32_t id = (int32_t)t.cl.size();
  t.cl.push_back(c);
  if (e - b <= t.leaf) return id;

  int axis = 0;
  double best = c.hi[0] - c.lo[0];
  for (int a = 1; a < 3; ++a)
    if (c.hi[a] - c.lo[a] > best) { best = c.hi[a] - c.lo[a]; axis = a; }
  const double mid = 0.5 * (c.lo[axis] + c.hi[axis]);
  auto first = t.perm.begin() + b, last = t.perm.begin() + e;
  auto it = std::stable_partition(first, last, [&](int64_t i) {
    return t.pts[3 * i + axis] <= mid;
  });
  int64_t split = b + (it - first);
  if (split == b || split == e) {
    std::stable_sort(first, last, [&](int64_t i, int64_t j) {
      return t.pts[3 * i + axis] < t.pts[3 * j + axis];
    });
    split = b + (e - b) / 2;
  }
  int32_t s0 = build_cluster(t, b, split, level + 1);
  int32_t s1 = build_cluster(t, split, e, level + 1);
  t.cl[id].son0 = s0;
  t.cl[id].son1 = s1;
  return id;
}

bool is_leaf(const Cluster& c) { return c.son0 < 0; }

// Block tree of Sec. 2.1: a block is a leaf if it is admissible or if either
// cluster is a leaf; otherwise both clusters are split together.
void build_blocks(hmg_tree& t, int32_t tau, int32_t sig) {
  const Cluster& x = t.cl[tau];
  const Cluster& y = t.cl[sig];
  double d = dist(x, y);
  bool adm = d > 0 && std::min(diam(x), diam(y)) <= t.eta * d;
  if (adm || is_leaf(x) || is_leaf(y)) {
    Block bl;
    bl.rb = x.begin; bl.re = x.end; bl.cb = y.begin; bl.ce = y.end;
    bl.tau = tau; bl.sigma = sig; bl.adm = adm ? 1 : 0; bl.rank = 0;
    t.blocks.push_back(std::move(bl));
    return;
  }
  int32_t xs[2] = {x.son0, x.son1}, ys[2] = {y.son0, y.son1};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) build_blocks(t, xs[i], ys[j]);
}

// ---------------------------------------------------------------- kernels

struct Eval {
  const hmg_tree& t;
  double operator()(int64_t i, int64_t j) const {
    const double* p = &t.pc[3 * i];
    const double* q = &t.pc[3 * j];
    switch (t.kernel) {
      case K_LAPLACE: {
        if (i == j) return 1.0 / (4.0 * kPi * t.kp[0]);
        double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        return 1.0 / (4.0 * kPi * std::sqrt(dx * dx + dy * dy + dz * dz));
      }
      case K_EXP: {
        double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        double v = std::exp(-std::sqrt(dx * dx + dy * dy + dz * dz) / t.kp[0]);
        return i == j ? v + t.kp[1] : v;
      }
      default:
        return (1.0 + p[0]) * std::exp(q[1]);
    }
  }
};

// ---------------------------------------------------------------- dense LA

// Householder QR of A (m x r, col-major, m >= r): A is overwritten with the
// explicit Q (m x r); R (r x r, col-major, upper triangular) is returned.
void qr_explicit(std::vector<double>& A, int64_t m, int r, std::vector<double>& R) {
  std::vector<double> tau(r, 0.0);
  for (int k = 0; k < r; ++k) {
    double* a = &A[(size_t)k * m];
    double nrm = 0;
    for (int64_t i = k; i < m; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0) { tau[k] = 0; continue; }
    double alpha = a[k] > 0 ? -nrm : nrm;   // new diagonal
    double v0 = a[k] - alpha;
    // v = [1, a[k+1..]/v0], tau = -v0/alpha
    for (int64_t i = k + 1; i < m; ++i) a[i] /= v0;
    tau[k] = -v0 / alpha;
    a[k] = alpha;
    for (int j = k + 1; j < r; ++j) {
      double* c = &A[(size_t)j * m];
      double s = c[k];
      for (int64_t i = k + 1; i < m; ++i) s += a[i] * c[i];
      s *= tau[k];
      c[k] -= s;
      for (int64_t i = k + 1; i < m; ++i) c[i] -= s * a[i];
    }
  }
  R.assign((size_t)r * r, 0.0);
  for (int j = 0; j < r; ++j)
    for (int i = 0; i <= j; ++i) R[(size_t)j * r + i] = A[(size_t)j * m + i];
  // Accumulate Q = H_0 ... H_{r-1} [I; 0] backwards, in place.
  std::vector<double> Q((size_t)m * r, 0.0);
  for (int j = 0; j < r; ++j) Q[(size_t)j * m + j] = 1.0;
  for (int k = r - 1; k >= 0; --k) {
    if (tau[k] == 0) continue;
    const double* v = &A[(size_t)k * m];
    for (int j = k; j < r; ++j) {
      double* q = &Q[(size_t)j * m];
      double s = q[k];
      for (int64_t i = k + 1; i < m; ++i) s += v[i] * q[i];
      s *= tau[k];
      q[k] -= s;
      for (int64_t i = k + 1; i < m; ++i) q[i] -= s * v[i];
    }
  }
  A.swap(Q);
}

// One-sided Jacobi SVD of a square r x r matrix B (col-major):
// B = Us diag(S) Vs^T with S sorted descending.
void jacobi_svd(const std::vector<double>& B, int r, std::vector<double>& Us,
                std::vector<double>& S, std::vector<double>& Vs) {
  std::vector<double> A = B;
  Vs.assign((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i) Vs[(size_t)i * r + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int p = 0; p < r - 1; ++p)
      for (int q = p + 1; q < r; ++q) {
        double* ap = &A[(size_t)p * r];
        double* aq = &A[(size_t)q * r];
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < r; ++i) {
          alpha += ap[i] * ap[i];
          beta += aq[i] * aq[i];
          gamma += ap[i] * aq[i];
        }
        if (gamma == 0) continue;
        double rel = std::fabs(gamma) / std::sqrt(alpha * beta);
        if (!(rel > 1e-15)) continue;
        off = std::max(off, rel);
        double zeta = (beta - alpha) / (2.0 * gamma);
        double tt = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + tt * tt), s = c * tt;
        for (int i = 0; i < r; ++i) {
          double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = &Vs[(size_t)p * r];
        double* vq = &Vs[(size_t)q * r];
        for (int i = 0; i < r; ++i) {
          double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (off <= 1e-15) break;
  }
  std::vector<double> nrm(r);
  for (int j = 0; j < r; ++j) {
    double s = 0;
    for (int i = 0; i < r; ++i) s += A[(size_t)j * r + i] * A[(size_t)j * r + i];
    nrm[j] = std::sqrt(s);
  }
  std::vector<int> order(r);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  Us.assign((size_t)r * r, 0.0);
  S.assign(r, 0.0);
  std::vector<double> V2((size_t)r * r);
  for (int jj = 0; jj < r; ++jj) {
    int j = order[jj];
    S[jj] = nrm[j];
    for (int i = 0; i < r; ++i) {
      Us[(size_t)jj * r + i] = nrm[j] > 0 ? A[(size_t)j * r + i] / nrm[j] : 0.0;
      V2[(size_t)jj * r + i] = Vs[(size_t)j * r + i];
    }
  }
  Vs.swap(V2);
}

// ---------------------------------------------------------------- ACA

// Partially pivoted adaptive cross approximation of block (rb.., cb..):
// first pivot row is the block's first row, next row is the argmax of the
// newest column over unused rows, column pivot is the argmax of the residual
// row; stop when |u_k||v_k| <= eps * |S_k|_F.  Returns rank r and fills
// U (m x r) and V (n x r) col-major so that the block ~ U V^T.
int aca(const Eval& ev, int64_t rb, int64_t m, int64_t cb, int64_t n, double eps,
        std::vector<double>& U, std::vector<double>& V) {
  const int64_t kmax = std::min(m, n);
  U.clear(); V.clear();
  std::vector<char> used(m, 0);
  std::vector<double> row(n), col(m);
  double normS2 = 0;
  int r = 0;
  int64_t i = 0;
  int64_t nused = 0;
  while (r < kmax && nused < m) {
    for (int64_t j = 0; j < n; ++j) row[j] = ev(rb + i, cb + j);
    for (int l = 0; l < r; ++l) {
      double ul = U[(size_t)l * m + i];
      const double* vl = &V[(size_t)l * n];
      for (int64_t j = 0; j < n; ++j) row[j] -= ul * vl[j];
    }
    used[i] = 1; ++nused;
    int64_t jp = 0;
    double best = std::fabs(row[0]);
    for (int64_t j = 1; j < n; ++j)
      if (std::fabs(row[j]) > best) { best = std::fabs(row[j]); jp = j; }
    if (best == 0) {
      int64_t nxt = -1;
      for (int64_t ii = 0; ii < m; ++ii) if (!used[ii]) { nxt = ii; break; }
      if (nxt < 0) break;
      i = nxt;
      continue;
    }
    const double piv = row[jp];
    for (int64_t ii = 0; ii < m; ++ii) col[ii] = ev(rb + ii, cb + jp);
    for (int l = 0; l < r; ++l) {
      double vl = V[(size_t)l * n + jp];
      const double* ul = &U[(size_t)l * m];
      for (int64_t ii = 0; ii < m; ++ii) col[ii] -= vl * ul[ii];
    }
    for (int64_t j = 0; j < n; ++j) row[j] /= piv;
    double nu = 0, nv = 0;
    for (int64_t ii = 0; ii < m; ++ii) nu += col[ii] * col[ii];
    for (int64_t j = 0; j < n; ++j) nv += row[j] * row[j];
    double cross = 0;
    for (int l = 0; l < r; ++l) {
      const double* ul = &U[(size_t)l * m];
      const double* vl = &V[(size_t)l * n];
      double a = 0, b = 0;
      for (int64_t ii = 0; ii < m; ++ii) a += col[ii] * ul[ii];
      for (int64_t j = 0; j < n; ++j) b += row[j] * vl[j];
      cross += a * b;
    }
    normS2 += 2.0 * cross + nu * nv;
    U.insert(U.end(), col.begin(), col.end());
    V.insert(V.end(), row.begin(), row.end());
    ++r;
    if (std::sqrt(nu * nv) <= eps * std::sqrt(std::fabs(normS2))) break;
    int64_t nxt = -1;
    double bu = -1;
    for (int64_t ii = 0; ii < m; ++ii)
      if (!used[ii] && std::fabs(col[ii]) > bu) { bu = std::fabs(col[ii]); nxt = ii; }
    if (nxt < 0) break;
    i = nxt;
  }
  return r;
}

// Algorithm 1 (truncation via QR + SVD).  rank() = smallest k whose
// Frobenius tail of singular values is <= eps times the total.  Columns of
// the SVD factors are the singular vectors.  Output W = Q_U U_s(:,1:k),
// X = Q_V V_s(:,1:k), S = S_s(1:k).
int truncate(std::vector<double>& U, std::vector<double>& V, int64_t m, int64_t n,
             int r, double eps, std::vector<double>& W, std::vector<double>& X,
             std::vector<double>& S) {
  if (r == 0) { W.clear(); X.clear(); S.clear(); return 0; }
  std::vector<double> RU, RV;
  qr_explicit(U, m, r, RU);
  qr_explicit(V, n, r, RV);
  std::vector<double> B((size_t)r * r, 0.0);   // R_U * R_V^T
  for (int j = 0; j < r; ++j)
    for (int l = 0; l < r; ++l) {
      double rv = RV[(size_t)l * r + j];          // R_V(j, l)
      if (rv == 0) continue;
      for (int i = 0; i < r; ++i) B[(size_t)j * r + i] += RU[(size_t)l * r + i] * rv;
    }
  std::vector<double> Us, Ss, Vs;
  jacobi_svd(B, r, Us, Ss, Vs);
  double tot = 0;
  for (double s : Ss) tot += s * s;
  int k = r;
  double tail = 0;
  // smallest k with sqrt(sum_{j>=k} s_j^2) <= eps * sqrt(tot)
  while (k > 0) {
    double t2 = tail + Ss[k - 1] * Ss[k - 1];
    if (std::sqrt(t2) <= eps * std::sqrt(tot)) { tail = t2; --k; } else break;
  }
  W.assign((size_t)m * k, 0.0);
  X.assign((size_t)n * k, 0.0);
  for (int c = 0; c < k; ++c)
    for (int l = 0; l < r; ++l) {
      double a = Us[(size_t)c * r + l], b = Vs[(size_t)c * r + l];
      const double* qu = &U[(size_t)l * m];
      const double* qv = &V[(size_t)l * n];
      double* w = &W[(size_t)c * m];
      double* x = &X[(size_t)c * n];
      for (int64_t i = 0; i < m; ++i) w[i] += qu[i] * a;
      for (int64_t i = 0; i < n; ++i) x[i] += qv[i] * b;
    }
  S.assign(Ss.begin(), Ss.begin() + k);
  return k;
}

// ---------------------------------------------------------------- rounding

// Round-to-nearest-even of a double to a binary format with p significand
// bits (implicit bit included), minimum normal exponent emin (value 2^emin)
// and largest finite value fmax; values above fmax overflow to infinity.
double round_fmt(double x, int p, int emin, double fmax) {
  if (x == 0 || !std::isfinite(x)) return x;
  int e;
  std::frexp(x, &e);            // |x| in [2^(e-1), 2^e)
  int q = std::max(e - 1, emin) - (p - 1);   // exponent of the last kept bit
  double scaled = std::ldexp(x, -q);
  double r = std::nearbyint(scaled);          // ties to even (default mode)
  double y = std::ldexp(r, q);
  if (std::fabs(y) > fmax) return x > 0 ? INFINITY : -INFINITY;
  return y;
}

enum Dt : int32_t {
  DT_F64 = 0, DT_F32 = 1, DT_F16 = 2, DT_BF16 = 3,
  DT_DFL32 = 4, DT_DFL40 = 5, DT_DFL48 = 6, DT_DFL16 = 7, DT_DFL24 = 8
};

// Bytes of a DFL format (Sec. 3.2: FP64's sign and exponent, the mantissa
// cut to whole bytes), 0 for the others.
int dfl_nbytes(int dt) {
  switch (dt) {
    case DT_DFL16: return 2;
    case DT_DFL24: return 3;
    case DT_DFL32: return 4;
    case DT_DFL40: return 5;
    case DT_DFL48: return 6;
    default: return 0;
  }
}

double rnd(double x, int dt) {
  switch (dt) {
    case DT_F32: return round_fmt(x, 24, -126, 3.4028234663852886e38);
    case DT_F16: return round_fmt(x, 11, -14, 65504.0);
    case DT_BF16: return round_fmt(x, 8, -126, 3.3895313892515355e38);
    default:
      if (int nb = dfl_nbytes(dt)) return round_fmt(x, 8 * nb - 11, -1022, 1.7976931348623157e308);
      return x;
  }
}

int dt_bytes(int dt) {
  if (int nb = dfl_nbytes(dt)) return nb;
  return dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2;
}

// Explicit mantissa bits an AFLP data block of nbytes-byte values keeps
// (Sec. 3.2): values scaled by the power of two 2^k at or below the smallest
// nonzero magnitude and shifted by 1 (d = |v| 2^-k + 1 >= 2); the exponent
// field takes the fewest bits e that hold the binary exponent of every
// rounded d, the mantissa the rest of the bytes, 8 nbytes - 1 - e.  -1 when
// no e <= 10 fits.
int aflp_mantissa(const double* v, size_t n, int nbytes) {
  double mn = HUGE_VAL, mx = 0;
  for (size_t i = 0; i < n; ++i) {
    const double a = std::fabs(v[i]);
    if (a > 0) { mn = std::min(mn, a); mx = std::max(mx, a); }
  }
  if (mx == 0) return 8 * nbytes - 1;
  const int k = std::ilogb(mn);                      // 2^k <= mn < 2^(k+1)
  const double dmax = std::ldexp(mx, -k) + 1.0;
  if (!std::isfinite(dmax)) return -1;
  const int top = std::ilogb(dmax);
  int e = 0;
  while ((1 << e) <= top) ++e;
  for (; e <= 10; ++e) {
    const int m = 8 * nbytes - 1 - e;
    if (m < 1) return -1;
    // dmax rounded to m mantissa bits (nearest, ties to even)
    const double q = std::ldexp(dmax, m - top);
    double r = std::nearbyint(q);
    if (std::ilogb(std::ldexp(r, top - m)) < (1 << e)) return m;
  }
  return -1;
}

}  // namespace

// ====================================================================== C API
extern "C" {

int hmg_build_tree(const double* pts, int64_t n, int32_t leaf, double eta, hmg_tree** out) {
  if (!pts || n <= 0 || leaf <= 0 || !out || !(eta >= 0)) return -1;
  hmg_tree* t = new hmg_tree();
  t->n = n; t->leaf = leaf; t->eta = eta;
  t->pts.assign(pts, pts + 3 * n);
  t->perm.resize(n);
  std::iota(t->perm.begin(), t->perm.end(), 0);
  build_cluster(*t, 0, n, 0);
  t->pc.resize(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) t->pc[3 * i + a] = t->pts[3 * t->perm[i] + a];
  build_blocks(*t, 0, 0);
  std::stable_sort(t->blocks.begin(), t->blocks.end(), [](const Block& x, const Block& y) {
    return x.rb != y.rb ? x.rb < y.rb : x.cb < y.cb;
  });
  *out = t;
  return 0;
}

void hmg_destroy(hmg_tree* t) { delete t; }

int64_t hmg_num_clusters(const hmg_tree* t) { return (int64_t)t->cl.size(); }
int64_t hmg_num_blocks(const hmg_tree* t) { return (int64_t)t->blocks.size(); }

void hmg_get_perm(const hmg_tree* t, int64_t* perm) {
  std::copy(t->perm.begin(), t->perm.end(), perm);
}

void hmg_get_clusters(const hmg_tree* t, int64_t* begin, int64_t* end, int32_t* son0,
                      int32_t* son1, int32_t* level, double* box) {
  for (size_t c = 0; c < t->cl.size(); ++c) {
    const Cluster& x = t->cl[c];
    begin[c] = x.begin; end[c] = x.end; son0[c] = x.son0; son1[c] = x.son1;
    level[c] = x.level;
    for (int a = 0; a < 3; ++a) { box[6 * c + a] = x.lo[a]; box[6 * c + 3 + a] = x.hi[a]; }
  }
}

void hmg_get_blocks(const hmg_tree* t, int64_t* rb, int64_t* re, int64_t* cb, int64_t* ce,
                    int32_t* adm, int32_t* tau, int32_t* sigma, int32_t* rank) {
  for (size_t i = 0; i < t->blocks.size(); ++i) {
    const Block& b = t->blocks[i];
    rb[i] = b.rb; re[i] = b.re; cb[i] = b.cb; ce[i] = b.ce;
    adm[i] = b.adm; tau[i] = b.tau; sigma[i] = b.sigma; rank[i] = b.rank;
  }
}

// Fill every leaf: dense entries for inadmissible leaves, ACA (tolerance
// eps_aca) followed by Algorithm 1 at eps for admissible ones.  With
// keep_sigma = 0 the singular values are folded into the first factor
// (U = W diag(S), V = X); otherwise W, S, X are kept separately.
// hmg_fill_part fills share `part` of `nparts` (blocks in size order, dealt
// round-robin, so every share has the same mix of sizes); calling it for
// part = 0 .. nparts-1 fills every block, exactly as hmg_fill does.
int hmg_fill_part(hmg_tree* t, int32_t kernel, const double* params, double eps_aca, double eps,
                  int32_t keep_sigma, int32_t nthreads, int32_t part, int32_t nparts) {
  if (!t || kernel < 0 || kernel > 2 || nparts < 1 || part < 0 || part >= nparts) return -1;
  if (part == 0) {
    t->kernel = kernel;
    for (int i = 0; i < 4; ++i) t->kp[i] = params ? params[i] : 0.0;
    t->keep_sigma = keep_sigma;
    t->filled = false;
  }
  Eval ev{*t};
  const int64_t nb = (int64_t)t->blocks.size();
  // Largest blocks first for load balance.
  std::vector<int64_t> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    const Block& a = t->blocks[x];
    const Block& b = t->blocks[y];
    return (a.re - a.rb) + (a.ce - a.cb) > (b.re - b.rb) + (b.ce - b.cb);
  });
  const int64_t nmine = nb > part ? (nb - part + nparts - 1) / nparts : 0;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  std::atomic<int> err{0};
#pragma omp parallel
  {
    std::vector<double> U, V, W, X, S;
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < nmine; ++q) {
      Block& b = t->blocks[order[part + q * nparts]];
      const int64_t m = b.re - b.rb, n = b.ce - b.cb;
      b.a.clear(); b.b.clear(); b.s.clear();
      if (!b.adm) {
        b.a.resize((size_t)m * n);
        for (int64_t j = 0; j < n; ++j)
          for (int64_t i = 0; i < m; ++i) b.a[(size_t)j * m + i] = ev(b.rb + i, b.cb + j);
        b.rank = 0;
        continue;
      }
      int r = aca(ev, b.rb, m, b.cb, n, eps_aca, U, V);
      int k = truncate(U, V, m, n, r, eps, W, X, S);
      b.rank = k;
      if (!keep_sigma)
        for (int c = 0; c < k; ++c)
          for (int64_t i = 0; i < m; ++i) W[(size_t)c * m + i] *= S[c];
      b.a = W;
      b.b = X;
      if (keep_sigma) b.s = S;
    }
  }
  if (part == nparts - 1) t->filled = err.load() == 0;
  return err.load();
}

int hmg_fill(hmg_tree* t, int32_t kernel, const double* params, double eps_aca, double eps,
             int32_t keep_sigma, int32_t nthreads) {
  return hmg_fill_part(t, kernel, params, eps_aca, eps, keep_sigma, nthreads, 0, 1);
}

// Kernel function and form of the leaves, for trees whose leaves are filled
// elsewhere (hmg_set_factors) or one by one (hmg_fill_blocks).
int hmg_set_kernel(hmg_tree* t, int32_t kernel, const double* params, int32_t keep_sigma) {
  if (!t || kernel < 0 || kernel > 2) return -1;
  t->kernel = kernel;
  for (int i = 0; i < 4; ++i) t->kp[i] = params ? params[i] : 0.0;
  t->keep_sigma = keep_sigma;
  return 0;
}

// Copies computed factors into `count` leaves idx[q] (data movement only).
// Leaf q's data start at buf + off[q]: a dense leaf's D (m x n); an
// admissible leaf's U / W (m x rank[q]) at column stride m, V / X (n x
// rank[q]) from off[q] + m cap[q], and with keep_sigma its s from
// off[q] + (m + n) cap[q].
int hmg_set_factors(hmg_tree* t, int64_t count, const int64_t* idx, const int32_t* rank, const double* buf,
                    const int64_t* off, const int32_t* cap) {
  if (!t) return -1;
  const int64_t nb = (int64_t)t->blocks.size();
  for (int64_t q = 0; q < count; ++q)
    if (idx[q] < 0 || idx[q] >= nb || rank[q] < 0) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < count; ++q) {
    Block& b = t->blocks[idx[q]];
    const int64_t m = b.re - b.rb, n = b.ce - b.cb;
    const double* p = buf + off[q];
    b.b.clear();
    b.s.clear();
    if (!b.adm) {
      b.a.assign(p, p + m * n);
      b.rank = 0;
      continue;
    }
    const int64_t k = rank[q], c = cap[q];
    b.a.assign(p, p + m * k);
    b.b.assign(p + m * c, p + m * c + n * k);
    if (t->keep_sigma) b.s.assign(p + (m + n) * c, p + (m + n) * c + k);
    b.rank = (int32_t)k;
  }
  return 0;
}

// Fills the leaves idx[0 .. count-1] on the host, as hmg_fill does, with the
// kernel set by hmg_set_kernel.
int hmg_fill_blocks(hmg_tree* t, int64_t count, const int64_t* idx, double eps_aca, double eps,
                    int32_t nthreads) {
  if (!t) return -1;
  const int64_t nb = (int64_t)t->blocks.size();
  for (int64_t q = 0; q < count; ++q)
    if (idx[q] < 0 || idx[q] >= nb) return -1;
  Eval ev{*t};
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
    std::vector<double> U, V, W, X, S;
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < count; ++q) {
      Block& b = t->blocks[idx[q]];
      const int64_t m = b.re - b.rb, n = b.ce - b.cb;
      b.a.clear(); b.b.clear(); b.s.clear();
      if (!b.adm) {
        b.a.resize((size_t)m * n);
        for (int64_t j = 0; j < n; ++j)
          for (int64_t i = 0; i < m; ++i) b.a[(size_t)j * m + i] = ev(b.rb + i, b.cb + j);
        b.rank = 0;
        continue;
      }
      int r = aca(ev, b.rb, m, b.cb, n, eps_aca, U, V);
      int k = truncate(U, V, m, n, r, eps, W, X, S);
      b.rank = k;
      if (!t->keep_sigma)
        for (int c = 0; c < k; ++c)
          for (int64_t i = 0; i < m; ++i) W[(size_t)c * m + i] *= S[c];
      b.a = W;
      b.b = X;
      if (t->keep_sigma) b.s = S;
    }
  }
  return 0;
}

// Per-block factor pointers (0 where absent) as integers, for marshalling.
void hmg_get_factor_ptrs(const hmg_tree* t, uint64_t* a, uint64_t* b, uint64_t* s) {
  for (size_t i = 0; i < t->blocks.size(); ++i) {
    const Block& bl = t->blocks[i];
    a[i] = bl.a.empty() ? 0 : (uint64_t)(uintptr_t)bl.a.data();
    b[i] = bl.b.empty() ? 0 : (uint64_t)(uintptr_t)bl.b.data();
    s[i] = bl.s.empty() ? 0 : (uint64_t)(uintptr_t)bl.s.data();
  }
}

void hmg_get_ranks(const hmg_tree* t, int32_t* rank) {
  for (size_t i = 0; i < t->blocks.size(); ++i) rank[i] = t->blocks[i].rank;
}

// Evaluate the kernel on an explicit list of (row, col) pairs in cluster
// order (used to check blocks against the generating function).
void hmg_eval(const hmg_tree* t, const int64_t* rows, const int64_t* cols, int64_t cnt,
              double* out) {
  Eval ev{*t};
  for (int64_t i = 0; i < cnt; ++i) out[i] = ev(rows[i], cols[i]);
}

// Per-block storage precision (needs keep_sigma = 1 for low-rank blocks).
// Every block is held to the block-relative accuracy used for the low-rank
// approximation itself (Sec. 3, Eq. (1)): |M_b - fl(M_b)|_F <= tol |M_b|_F.
// Dense blocks take the cheapest whole-block format that meets it.  Low-rank
// blocks W diag(S) X^T split their columns into format groups (Sec. 3.3):
// starting from all columns (and S) in FP32, columns are lowered from the
// smallest singular value upward to FP16 (or BF16 where FP16 overflows)
// while the sum of per-column errors stays within the budget; the sum is a
// rigorous bound by the triangle inequality.
// flags: bit 0 (allow FP64) lets a block whose FP32 error alone exceeds the
// budget fall back to FP64; bit 1 (dense FP64) keeps every dense block in
// FP64; bit 2 (s in FP64) prices the columns with s exact, for products
// that accumulate in FP64 and keep s in FP64.
// Output per block: ngroups, group_cols[4], group_dtype[4]; for low-rank
// blocks the groups are in column order (largest singular values first).
// Returns the number of blocks whose storage misses the budget (or that
// need more than 4 column groups); 0 when every block meets it.
int hmg_select_precision(const hmg_tree* t, double tol, int32_t flags, int32_t* ngroups,
                         int32_t* group_cols, int32_t* group_dtype, double* err_bound) {
  const bool allow_f64 = flags & 1, dense_f64 = flags & 2, sigma_f64 = flags & 4;
  const int64_t nb = (int64_t)t->blocks.size();
  std::atomic<int> bad{0};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t bi = 0; bi < nb; ++bi) {
    const Block& b = t->blocks[bi];
    const int64_t m = b.re - b.rb, n = b.ce - b.cb;
    int32_t* gc = &group_cols[4 * bi];
    int32_t* gd = &group_dtype[4 * bi];
    for (int q = 0; q < 4; ++q) { gc[q] = 0; gd[q] = 0; }
    if (!b.adm) {
      double nrm2 = 0;
      for (double v : b.a) nrm2 += v * v;
      const double budget = tol * std::sqrt(nrm2);
      int chosen = DT_F64;
      double chosen_err = 0;
      const int cands[3] = {DT_F16, DT_BF16, DT_F32};
      for (int dt : cands) {
        if (dense_f64) break;
        double e2 = 0;
        bool fin = true;
        for (double v : b.a) {
          double r = rnd(v, dt);
          if (!std::isfinite(r)) { fin = false; break; }
          e2 += (v - r) * (v - r);
        }
        if (fin && std::sqrt(e2) <= budget) { chosen = dt; chosen_err = std::sqrt(e2); break; }
      }
      if (chosen == DT_F64 && !allow_f64 && !dense_f64) {
        double e2 = 0;
        for (double v : b.a) { double r = rnd(v, DT_F32); e2 += (v - r) * (v - r); }
        chosen = DT_F32; chosen_err = std::sqrt(e2); bad.fetch_add(1);
      }
      ngroups[bi] = 1; gc[0] = 0; gd[0] = chosen;
      if (err_bound) err_bound[bi] = chosen_err;
      continue;
    }
    const int k = b.rank;
    if (k == 0) { ngroups[bi] = 1; gc[0] = 0; gd[0] = DT_F32; if (err_bound) err_bound[bi] = 0; continue; }
    if (b.s.empty()) { bad.fetch_add(1); ngroups[bi] = 0; continue; }
    double nrm2 = 0;
    for (double s : b.s) nrm2 += s * s;
    const double budget = tol * std::sqrt(nrm2);
    // e[c][dt]: exact Frobenius error of column c's rank-one term
    // s w x^T when w, x and s are rounded to format dt (s to FP32 unless dt is
    // FP64).  Computed as |a x^T + s^ w^ d^T| with a = s w - s^ w^, d = x - x^.
    auto col_err = [&](int c, int dt, bool& finite) {
      const double* w = &b.a[(size_t)c * m];
      const double* x = &b.b[(size_t)c * n];
      const double s = b.s[c];
      const double sh = dt == DT_F64 || sigma_f64 ? s : rnd(s, DT_F32);
      double aa = 0, xx = 0, wh2 = 0, dd = 0, aw = 0, xd = 0;
      finite = true;
      for (int64_t i = 0; i < m; ++i) {
        double wh = rnd(w[i], dt);
        if (!std::isfinite(wh)) finite = false;
        double a = s * w[i] - sh * wh;
        aa += a * a; wh2 += wh * wh; aw += a * wh;
      }
      for (int64_t i = 0; i < n; ++i) {
        double xh = rnd(x[i], dt);
        if (!std::isfinite(xh)) finite = false;
        double d = x[i] - xh;
        xx += x[i] * x[i]; dd += d * d; xd += x[i] * d;
      }
      double e2 = aa * xx + sh * sh * wh2 * dd + 2.0 * sh * aw * xd;
      return std::sqrt(std::max(e2, 0.0));
    };
    std::vector<int> fmt(k, DT_F32);
    std::vector<double> e32(k);
    double sum32 = 0;
    bool fin;
    for (int c = 0; c < k; ++c) { e32[c] = col_err(c, DT_F32, fin); sum32 += e32[c]; }
    double total = sum32;
    if (sum32 > budget) {
      if (allow_f64) {
        // Promote leading columns to FP64 until the FP32 remainder fits.
        for (int c = 0; c < k && total > budget; ++c) { fmt[c] = DT_F64; total -= e32[c]; }
      } else {
        bad.fetch_add(1);
      }
    } else {
      double room = budget - sum32;
      for (int c = k - 1; c >= 0; --c) {
        double e16 = col_err(c, DT_F16, fin);
        if (fin && e16 - e32[c] <= room) { fmt[c] = DT_F16; room -= e16 - e32[c]; total += e16 - e32[c]; continue; }
        double eb = col_err(c, DT_BF16, fin);
        if (fin && eb - e32[c] <= room) { fmt[c] = DT_BF16; room -= eb - e32[c]; total += eb - e32[c]; continue; }
        break;
      }
    }
    // Contiguous groups in column order.
    int ng = 0;
    for (int c = 0; c < k; ++c) {
      if (ng == 0 || gd[ng - 1] != fmt[c]) {
        if (ng == 4) { bad.fetch_add(1); break; }
        gd[ng] = fmt[c]; gc[ng] = 0; ++ng;
      }
      gc[ng - 1] += 1;
    }
    ngroups[bi] = ng;
    if (err_bound) err_bound[bi] = total;
  }
  return bad.load();
}

// Adaptive per-column precision (APLR, Sec. 3.3) over the DFL formats, for
// FP64 accumulation with s_b kept in FP64.  Every block is held to
// ||M_b - M^_b||_F <= tol ||M_b||_F.  Dense blocks take the narrowest DFL
// format whose exact error meets it, else FP64.  Low-rank blocks: columns go
// from the smallest singular value up, each to the narrowest format (DFL16,
// DFL24, DFL32, DFL40, DFL48, FP64) that is at least as wide as the next
// column's and whose exact error (as in hmg_select_precision, with s exact)
// fits what is left of the budget; formats then rise towards the large
// singular values, and the narrowest groups are widened until at most 4
// remain.  err_bound: the sum of the exact column errors (a bound by the
// triangle inequality).
// AFLP storage per block (one format for all its columns): the fewest bytes
// B in 2 .. 6 whose AFLP mantissa reaches mant_bits for every data block of
// the block (D_b; U_b and V_b share B), as AFLP16 ... AFLP48 (9 .. 13); FP64
// where no B does.  Returns the number of blocks left in FP64.
int hmg_select_aflp(const hmg_tree* t, int mant_bits, int32_t* ngroups, int32_t* group_cols,
                    int32_t* group_dtype) {
  const int64_t nb = (int64_t)t->blocks.size();
  std::atomic<int> f64{0};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t bi = 0; bi < nb; ++bi) {
    const Block& b = t->blocks[bi];
    int32_t* gc = &group_cols[4 * bi];
    int32_t* gd = &group_dtype[4 * bi];
    for (int q = 0; q < 4; ++q) { gc[q] = 0; gd[q] = 0; }
    ngroups[bi] = 1;
    gc[0] = b.adm ? b.rank : 0;
    int chosen = DT_F64;
    for (int B = 2; B <= 6; ++B) {
      bool fits = aflp_mantissa(b.a.data(), b.a.size(), B) >= mant_bits;
      if (fits && b.adm) fits = aflp_mantissa(b.b.data(), b.b.size(), B) >= mant_bits;
      if (fits) { chosen = 9 + (B - 2); break; }
    }
    if (chosen == DT_F64) f64.fetch_add(1);
    gd[0] = chosen;
  }
  return f64.load();
}

int hmg_select_precision_dfl(const hmg_tree* t, double tol, int32_t* ngroups, int32_t* group_cols,
                             int32_t* group_dtype, double* err_bound) {
  static const int kWidth[6] = {DT_DFL16, DT_DFL24, DT_DFL32, DT_DFL40, DT_DFL48, DT_F64};
  const int64_t nb = (int64_t)t->blocks.size();
  std::atomic<int> bad{0};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t bi = 0; bi < nb; ++bi) {
    const Block& b = t->blocks[bi];
    const int64_t m = b.re - b.rb, n = b.ce - b.cb;
    int32_t* gc = &group_cols[4 * bi];
    int32_t* gd = &group_dtype[4 * bi];
    for (int q = 0; q < 4; ++q) { gc[q] = 0; gd[q] = 0; }
    if (!b.adm) {
      double nrm2 = 0;
      for (double v : b.a) nrm2 += v * v;
      const double budget = tol * std::sqrt(nrm2);
      int chosen = DT_F64;
      double chosen_err = 0;
      for (int w = 0; w < 5; ++w) {
        double e2 = 0;
        for (double v : b.a) { const double r = rnd(v, kWidth[w]); e2 += (v - r) * (v - r); }
        if (std::sqrt(e2) <= budget) { chosen = kWidth[w]; chosen_err = std::sqrt(e2); break; }
      }
      ngroups[bi] = 1; gc[0] = 0; gd[0] = chosen;
      if (err_bound) err_bound[bi] = chosen_err;
      continue;
    }
    const int k = b.rank;
    if (k == 0) { ngroups[bi] = 1; gc[0] = 0; gd[0] = DT_DFL16; if (err_bound) err_bound[bi] = 0; continue; }
    if (b.s.empty()) { bad.fetch_add(1); ngroups[bi] = 0; continue; }
    double nrm2 = 0;
    for (double s : b.s) nrm2 += s * s;
    const double budget = tol * std::sqrt(nrm2);
    // exact Frobenius error of column c's term s w x^T with w and x rounded
    // to format dt and s exact: |a x^T + s w^ d^T|, a = s (w - w^), d = x - x^
    auto col_err = [&](int c, int dt) {
      const double* w = &b.a[(size_t)c * m];
      const double* x = &b.b[(size_t)c * n];
      const double s = b.s[c];
      double aa = 0, xx = 0, wh2 = 0, dd = 0, aw = 0, xd = 0;
      for (int64_t i = 0; i < m; ++i) {
        const double wh = rnd(w[i], dt), a = s * (w[i] - wh);
        aa += a * a; wh2 += wh * wh; aw += a * wh;
      }
      for (int64_t i = 0; i < n; ++i) {
        const double xh = rnd(x[i], dt), d = x[i] - xh;
        xx += x[i] * x[i]; dd += d * d; xd += x[i] * d;
      }
      const double e2 = aa * xx + s * s * wh2 * dd + 2.0 * s * aw * xd;
      return std::sqrt(std::max(e2, 0.0));
    };
    std::vector<int> wi(k, 5);                      // width index per column
    std::vector<double> err(k, 0.0);
    double room = budget;
    int lo = 0;                                     // narrowest width allowed (the next column's)
    for (int c = k - 1; c >= 0; --c) {
      int w = lo;
      for (; w < 5; ++w) {
        const double e = col_err(c, kWidth[w]);
        if (e <= room) { err[c] = e; room -= e; break; }
      }
      wi[c] = w;                                    // w == 5: FP64, no error
      lo = w;
    }
    // at most 4 groups: widen the narrowest groups (less error, still in budget)
    for (;;) {
      int distinct = 0, narrowest = 6;
      for (int w = 0; w < 6; ++w) {
        bool any = false;
        for (int c = 0; c < k; ++c) any = any || wi[c] == w;
        if (any) { ++distinct; narrowest = std::min(narrowest, w); }
      }
      if (distinct <= 4) break;
      int next = narrowest + 1;
      for (;; ++next) {
        bool any = false;
        for (int c = 0; c < k; ++c) any = any || wi[c] == next;
        if (any) break;
      }
      for (int c = 0; c < k; ++c)
        if (wi[c] == narrowest) { wi[c] = next; err[c] = next == 5 ? 0.0 : col_err(c, kWidth[next]); }
    }
    double total = 0;
    for (int c = 0; c < k; ++c) total += err[c];
    int ng = 0;
    for (int c = 0; c < k; ++c) {
      const int dt = kWidth[wi[c]];
      if (ng == 0 || gd[ng - 1] != dt) { gd[ng] = dt; gc[ng] = 0; ++ng; }
      gc[ng - 1] += 1;
    }
    ngroups[bi] = ng;
    if (err_bound) err_bound[bi] = total;
  }
  return bad.load();
}

// Algorithm 1 on caller-supplied factors (U m x r, V n x r, col-major; both
// are copied).  Writes W (m x k), X (n x k), S (k) into buffers sized for
// r columns and returns k.
int hmg_truncate(const double* U, const double* V, int64_t m, int64_t n, int32_t r, double eps,
                 double* W, double* X, double* S) {
  std::vector<double> u(U, U + (size_t)m * r), v(V, V + (size_t)n * r), w, x, s;
  int k = truncate(u, v, m, n, r, eps, w, x, s);
  std::copy(w.begin(), w.end(), W);
  std::copy(x.begin(), x.end(), X);
  std::copy(s.begin(), s.end(), S);
  return k;
}

// Bytes per element of a storage format (for reporting).
int32_t hmg_dtype_bytes(int32_t dt) { return dt_bytes(dt); }

// Exported for the format tests: RNE rounding of doubles to a format.
void hmg_round(const double* x, int64_t cnt, int32_t dt, double* out) {
  for (int64_t i = 0; i < cnt; ++i) out[i] = rnd(x[i], dt);
}

}  // extern "C"
