// libbbp: the blockBP update, imaginary time evolution of a finite PEPS with
// block-BP environments (App. B of Guo, Poletti, Arad; Eq. (Ut)).
//
// One Trotter step applies the gate G = exp(-h dtau) to every nearest-
// neighbour bond, horizontal bonds row by row, then vertical bonds column
// by column, with the context's current messages as the boundary of every
// region.  A gate is fitted by minimising ||psi' - G psi||^2 over the two
// tensors of its bond in the reduced form of the full update: the first
// tensor is split by QR into an isometry on its three outer legs and a
// reduced tensor [k][s][shared], the second by LQ into [shared][s][k'] and
// an isometry; the environment of the two reduced tensors is the two-site
// reduced density matrix of the network in which the two sites carry their
// isometries (the isometry bond as the physical index, the shared leg cut to
// index 0) -- computed on the GPU by a second context that shares the
// lattice, the block partition and the messages; the reduced tensors are
// then fitted by alternating least squares on the host (their systems have
// at most k d D unknowns), and the new tensors replace the old ones.
//
// With the messages fixed, gates in different blocks are independent (the
// blocks run in parallel, Sec. II): the gates are grouped into levels of
// gates whose regions share no block, and each level's environments are
// contracted in one batched call and its fits run on host threads.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bbp.h"
#include "bbp_internal.h"

namespace {

using Mat = std::vector<double>;  // row-major

// Thin Householder QR of an m x n matrix (m >= n or not): Q (m x k), R
// (k x n), k = min(m, n); Q's columns orthonormal, A = Q R.
void qr_thin(const Mat &A, int m, int n, Mat &Q, Mat &R) {
  const int k = std::min(m, n);
  Mat a = A;
  std::vector<Mat> vs;
  std::vector<double> taus;
  for (int j = 0; j < k; ++j) {
    double sigma = 0.0;
    for (int i = j + 1; i < m; ++i) sigma += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    const double alpha = a[(size_t)j * n + j];
    Mat v(m, 0.0);
    double tau = 0.0;
    if (sigma > 0.0) {
      const double nrm = std::sqrt(alpha * alpha + sigma);
      const double beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      v[j] = 1.0;
      for (int i = j + 1; i < m; ++i) v[i] = a[(size_t)i * n + j] * scal;
      // apply H = I - tau v v^T to the columns j..n-1
      for (int c = j; c < n; ++c) {
        double w = 0.0;
        for (int i = j; i < m; ++i) w += v[i] * a[(size_t)i * n + c];
        w *= tau;
        for (int i = j; i < m; ++i) a[(size_t)i * n + c] -= w * v[i];
      }
    }
    vs.push_back(v);
    taus.push_back(tau);
  }
  R.assign((size_t)k * n, 0.0);
  for (int i = 0; i < k; ++i)
    for (int c = i; c < n; ++c) R[(size_t)i * n + c] = a[(size_t)i * n + c];
  // Q = H_0 ... H_{k-1} [I_k; 0]
  Q.assign((size_t)m * k, 0.0);
  for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
  for (int j = k - 1; j >= 0; --j) {
    if (taus[j] == 0.0) continue;
    const Mat &v = vs[j];
    for (int c = 0; c < k; ++c) {
      double w = 0.0;
      for (int i = j; i < m; ++i) w += v[i] * Q[(size_t)i * k + c];
      w *= taus[j];
      for (int i = j; i < m; ++i) Q[(size_t)i * k + c] -= w * v[i];
    }
  }
}

// Singular value decomposition of an m x n matrix by one-sided Jacobi
// rotations of its columns (Hestenes): A = U diag(S) V^T with S descending,
// U m x n, V n x n.
void svd_jacobi(const Mat &A, int m, int n, Mat &U, std::vector<double> &S, Mat &V) {
  Mat a = A;
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int r = 0; r < m; ++r) {
          al += a[(size_t)r * n + p] * a[(size_t)r * n + p];
          be += a[(size_t)r * n + q] * a[(size_t)r * n + q];
          ga += a[(size_t)r * n + p] * a[(size_t)r * n + q];
        }
        if (std::fabs(ga) <= 1e-300 || al == 0.0 || be == 0.0) continue;
        off = std::max(off, std::fabs(ga) / std::sqrt(al * be));
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int r = 0; r < m; ++r) {
          const double x = a[(size_t)r * n + p], y = a[(size_t)r * n + q];
          a[(size_t)r * n + p] = cs * x - sn * y;
          a[(size_t)r * n + q] = sn * x + cs * y;
        }
        for (int r = 0; r < n; ++r) {
          const double x = V[(size_t)r * n + p], y = V[(size_t)r * n + q];
          V[(size_t)r * n + p] = cs * x - sn * y;
          V[(size_t)r * n + q] = sn * x + cs * y;
        }
      }
    if (off < 1e-15) break;
  }
  std::vector<double> nrm(n);
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int r = 0; r < m; ++r) s += a[(size_t)r * n + c] * a[(size_t)r * n + c];
    nrm[c] = std::sqrt(s);
  }
  std::vector<int> order(n);
  for (int c = 0; c < n; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  U.assign((size_t)m * n, 0.0);
  S.assign(n, 0.0);
  Mat Vs((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    const int o = order[c];
    S[c] = nrm[o];
    for (int r = 0; r < m; ++r) U[(size_t)r * n + c] = nrm[o] > 0 ? a[(size_t)r * n + o] / nrm[o] : 0.0;
    for (int r = 0; r < n; ++r) Vs[(size_t)r * n + c] = V[(size_t)r * n + o];
  }
  V.swap(Vs);
}

// Solves M x = y for the normal equations of a fit: M symmetrised, 1e-12
// trace/n added to the diagonal, Gaussian elimination with partial pivoting.
bool solve_normal(Mat M, int n, std::vector<double> &y) {
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += M[(size_t)i * n + i];
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
      M[(size_t)i * n + j] = M[(size_t)j * n + i] = s;
    }
  for (int i = 0; i < n; ++i) M[(size_t)i * n + i] += 1e-12 * tr / n;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)piv * n + c])) piv = r;
    if (M[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)c * n + j], M[(size_t)piv * n + j]);
      std::swap(y[c], y[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = M[(size_t)r * n + c] / M[(size_t)c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) M[(size_t)r * n + j] -= f * M[(size_t)c * n + j];
      y[r] -= f * y[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = y[c];
    for (int j = c + 1; j < n; ++j) s -= M[(size_t)c * n + j] * y[j];
    y[c] = s / M[(size_t)c * n + c];
  }
  return true;
}

// Offset of the site tensor entry leg = (s, u, l, d, r), every virtual leg
// of dimension D (the physical index leg[0] is the slowest).
inline size_t aidx5(int D, const int leg[5]) {
  return ((((size_t)leg[0] * D + leg[1]) * D + leg[2]) * D + leg[3]) * D + leg[4];
}

// The reduced-tensor fit of one gate: R[ka][s][r] L[r][t][kb] (bond D)
// closest to T = G Theta in the metric of the environment
// N[(ka,kb)][(ka',kb')], by alternating least squares started from the
// rank-D truncated SVD of T with the singular values split evenly and each
// singular pair signed so that the largest-magnitude entry of its left
// vector is positive.  Writes
// the relative error of the fit in that metric to *loss.
bool fit_pair(int d, int D, int k, int kb, const double *Nm, const double *Th,
              const double *gate, int n_als, double *Rout, double *Lout, double *loss) {
  auto N = [&](int a, int b, int a2, int b2) {
    return Nm[((size_t)(a * kb + b) * k + a2) * kb + b2];
  };
  const int nT = k * d * d * kb;
  std::vector<double> T(nT, 0.0);
  for (int a = 0; a < k; ++a)
    for (int s2 = 0; s2 < d; ++s2)
      for (int t2 = 0; t2 < d; ++t2)
        for (int b = 0; b < kb; ++b) {
          double v = 0.0;
          for (int s = 0; s < d; ++s)
            for (int t = 0; t < d; ++t)
              v += gate[(size_t)(s2 * d + t2) * d * d + s * d + t] *
                   Th[((a * d + s) * d + t) * kb + b];
          T[((a * d + s2) * d + t2) * kb + b] = v;
        }
  Mat Tm(T.begin(), T.end()), U, V;
  std::vector<double> S;
  const int nc = d * kb, rk = std::min(D, std::min(k * d, nc));
  if (k * d >= nc) {
    svd_jacobi(Tm, k * d, nc, U, S, V);
  } else {
    // more columns than rows: decompose T^T = V S U^T instead
    Mat Tt((size_t)nc * k * d);
    for (int i = 0; i < k * d; ++i)
      for (int j = 0; j < nc; ++j) Tt[(size_t)j * k * d + i] = Tm[(size_t)i * nc + j];
    svd_jacobi(Tt, nc, k * d, V, S, U);
  }
  const int ur = (int)(U.size() / (size_t)(k * d)), vr = (int)(V.size() / (size_t)nc);
  // sign of each singular pair: the largest-magnitude entry of u_r positive
  // (the first one on ties), which fixes the bond gauge of the fitted pair
  for (int r = 0; r < rk; ++r) {
    int im = 0;
    for (int i = 1; i < k * d; ++i)
      if (std::fabs(U[(size_t)i * ur + r]) > std::fabs(U[(size_t)im * ur + r])) im = i;
    if (U[(size_t)im * ur + r] < 0.0) {
      for (int i = 0; i < k * d; ++i) U[(size_t)i * ur + r] = -U[(size_t)i * ur + r];
      for (int j = 0; j < nc; ++j) V[(size_t)j * vr + r] = -V[(size_t)j * vr + r];
    }
  }
  std::vector<double> R((size_t)k * d * D, 0.0), L((size_t)D * nc, 0.0);
  for (int i = 0; i < k * d; ++i)
    for (int r = 0; r < rk; ++r) R[(size_t)i * D + r] = U[(size_t)i * ur + r] * std::sqrt(S[r]);
  for (int r = 0; r < rk; ++r)
    for (int j = 0; j < nc; ++j) L[(size_t)r * nc + j] = std::sqrt(S[r]) * V[(size_t)j * vr + r];
  for (int pass = 0; pass < n_als; ++pass) {
    // R with L fixed: M[(a,s,r),(a',s,q)] = sum L[r,u,b] N[a,b,a',b'] L[q,u,b']
    const int nr = k * d * D;
    Mat Mr((size_t)nr * nr, 0.0);
    std::vector<double> y(nr, 0.0);
    for (int a = 0; a < k; ++a)
      for (int r = 0; r < D; ++r)
        for (int a2 = 0; a2 < k; ++a2)
          for (int q = 0; q < D; ++q) {
            double v = 0.0;
            for (int u = 0; u < d; ++u)
              for (int b = 0; b < kb; ++b)
                for (int b2 = 0; b2 < kb; ++b2)
                  v += L[((size_t)r * d + u) * kb + b] * N(a, b, a2, b2) *
                       L[((size_t)q * d + u) * kb + b2];
            for (int s = 0; s < d; ++s)
              Mr[((size_t)(a * d + s) * D + r) * nr + (a2 * d + s) * D + q] = v;
          }
    for (int a = 0; a < k; ++a)
      for (int s = 0; s < d; ++s)
        for (int r = 0; r < D; ++r) {
          double v = 0.0;
          for (int u = 0; u < d; ++u)
            for (int b = 0; b < kb; ++b)
              for (int a2 = 0; a2 < k; ++a2)
                for (int b2 = 0; b2 < kb; ++b2)
                  v += L[((size_t)r * d + u) * kb + b] * N(a, b, a2, b2) *
                       T[((a2 * d + s) * d + u) * kb + b2];
          y[(a * d + s) * D + r] = v;
        }
    if (!solve_normal(Mr, nr, y)) return false;
    R.assign(y.begin(), y.end());
    // L with R fixed: M[(r,u,b),(q,u,b')] = sum R[a,s,r] N[a,b,a',b'] R[a',s,q]
    const int nl = D * d * kb;
    Mat Ml((size_t)nl * nl, 0.0);
    std::vector<double> z(nl, 0.0);
    for (int r = 0; r < D; ++r)
      for (int b = 0; b < kb; ++b)
        for (int q = 0; q < D; ++q)
          for (int b2 = 0; b2 < kb; ++b2) {
            double v = 0.0;
            for (int a = 0; a < k; ++a)
              for (int s = 0; s < d; ++s)
                for (int a2 = 0; a2 < k; ++a2)
                  v += R[((size_t)a * d + s) * D + r] * N(a, b, a2, b2) *
                       R[((size_t)a2 * d + s) * D + q];
            for (int u = 0; u < d; ++u)
              Ml[((size_t)(r * d + u) * kb + b) * nl + (q * d + u) * kb + b2] = v;
          }
    for (int r = 0; r < D; ++r)
      for (int u = 0; u < d; ++u)
        for (int b = 0; b < kb; ++b) {
          double v = 0.0;
          for (int a = 0; a < k; ++a)
            for (int s = 0; s < d; ++s)
              for (int a2 = 0; a2 < k; ++a2)
                for (int b2 = 0; b2 < kb; ++b2)
                  v += R[((size_t)a * d + s) * D + r] * N(a, b, a2, b2) *
                       T[((a2 * d + s) * d + u) * kb + b2];
          z[(r * d + u) * kb + b] = v;
        }
    if (!solve_normal(Ml, nl, z)) return false;
    L.assign(z.begin(), z.end());
  }
  double num = 0.0, den = 0.0;
  std::vector<double> diff(nT);
  for (int a = 0; a < k; ++a)
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t)
        for (int b = 0; b < kb; ++b) {
          double v = 0.0;
          for (int r = 0; r < D; ++r)
            v += R[((size_t)a * d + s) * D + r] * L[((size_t)r * d + t) * kb + b];
          diff[((a * d + s) * d + t) * kb + b] = v - T[((a * d + s) * d + t) * kb + b];
        }
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < kb; ++b)
      for (int a2 = 0; a2 < k; ++a2)
        for (int b2 = 0; b2 < kb; ++b2) {
          const double n4 = N(a, b, a2, b2);
          for (int s = 0; s < d; ++s)
            for (int t = 0; t < d; ++t) {
              num += diff[((a * d + s) * d + t) * kb + b] * n4 *
                     diff[((a2 * d + s) * d + t) * kb + b2];
              den += T[((a * d + s) * d + t) * kb + b] * n4 * T[((a2 * d + s) * d + t) * kb + b2];
            }
        }
  *loss = den > 0.0 ? num / den : 0.0;
  for (double v : R)
    if (!std::isfinite(v)) return false;
  for (double v : L)
    if (!std::isfinite(v)) return false;
  std::copy(R.begin(), R.end(), Rout);
  std::copy(L.begin(), L.end(), Lout);
  return true;
}

// One gate of a Trotter step and its work: the bond (x0, y0, x1, y1), the
// first site the left or upper one; the reduced tensors of its two sites.
struct Gate {
  std::array<int, 4> b;
  int level = 0;
  int ia = 0, ib = 0, sa = 0, sb = 0, oa[3] = {}, ob[3] = {};
  int da[5] = {}, db[5] = {};  // true leg extents (s, u, l, d, r)
  int rows_a = 0, cols_b = 0, k = 0, kb = 0;
  Mat Xa, Ra, Qt, Rt;  // Ma = Xa Ra; Mb^T = Qt Rt
};

// f(0..n-1) on up to `threads` host threads.
template <class F>
void parallel_for(int n, int threads, F f) {
  threads = std::min(threads, n);
  if (threads <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (int i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto &th : pool) th.join();
}

// Row of a site entry among the rows formed by three legs o (true extents n).
inline size_t row_of(const int leg[5], const int o[3], const int n[5]) {
  return ((size_t)leg[o[0]] * n[o[1]] + leg[o[1]]) * n[o[2]] + leg[o[2]];
}

// True extents of the legs of site (x, y): 1 on the lattice edge, so that
// the isometries span physical directions only.
void leg_dims(int x, int y, int d, int D, int Lx, int Ly, int n[5]) {
  n[0] = d;
  n[1] = y == 0 ? 1 : D;
  n[2] = x == 0 ? 1 : D;
  n[3] = y == Ly - 1 ? 1 : D;
  n[4] = x == Lx - 1 ? 1 : D;
}

// QR of the first site over its outer legs, LQ of the second (App. B's
// reduced tensors): Ma[(outer), (s, shared)] = Xa Ra and
// Mb[(shared, s), (outer)] = Rt^T Qt^T.
void split_gate(Gate &g, const double *A, int d, int D, int Lx, int Ly) {
  const size_t ss = (size_t)d * D * D * D * D;
  const bool horiz = g.b[1] == g.b[3];
  g.ia = g.b[1] * Lx + g.b[0];
  g.ib = g.b[3] * Lx + g.b[2];
  g.sa = horiz ? 4 : 3;  // shared leg of each site (0 = s)
  g.sb = horiz ? 2 : 1;
  for (int t = 1, u = 0, w = 0; t <= 4; ++t) {
    if (t != g.sa) g.oa[u++] = t;
    if (t != g.sb) g.ob[w++] = t;
  }
  leg_dims(g.b[0], g.b[1], d, D, Lx, Ly, g.da);
  leg_dims(g.b[2], g.b[3], d, D, Lx, Ly, g.db);
  g.rows_a = g.da[g.oa[0]] * g.da[g.oa[1]] * g.da[g.oa[2]];
  g.cols_b = g.db[g.ob[0]] * g.db[g.ob[1]] * g.db[g.ob[2]];
  const double *Aa = A + g.ia * ss, *Ab = A + g.ib * ss;
  Mat Ma((size_t)g.rows_a * d * D, 0.0), MbT((size_t)g.cols_b * D * d, 0.0);
  int leg[5];
  for (leg[0] = 0; leg[0] < d; ++leg[0])
    for (leg[1] = 0; leg[1] < D; ++leg[1])
      for (leg[2] = 0; leg[2] < D; ++leg[2])
        for (leg[3] = 0; leg[3] < D; ++leg[3])
          for (leg[4] = 0; leg[4] < D; ++leg[4]) {
            const size_t src = aidx5(D, leg);
            if (leg[1] < g.da[1] && leg[2] < g.da[2] && leg[3] < g.da[3] && leg[4] < g.da[4])
              Ma[row_of(leg, g.oa, g.da) * d * D + (size_t)leg[0] * D + leg[g.sa]] = Aa[src];
            if (leg[1] < g.db[1] && leg[2] < g.db[2] && leg[3] < g.db[3] && leg[4] < g.db[4])
              MbT[row_of(leg, g.ob, g.db) * D * d + (size_t)leg[g.sb] * d + leg[0]] = Ab[src];
          }
  qr_thin(Ma, g.rows_a, d * D, g.Xa, g.Ra);
  qr_thin(MbT, g.cols_b, D * d, g.Qt, g.Rt);
  g.k = std::min(g.rows_a, d * D);
  g.kb = std::min(g.cols_b, D * d);
}

// The gate's two sites in the environment network (site stride sp): the
// isometry columns as the physical index, the shared leg at index 0.
void place_isometries(const Gate &g, double *M, size_t sp, int D) {
  const size_t D4 = (size_t)D * D * D * D;
  std::fill(M + g.ia * sp, M + (g.ia + 1) * sp, 0.0);
  std::fill(M + g.ib * sp, M + (g.ib + 1) * sp, 0.0);
  for (int q = 0; q < g.k; ++q)
    for (int r = 0; r < g.rows_a; ++r) {
      int lg[5] = {0, 0, 0, 0, 0};
      lg[g.oa[0]] = r / (g.da[g.oa[1]] * g.da[g.oa[2]]);
      lg[g.oa[1]] = r / g.da[g.oa[2]] % g.da[g.oa[1]];
      lg[g.oa[2]] = r % g.da[g.oa[2]];
      M[g.ia * sp + (size_t)q * D4 + aidx5(D, lg)] = g.Xa[(size_t)r * g.k + q];
    }
  for (int q = 0; q < g.kb; ++q)
    for (int cc = 0; cc < g.cols_b; ++cc) {
      int lg[5] = {0, 0, 0, 0, 0};
      lg[g.ob[0]] = cc / (g.db[g.ob[1]] * g.db[g.ob[2]]);
      lg[g.ob[1]] = cc / g.db[g.ob[2]] % g.db[g.ob[1]];
      lg[g.ob[2]] = cc % g.db[g.ob[2]];
      M[g.ib * sp + (size_t)q * D4 + aidx5(D, lg)] = g.Qt[(size_t)cc * g.kb + q];
    }
}

// Fit of one gate from its environment rho (the two-site RDM of the
// isometry network, dp^4 doubles), then the new tensors A_a = Xa R and
// A_b = L Qt^T written into A, each scaled to a largest entry of 1.
bool fit_gate(const Gate &g, const double *rho, int dp, const double *gate, int n_als, int d,
              int D, double *A, double *loss) {
  const int k = g.k, kb = g.kb;
  const size_t ss = (size_t)d * D * D * D * D;
  std::vector<double> Nm((size_t)k * kb * k * kb);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < kb; ++b)
      for (int a2 = 0; a2 < k; ++a2)
        for (int b2 = 0; b2 < kb; ++b2)
          Nm[((size_t)(a * kb + b) * k + a2) * kb + b2] =
              rho[((size_t)a * dp + b) * dp * dp + (size_t)a2 * dp + b2];
  // Theta[ka][s][t][kb] = sum_r Ra[ka][(s, r)] Lb[(r, t)][kb], Lb = Rt^T
  std::vector<double> Th((size_t)k * d * d * kb, 0.0);
  for (int a = 0; a < k; ++a)
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t)
        for (int b = 0; b < kb; ++b) {
          double v = 0.0;
          for (int r = 0; r < D; ++r)
            v += g.Ra[(size_t)a * d * D + s * D + r] * g.Rt[(size_t)b * D * d + r * d + t];
          Th[((a * d + s) * d + t) * kb + b] = v;
        }
  std::vector<double> R((size_t)k * d * D), L((size_t)D * d * kb);
  if (!fit_pair(d, D, k, kb, Nm.data(), Th.data(), gate, n_als, R.data(), L.data(), loss))
    return false;
  std::vector<double> na(ss, 0.0), nb(ss, 0.0);
  int leg[5];
  for (leg[0] = 0; leg[0] < d; ++leg[0])
    for (leg[1] = 0; leg[1] < D; ++leg[1])
      for (leg[2] = 0; leg[2] < D; ++leg[2])
        for (leg[3] = 0; leg[3] < D; ++leg[3])
          for (leg[4] = 0; leg[4] < D; ++leg[4]) {
            const size_t dst = aidx5(D, leg);
            if (leg[1] < g.da[1] && leg[2] < g.da[2] && leg[3] < g.da[3] && leg[4] < g.da[4]) {
              const size_t ra = row_of(leg, g.oa, g.da);
              double v = 0.0;
              for (int q = 0; q < k; ++q)
                v += g.Xa[ra * k + q] * R[((size_t)q * d + leg[0]) * D + leg[g.sa]];
              na[dst] = v;
            }
            if (leg[1] < g.db[1] && leg[2] < g.db[2] && leg[3] < g.db[3] && leg[4] < g.db[4]) {
              const size_t cb = row_of(leg, g.ob, g.db);
              double w = 0.0;
              for (int q = 0; q < kb; ++q)
                w += L[((size_t)leg[g.sb] * d + leg[0]) * kb + q] * g.Qt[cb * kb + q];
              nb[dst] = w;
            }
          }
  double ma = 0.0, mb = 0.0;
  for (size_t i = 0; i < ss; ++i) {
    ma = std::max(ma, std::fabs(na[i]));
    mb = std::max(mb, std::fabs(nb[i]));
  }
  if (!(ma > 0.0) || !(mb > 0.0) || !std::isfinite(ma) || !std::isfinite(mb)) return false;
  for (size_t i = 0; i < ss; ++i) {
    A[g.ia * ss + i] = na[i] / ma;
    A[g.ib * ss + i] = nb[i] / mb;
  }
  return true;
}

}  // namespace

extern "C" bbp_status bbp_ite_step(bbp_ctx *c, const double *gate, int32_t n_als,
                                   double *info) {
  if (!c) return BBP_EINVAL;
  bbp::CtxInfo ci;
  bbp_status st = bbp::ctx_info(c, &ci);
  if (st != BBP_OK) return st;
  if (!gate || n_als < 1 || n_als > 64)
    return bbp::ctx_fail(c, BBP_EINVAL, "gate needed and n_als in [1, 64]");
  if (ci.infinite || ci.single_layer)
    return bbp::ctx_fail(c, BBP_EINVAL, "the update is for finite double-layer lattices");
  const int d = ci.d, D = ci.D, Lx = ci.Lx, Ly = ci.Ly;
  for (int i = 0; i < d * d * d * d; ++i)
    if (!std::isfinite(gate[i])) return bbp::ctx_fail(c, BBP_EINVAL, "non-finite gate");
  size_t nA = 0;
  const double *A0 = bbp::ctx_tensors(c, &nA);
  std::vector<double> A(A0, A0 + nA);
  const size_t ss = (size_t)d * D * D * D * D, D3 = (size_t)D * D * D;
  // physical dimension of the environment network: the widest isometry bond
  const int dp = std::max(d, (int)std::min<size_t>(D3, (size_t)d * D));
  if (dp > 8)
    return bbp::ctx_fail(c, BBP_EINVAL, "the update needs min(D^3, d D) <= 8 (the environment's "
                                        "physical dimension)");
  if (Lx < 2 && Ly < 2) return bbp::ctx_fail(c, BBP_EINVAL, "a lattice without bonds");
  // the messages every region's boundary is built from, kept through the step
  size_t need = 0;
  if ((st = bbp_get_messages(c, nullptr, 0, &need)) != BBP_OK) return st;
  std::vector<double> msgs(need);
  if ((st = bbp_get_messages(c, msgs.data(), need, &need)) != BBP_OK) return st;
  // the environment context: the same lattice, partition, bond caps and fit
  // settings, physical dimension dp (the isometry bond of the two sites)
  bbp_ctx *e = nullptr;
  if ((st = bbp_create(&e, 0, Lx, Ly, 0, 0, ci.bx, ci.by, D, ci.chi)) != BBP_OK)
    return bbp::ctx_fail(c, st, "environment context");
  struct Free {
    bbp_ctx *e;
    ~Free() { bbp_destroy(e); }
  } free_e{e};
  const std::pair<const char *, double> opts[] = {
      {"d", (double)dp}, {"chi_env", (double)ci.chi_env}, {"n_fit", (double)ci.n_fit},
      {"seed", (double)ci.seed}, {"shift_x", (double)ci.sx}, {"shift_y", (double)ci.sy}};
  for (auto &o : opts)
    if ((st = bbp_set_option(e, o.first, o.second)) != BBP_OK)
      return bbp::ctx_fail(c, st, std::string("environment option ") + o.first + ": " +
                                      bbp_last_error(e));
  (void)bbp_set_stream(e, ci.stream);
  // device memory as the caller's context obtains it: its allocator, and a
  // budget of its own equal to the context's
  if (ci.alloc_fn &&
      (st = bbp_set_allocator(e, ci.alloc_fn, ci.free_fn, ci.alloc_user)) != BBP_OK)
    return bbp::ctx_fail(c, st, std::string("environment allocator: ") + bbp_last_error(e));
  if (ci.hbm_budget &&
      (st = bbp_set_option(e, "hbm_budget", (double)ci.hbm_budget)) != BBP_OK)
    return bbp::ctx_fail(c, st, std::string("environment budget: ") + bbp_last_error(e));
  // gate order: horizontal bonds row by row, then vertical bonds column by column
  std::vector<Gate> gl;
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x + 1 < Lx; ++x) gl.push_back(Gate{{x, y, x + 1, y}});
  for (int x = 0; x < Lx; ++x)
    for (int y = 0; y + 1 < Ly; ++y) gl.push_back(Gate{{x, y, x, y + 1}});
  // Schedule.  With the messages fixed, a gate's result depends on the
  // tensors of its region only: the block of its bond, or the two blocks a
  // bond between blocks joins.  Two gates whose regions share no block
  // therefore commute, and the gates are grouped into levels: a gate's level
  // is one more than the last level that touched any block of its region.
  // Running the levels in order, each level's gates together, gives the
  // result of the sequential order gate for gate.
  const int gx = (Lx + ci.sx + ci.bx - 1) / ci.bx, gy = (Ly + ci.sy + ci.by - 1) / ci.by;
  std::vector<int> last((size_t)gx * gy, -1);
  int n_levels = 0;
  for (Gate &g : gl) {
    const int b0 = ((g.b[1] + ci.sy) / ci.by) * gx + (g.b[0] + ci.sx) / ci.bx;
    const int b1 = ((g.b[3] + ci.sy) / ci.by) * gx + (g.b[2] + ci.sx) / ci.bx;
    g.level = std::max(last[b0], last[b1]) + 1;
    last[b0] = last[b1] = g.level;
    n_levels = std::max(n_levels, g.level + 1);
  }
  std::vector<std::vector<int>> levels(n_levels);
  for (size_t q = 0; q < gl.size(); ++q) levels[gl[q].level].push_back((int)q);
  std::vector<double> M((size_t)Lx * Ly * dp * D * D * D * D);
  const size_t sp = (size_t)dp * D * D * D * D;
  const int nthreads =
      (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  double loss_sum = 0.0, t_env = 0.0, t_host = 0.0;
  int gates = 0;
  using clk = std::chrono::steady_clock;
  auto secs = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  // the environment network, padded to dp (every site's current tensor)
  for (int i = 0; i < Lx * Ly; ++i)
    std::copy(A.begin() + i * ss, A.begin() + (i + 1) * ss, M.begin() + i * sp);
  std::vector<int> prev_sites;  // the previous level's gate sites
  bool env_ready = false;
  for (const std::vector<int> &lv : levels) {
    const auto t0 = clk::now();
    // 1. reduced tensors of every gate of the level (their sites differ)
    parallel_for((int)lv.size(), nthreads,
                 [&](int q) { split_gate(gl[lv[q]], A.data(), d, D, Lx, Ly); });
    // 2. the environment network: current tensors padded to dp, each gate's
    // two sites carrying its isometries.  The environment context holds the
    // network of the previous level; only the sites that differ are replaced
    // (the previous level's sites, now with their new tensors, and this
    // level's), so that boundary stacks over unchanged rows or columns are
    // reused.
    std::vector<int> changed(prev_sites);
    prev_sites.clear();
    for (int q : lv) {
      prev_sites.push_back(gl[q].ia);
      prev_sites.push_back(gl[q].ib);
    }
    changed.insert(changed.end(), prev_sites.begin(), prev_sites.end());
    for (int i : changed) {
      std::fill(M.begin() + i * sp, M.begin() + (i + 1) * sp, 0.0);
      std::copy(A.begin() + i * ss, A.begin() + (i + 1) * ss, M.begin() + i * sp);
    }
    for (int q : lv) place_isometries(gl[q], M.data(), sp, D);
    std::vector<double> sites_buf(changed.size() * sp);
    for (size_t q = 0; q < changed.size(); ++q)
      std::copy(M.begin() + changed[q] * sp, M.begin() + (changed[q] + 1) * sp,
                sites_buf.begin() + q * sp);
    const auto t1 = clk::now();
    if (!env_ready) {
      if ((st = bbp_set_tensors(e, M.data(), M.size())) != BBP_OK ||
          (!msgs.empty() && (st = bbp_set_messages(e, msgs.data(), msgs.size())) != BBP_OK))
        return bbp::ctx_fail(c, st, std::string("environment: ") + bbp_last_error(e));
      bbp::ctx_keep_stacks(e);
      env_ready = true;
    } else if ((st = bbp::ctx_replace_sites(e, (int)changed.size(), changed.data(),
                                            sites_buf.data())) != BBP_OK) {
      return bbp::ctx_fail(c, st, std::string("environment: ") + bbp_last_error(e));
    }
    const int n = (int)lv.size();
    std::vector<int32_t> x0(n), y0(n), x1(n), y1(n);
    for (int q = 0; q < n; ++q) {
      x0[q] = gl[lv[q]].b[0];
      y0[q] = gl[lv[q]].b[1];
      x1[q] = gl[lv[q]].b[2];
      y1[q] = gl[lv[q]].b[3];
    }
    std::vector<double> rho((size_t)n * dp * dp * dp * dp);
    if ((st = bbp::rdm_bonds_only(e, n, x0.data(), y0.data(), x1.data(), y1.data(),
                                  rho.data())) != BBP_OK)
      return bbp::ctx_fail(c, st, std::string("environment: ") + bbp_last_error(e));
    // 3. fits and new tensors, every gate of the level at once
    const auto t2 = clk::now();
    std::vector<int> ok(n, 1);
    std::vector<double> loss(n, 0.0);
    parallel_for(n, nthreads, [&](int q) {
      ok[q] = fit_gate(gl[lv[q]], rho.data() + (size_t)q * dp * dp * dp * dp, dp, gate, n_als,
                       d, D, A.data(), &loss[q]);
    });
    for (int q = 0; q < n; ++q) {
      if (!ok[q])
        return bbp::ctx_fail(c, BBP_ENUMERIC,
                             "singular reduced-tensor fit or vanishing fitted tensor");
      loss_sum += loss[q];
      ++gates;
    }
    t_host += secs(t0, t1) + secs(t2, clk::now());
    t_env += secs(t1, t2);
  }
  // the new tensors, with the messages the step started from
  if ((st = bbp_set_tensors(c, A.data(), A.size())) != BBP_OK) return st;
  if (!msgs.empty() && (st = bbp_set_messages(c, msgs.data(), msgs.size())) != BBP_OK)
    return st;
  if (info) {
    info[0] = gates;
    info[1] = loss_sum;
    info[2] = t_env;
    info[3] = t_host;
    info[4] = n_levels;
  }
  return BBP_OK;
}

extern "C" bbp_status bbp_ite_fit(int32_t d, int32_t D, int32_t k, int32_t kb, const double *N,
                                  const double *theta, const double *gate, int32_t n_als,
                                  double *R, double *L, double *loss) {
  if (d < 1 || d > 8 || D < 1 || D > 8 || k < 1 || k > 64 || kb < 1 || kb > 64 || n_als < 1 ||
      n_als > 64 || !N || !theta || !gate || !R || !L)
    return BBP_EINVAL;
  const size_t nn = (size_t)k * kb * k * kb, nt = (size_t)k * d * d * kb;
  for (size_t i = 0; i < nn; ++i)
    if (!std::isfinite(N[i])) return BBP_EINVAL;
  for (size_t i = 0; i < nt; ++i)
    if (!std::isfinite(theta[i])) return BBP_EINVAL;
  for (int i = 0; i < d * d * d * d; ++i)
    if (!std::isfinite(gate[i])) return BBP_EINVAL;
  double l = 0.0;
  if (!fit_pair(d, D, k, kb, N, theta, gate, n_als, R, L, &l)) return BBP_ENUMERIC;
  if (loss) *loss = l;
  return BBP_OK;
}
