// Sum-factorised FP64 stage: the volume term, surface term, inverse mass and
// LSRK update evaluated through the collapsed tensor structure of the
// semi-nodal basis (the cheaper evaluation of volume integrals proposed in
// Section 4.4),
//   phi_ijk(a, b, c) = l^k_i(a) l^k_j(b) g_k(c),  g_k = h^k P^{(2k+3,0)}_{N-k}(c),
// h = (1-c)/2, on the tensor cubature (a_p, b_m, c_r) of Section 4.1.  Every
// contraction is a product with a one-dimensional factor, so a stage costs
// O(N^4) per element instead of the O(N^6) of the dense operators; results
// equal the dense contractions up to rounding order.
//
// Derivatives in the reference coordinates (r, s, t) of one field u:
//   d_r u = sum_k Gt_k(c) sum_j l_j(b) sum_i l'_i(a) u_ijk,
//   d_s u = sum_k Gt_k(c) sum_j l'_j(b) sum_i l_i(a) u_ijk,
//   d_t u = sum_k g'_k(c) sum_j l_j(b) sum_i l_i(a) u_ijk
//           + (1+a)/2 d_r u + (1+b)/2 d_s u,
// with Gt_k = h^(k-1) P_{N-k} (the factor 2/(1-c) of the collapsed
// derivatives absorbed).  The metric J dR/dx depends on (a, b) only (Lemma 1
// generalised), so it is evaluated once per (a, b) column.
//
// Faces.  A trace is kept as two numbers per face point, the pressure and the
// normal velocity u . n with the element's own outward unit normal n: the
// penalty flux (Section 4.3) needs only the jumps [[p]] and n . [[u]], and on a
// conforming face the neighbour's outward normal is -n.  The pyramids of one
// hexahedron pair their four triangle faces among themselves; when the mesh
// comes in such groups a workgroup owns whole hexahedra and exchanges the
// triangle traces in LDS, and only the quadrilateral base traces go through
// HBM (written by k_sf_trace).  Otherwise (general meshes, and N >= 6 where
// six elements do not fit four waves) k_sf_trace_all writes the (p, u.n)
// pairs of all five faces, [K][Nfc][2], and the stage reads its neighbours'
// from HBM.
//
// Work shape.  A workgroup owns E elements (at most 256 columns) and one
// thread per (element, a, b) column.  The four fields are processed one at a
// time through LDS, the velocities first: the a-direction contraction at the
// a-points and at a = -1, +1 (all threads), then per column the b- and
// c-direction contractions, the FP64 metric and the projection onto the c
// factors, accumulated in registers across the fields, and beside them the
// triangle traces as b- and c-contractions of the a-direction results; the
// next field's coefficients are loaded while the current one is contracted.
// After the face fluxes (folded along c, then summed once per row into the
// triangle lift sums) the projection is finished field by field
// (b-direction, then a-direction with the triangle lifts, inverse mass and
// the LSRK stage, the RK state loaded ahead).  LDS stays under 60 KiB per
// workgroup and no kernel keeps arrays in private memory; setup checks LDS,
// private memory and block size (hipFuncGetAttributes against the device's
// limits) before the first launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"

namespace dgpyr {
namespace {

constexpr int kLdsBudget = 60 * 1024;  // bytes of LDS a workgroup may use
// Private memory a work item may reserve: the compiler keeps a small frame of
// up to 68 bytes per lane for some of these kernels that no instruction
// touches (the register scavenger's reserve); anything larger would mean
// arrays spilled to private memory.
constexpr size_t kPrivateBudget = 256;

__device__ __host__ constexpr int round64(int x) { return (x + 63) / 64 * 64; }

// Sizes of the sum-factorised stage at degree N.
template <int N>
struct SfDims {
  static constexpr int n1 = N + 1;
  static constexpr int n2 = n1 * n1;
  static constexpr int n3 = n2 * n1;
  static constexpr int Np = n1 * (n1 + 1) * (2 * n1 + 1) / 6;
  static constexpr int KJ = n1 * (n1 + 1) / 2;  // pairs (k, j <= k)
  static constexpr int Nfc = 5 * n2;
  // per-element LDS regions (doubles):
  static constexpr int UD = KJ * n1;      // U of one field, then D [kj][p]
  // A, A' [2][kj][p] and the a = -1, +1 values Ae [kj][2]; then B [k][m][p]
  // (n3 <= AB)
  static constexpr int AB = 2 * KJ * n1 + 2 * KJ;
  static constexpr int TT = 8 * n2;       // triangle traces [face][p, u.n][point]
  // folded triangle fluxes [face][2][k][p] overwrite the traces when every
  // thread owns at most one (element, face, a) item (4 n1 <= n2), else they
  // need a region of their own
  static constexpr bool kSeparateC = 4 * n1 > n2;
  static constexpr int CC = kSeparateC ? 8 * n2 : 0;
  // vertices, normals, rho c, material, Jacobian coefficients, ints
  static constexpr int kTables = 16 + 16 + 5 + 4 + 4 + 10;
  static constexpr int PER_ELEM = kTables + UD + AB + TT + CC;
  // permutations, padded positions, index tables
  static constexpr int PERM_BYTES = 10 * n2 * 4 + 2 * Np * 4 + KJ * 4;
  // one-dimensional factors read with lane-dependent indices, staged in LDS
  // once per workgroup: l^k_i(x_p), d/da l^k_i(x_p) [k][p][i], l^k_i(-1, +1)
  // [k][s][i]
  static constexpr int TAB = 2 * n3 + 2 * n2;
  static constexpr int bytes(int E) { return E * PER_ELEM * 8 + PERM_BYTES + TAB * 8; }
  // Elements per workgroup: at most 256 columns (four waves), so that
  // several workgroups share a CU at the two or three waves per SIMD these
  // kernels' registers allow.  Measured at 64^3 x 6: one hexahedron per
  // workgroup instead of two halves the stage at N = 3 and 4 (8.55 -> 4.28
  // ms, 16.4 -> 9.3 ms); at N = 6, where one hexahedron needs five waves and
  // only one such workgroup fits a CU, the general variant with 5 elements
  // per workgroup is faster despite its all-face traces (stage 46.9 -> 35.0
  // ms, trace 7.3 -> 9.3 ms).
  // Whole hexahedra (6 elements each), 0 if not even one fits:
  static constexpr int hex_elems() {
    int best = 0;
    for (int H = 1; 6 * H * n2 <= 256 && bytes(6 * H) <= kLdsBudget; ++H) best = 6 * H;
    return best;
  }
  static constexpr int free_elems() {
    int best = 1;
    // (N = 7: two elements, two waves, four workgroups per CU: 51.0 -> 49.6
    // ms against four elements at 64^3 x 6)
    for (int E = 1; E * n2 <= (N == 7 ? 128 : 256) && bytes(E) <= kLdsBudget; ++E) best = E;
    return best;
  }
};

template <int N, bool LOCAL>
struct SfShape {
  using D = SfDims<N>;
  static constexpr int E = LOCAL ? D::hex_elems() : D::free_elems();
  static constexpr int THREADS = round64(E * D::n2);
};

__device__ __forceinline__ int kofs(int k) { return k * (k + 1) * (2 * k + 1) / 6; }
__device__ __forceinline__ int kjofs(int k) { return k * (k + 1) / 2; }

// (k, j) of a pair index kj = k (k+1)/2 + j, 0 <= kj < (N+1)(N+2)/2, by N
// comparisons (no lane-divergent loop).
template <int N>
__device__ __forceinline__ void kj_split(int kj, int& k, int& j) {
  k = 0;
#pragma unroll
  for (int t = 1; t <= N; ++t) k += kj >= kjofs(t) ? 1 : 0;
  j = kj - kjofs(k);
}

// (k, j, i) of a coefficient index n = kofs(k) + j (k+1) + i, 0 <= n < Np,
// by comparisons only.
template <int N>
__device__ __forceinline__ void kji_split(int n, int& k, int& j, int& i) {
  k = 0;
#pragma unroll
  for (int t = 1; t <= N; ++t) k += n >= kofs(t) ? 1 : 0;
  const int rem = n - kofs(k);
  j = 0;
#pragma unroll
  for (int t = 1; t <= N; ++t) j += rem >= t * (k + 1) ? 1 : 0;
  i = rem - j * (k + 1);
}

// Penalty flux from the jumps at one face point (Section 4.3):
//   Fp = w (n.[[u]] - tau_p [[p]]) / 2,  Pu = w ([[p]] - tau_u n.[[u]]) / 2,
// the velocity rows' flux being n Pu; w = face weight x surface Jacobian.
__device__ __forceinline__ void jump_flux(double jp, double jun, double zm, double zp,
                                          double alpha, double w, double& Fp, double& Pu) {
  const double zavg = 0.5 * (zm + zp);
  const double taup = alpha / zavg, tauu = alpha * zavg;
  Fp = 0.5 * w * (jun - taup * jp);
  Pu = 0.5 * w * (jp - tauu * jun);
}

// Exterior values (p+, n.u+) at a face point from the neighbour's stored
// (p, u.n') with n' = -n, or the mirror state of the boundary condition.
__device__ __forceinline__ void exterior(bool inner, double nbp, double nbun, double pm, double unm,
                                         int bc, double& pp, double& unp) {
  if (inner) {
    pp = nbp;
    unp = -nbun;
  } else if (bc == DGPYR_BC_WALL) {  // p+ = p-, u+ = u- - 2 (n.u-) n
    pp = pm;
    unp = -unm;
  } else {  // free surface: p+ = -p-, u+ = u-
    pp = -pm;
    unp = unm;
  }
}

// ---------------------------------------------------------------------------
// Base traces (p, u.n) of every element, T2[K][n2][2] (NF = 1), one thread per
// face point; the state of the workgroup's elements and the one-dimensional
// factors are staged in LDS.
template <int N, int NF>
struct TraceShape {
  using D = SfDims<N>;
  static constexpr int PTS = NF * D::n2;  // points per element
  static constexpr int E = 256 / PTS < 1 ? 1 : (256 / PTS > 64 ? 64 : 256 / PTS);
  static constexpr int THREADS = round64(E * PTS);
};

// Stages the one-dimensional factors of the basis into LDS (La, Da [k][p][i],
// Le [k][s][i]).
template <int N>
__device__ __forceinline__ void stage_tables(const SfOps& sf, double* sLa, double* sDa, double* sLe,
                                             int tid, int nt) {
  constexpr int n1 = N + 1, n3 = n1 * n1 * n1;
  for (int x = tid; x < n3; x += nt) {
    sLa[x] = sf.La[x];
    sDa[x] = sf.Da[x];
  }
  for (int x = tid; x < 2 * n1 * n1; x += nt) sLe[x] = sf.Le[x];
}

// Value of field u (coefficients of one element) at point pt = p + n1 m of
// face f: base (f = 0) at (a_p, b_m, -1); a = -1, +1 (f = 1, 2) at
// (b_p, c_m); b = -1, +1 (f = 3, 4) at (a_p, c_m) (c_m the Gauss-Jacobi(1,0)
// nodes).
template <int N>
__device__ __forceinline__ double face_value(const double* u, int f, int p, int m, const SfOps& sf,
                                             const double* sLa, const double* sLe) {
  constexpr int n1 = N + 1;
  double val = 0.0;
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    const double* uk = u + kofs(k);
    const double* La_p = sLa + (k * n1 + p) * n1;
    double Y = 0.0;
    if (f == 0) {
      const double* La_m = sLa + (k * n1 + m) * n1;
      // rows j one at a time: unrolled, the compiler loads all coefficients
      // ahead and needs more registers than the kernel has
#pragma unroll 1
      for (int j = 0; j <= k; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) acc += La_p[i] * uk[j * (k + 1) + i];
        Y += La_m[j] * acc;
      }
      val += sf.Gb[k] * Y;
    } else {
      const double* Le_s = sLe + (k * 2 + ((f == 2 || f == 4) ? 1 : 0)) * n1;
      const bool afc = f <= 2;  // a = -1/+1: the a-factor at the face, b at the edge point
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) acc += (afc ? Le_s[i] : La_p[i]) * uk[j * (k + 1) + i];
        Y += (afc ? La_p[j] : Le_s[j]) * acc;
      }
      val += sf.Gf[m * n1 + k] * Y;
    }
  }
  return val;
}

// Four waves per SIMD (at most 128 registers, no spills up to N = 5): the
// kernel waits on memory most of its time, and the compiler's own choice
// (138 registers at N = 5) leaves three (2.65 -> 2.61 ms at 64^3 x 6, N = 5;
// five waves spill and take 3.73 ms).
template <int N, int NF>
__global__ __launch_bounds__((TraceShape<N, NF>::THREADS), 4) void k_sf_trace(
    const double* __restrict__ U, double* __restrict__ T2, SfOps sf, DevOps ops,
    const double* __restrict__ verts, int64_t K) {
  using D = SfDims<N>;
  using TS = TraceShape<N, NF>;
  constexpr int n1 = D::n1, n2 = D::n2, Np = D::Np, E = TS::E, NT = TS::THREADS, PTS = TS::PTS;
  __shared__ double sU[E][4 * Np];
  __shared__ double sX[E][16];
  __shared__ double sLa[D::n3], sLe[2 * n2];
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)(K - e0 < E ? K - e0 : E);
  // The workgroup's state: every load of a thread issued before the first
  // store (a compile-time count), so the loads overlap instead of each
  // waiting out a memory round trip; the tables load meanwhile.
  constexpr int ST = (E * 4 * Np + NT - 1) / NT;
  const int nU = ne * 4 * Np;
  const double* Ug = U + e0 * 4 * Np;
  double ru[ST];
#pragma unroll
  for (int it = 0; it < ST; ++it) {
    const int x = tid + it * NT;
    ru[it] = x < nU ? Ug[x] : 0.0;
  }
  for (int x = tid; x < ne * 16; x += NT) sX[x / 16][x % 16] = verts[e0 * 16 + x];
  for (int x = tid; x < D::n3; x += NT) sLa[x] = sf.La[x];
  for (int x = tid; x < 2 * n2; x += NT) sLe[x] = sf.Le[x];
  double* sUf = &sU[0][0];
#pragma unroll
  for (int it = 0; it < ST; ++it) {
    const int x = tid + it * NT;
    if (x < nU) sUf[x] = ru[it];
  }
  __syncthreads();
  for (int x = tid; x < ne * PTS; x += NT) {
    const int le = x / PTS, q = x % PTS;
    const int f = q / n2, pt = q % n2, p = pt % n1, m = pt / n1;
    double nr[4];
    if (f == 0) face_normal_unit(sX[le], 0, ops.xg[p], ops.xg[m], nr);
    else face_normal_unit(sX[le], f, ops.fa[f * n2], ops.fb[f * n2], nr);
    double outp = 0.0, outu = 0.0;
#pragma unroll
    for (int fld = 0; fld < 4; ++fld) {
      const double v = face_value<N>(sU[le] + fld * Np, f, p, m, sf, sLa, sLe);
      const double nd = fld == 1 ? nr[0] : fld == 2 ? nr[1] : nr[2];
      if (fld == 0) outp = v;
      else outu += nd * v;
    }
    T2[(e0 * PTS + x) * 2 + 0] = outp;  // row of element e0 + le, point q
    T2[(e0 * PTS + x) * 2 + 1] = outu;
  }
}

// ---------------------------------------------------------------------------
// Traces (p, u.n) of all five faces, T2[K][5 (N+1)^2][2] in the face order of
// the face points (base, then a = -1, +1, b = -1, +1), for the general variant
// of the stage.  The workgroup's state is staged in LDS; field by field the
// a-direction contractions at the a-points and at a = -1, +1, then one item
// per base point (b- and c-directions) and one per triangle edge point p (the
// line of face points (p, c_m), as in the stage).  The pressure is written at
// once, the normal velocity after the last field.  At 64^3 x 6 it takes
// 10.9 ms at N = 6 and 12.6 ms at N = 7, against 9.3 and 16.9 ms for the
// four-field matrix-core trace it replaces (the stage then reads half the
// trace bytes); all four fields' a-direction results at once, behind a single
// barrier, measured slower (12.9 and 15.4 ms) from the registers the fused
// item loops need.
template <int N>
struct TraceAllShape {
  using D = SfDims<N>;
  static constexpr int P = D::n2 + 4 * D::n1;  // items per element
  static constexpr int E = 256 / P < 1 ? 1 : 256 / P;
  static constexpr int THREADS = round64(E * P);
};

template <int N>
__global__ __launch_bounds__((TraceAllShape<N>::THREADS)) void k_sf_trace_all(
    const double* __restrict__ U, double* __restrict__ T2, SfOps sf, DevOps ops,
    const double* __restrict__ verts, int64_t K) {
  using D = SfDims<N>;
  using TS = TraceAllShape<N>;
  constexpr int n1 = D::n1, n2 = D::n2, Np = D::Np, KJ = D::KJ, E = TS::E, NT = TS::THREADS;
  constexpr int P = TS::P;
  __shared__ double sU[E][4 * Np];
  __shared__ double sA[E][KJ * n1 + 2 * KJ];  // A [kj][p], Ae [kj][2]
  __shared__ double sX[E][16];
  __shared__ double sN[E][4][4];  // triangle faces: unit normal, sJ
  __shared__ double sLa[D::n3], sLe[2 * n2];
  __shared__ int sKJ[KJ];  // (k, j) of a row index kj, packed k | j << 8
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)(K - e0 < E ? K - e0 : E);
  // state loads all in flight before the LDS stores, as in k_sf_trace
  constexpr int ST = (E * 4 * Np + NT - 1) / NT;
  const int nU = ne * 4 * Np;
  const double* Ug = U + e0 * 4 * Np;
  double ru[ST];
#pragma unroll
  for (int it = 0; it < ST; ++it) {
    const int x = tid + it * NT;
    ru[it] = x < nU ? Ug[x] : 0.0;
  }
  for (int x = tid; x < ne * 16; x += NT) sX[x / 16][x % 16] = verts[e0 * 16 + x];
  for (int x = tid; x < D::n3; x += NT) sLa[x] = sf.La[x];
  for (int x = tid; x < 2 * n2; x += NT) sLe[x] = sf.Le[x];
  double* sUf = &sU[0][0];
#pragma unroll
  for (int it = 0; it < ST; ++it) {
    const int x = tid + it * NT;
    if (x < nU) sUf[x] = ru[it];
  }
  for (int kj = tid; kj < KJ; kj += NT) {
    int k, j;
    kj_split<N>(kj, k, j);
    sKJ[kj] = k | j << 8;
  }
  __syncthreads();
  for (int x = tid; x < ne * 4; x += NT) {
    const int l = x / 4, f = x % 4 + 1;
    face_normal_unit(sX[l], f, ops.fa[f * n2], ops.fb[f * n2], sN[l][f - 1]);
  }
  // this thread's item: element l, base point q < n2 or triangle edge point
  const bool item = tid < ne * P;
  const int l = item ? tid / P : 0, q = tid % P;
  const bool base = q < n2;
  const int ft = base ? 0 : (q - n2) / n1, pp = base ? q % n1 : (q - n2) % n1;
  const int m = base ? q / n1 : 0;
  double nb[4] = {0.0, 0.0, 0.0, 0.0};
  if (item && base) face_normal_unit(sX[l], 0, ops.xg[pp], ops.xg[m], nb);
  double* row = T2 + (e0 + l) * 5 * n2 * 2;  // this element's pairs
  double un[n1];                              // u.n along this thread's line
#pragma unroll
  for (int mm = 0; mm < n1; ++mm) un[mm] = 0.0;
#pragma unroll
  for (int fld = 0; fld < 4; ++fld) {
    for (int x = tid; x < ne * KJ * n1; x += NT) {
      const int el = x / (KJ * n1), rem = x % (KJ * n1);
      const int kj = rem / n1, p = rem % n1;
      const int kjc = sKJ[kj], k = kjc & 255, j = kjc >> 8;
      const double* u = sU[el] + fld * Np + kofs(k) + j * (k + 1);
      double uu[n1];
#pragma unroll
      for (int i = 0; i < n1; ++i) uu[i] = i <= k ? u[i] : 0.0;
      const double* La = sLa + (k * n1 + p) * n1;
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < n1; ++i) a += La[i] * uu[i];
      sA[el][kj * n1 + p] = a;
      for (int sd = p; sd < 2; sd += n1) {
        const double* Le = sLe + (k * 2 + sd) * n1;
        double ae = 0.0;
#pragma unroll
        for (int i = 0; i < n1; ++i) ae += Le[i] * uu[i];
        sA[el][KJ * n1 + kj * 2 + sd] = ae;
      }
    }
    __syncthreads();
    if (item && base) {
      // u(a_p, b_m, -1) = sum_k g_k(-1) sum_j l_j(b_m) A[kj][p]
      double v = 0.0;
#pragma unroll
      for (int k = 0; k <= N; ++k) {
        const double* Lm = sLa + (k * n1 + m) * n1;
        double Y = 0.0;
#pragma unroll
        for (int j = 0; j <= k; ++j) Y += Lm[j] * sA[l][(kjofs(k) + j) * n1 + pp];
        v += sf.Gb[k] * Y;
      }
      if (fld == 0) row[q * 2] = v;
      else un[0] += nb[fld - 1] * v;
    } else if (item) {
      // faces 1, 2 (a = -1, +1): sum_k g_k(c_m) sum_j l_j(b_p) Ae[kj][s];
      // faces 3, 4 (b = -1, +1): sum_k g_k(c_m) sum_j l_j(-1 or +1) A[kj][p]
      const int f = ft + 1, sd = (f == 2 || f == 4) ? 1 : 0;
      const bool afc = f <= 2;
      double val[n1];
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) val[mm] = 0.0;
#pragma unroll
      for (int k = 0; k <= N; ++k) {
        const double* w = afc ? sLa + (k * n1 + pp) * n1 : sLe + (k * 2 + sd) * n1;
        const double* X = afc ? sA[l] + KJ * n1 + kjofs(k) * 2 + sd : sA[l] + kjofs(k) * n1 + pp;
        const int xs = afc ? 2 : n1;
        double Y = 0.0;
#pragma unroll
        for (int j = 0; j <= k; ++j) Y += w[j] * X[j * xs];
#pragma unroll
        for (int mm = 0; mm < n1; ++mm) val[mm] += sf.Gf[mm * n1 + k] * Y;
      }
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) {
        if (fld == 0) row[(f * n2 + pp + n1 * mm) * 2] = val[mm];
        else un[mm] += sN[l][ft][fld - 1] * val[mm];
      }
    }
    __syncthreads();
  }
  if (item && base) {
    row[q * 2 + 1] = un[0];
  } else if (item) {
#pragma unroll
    for (int mm = 0; mm < n1; ++mm) row[((ft + 1) * n2 + pp + n1 * mm) * 2 + 1] = un[mm];
  }
}

// ---------------------------------------------------------------------------
// Fused stage.  LOCAL: workgroups own whole hexahedra (triangle neighbours
// are in the workgroup, T2 holds (p, u.n) base traces only); otherwise T2
// holds the (p, u.n) pairs of all five faces, [K][Nfc][2].
// Waves per SIMD the stage is compiled for: three at N = 5 (whole
// hexahedra, three workgroups per CU; 30.3 -> 27.2 ms per stage at 64^3 x 6
// when it was introduced) and N = 6 (general variant, 5 elements per
// workgroup, three workgroups per CU: 32.3 -> 28.7 ms); at N = 4 three waves
// measured slower (20.7 -> 22.5 ms), and the other orders are left to the
// compiler.
template <int N>
struct SfWaves {
  static constexpr int value = N == 5 || N == 6 ? 3 : 1;
};

template <int N, int MODE, bool LOCAL>
__global__ __launch_bounds__((SfShape<N, LOCAL>::THREADS), (SfWaves<N>::value)) void k_sf_stage(
    const double* U, const double* __restrict__ T2, SfOps sf, DevOps ops, DevMesh mesh,
    double* out, double* R, double ra, double rb, double dt) {
  using D = SfDims<N>;
  constexpr int n1 = D::n1, n2 = D::n2, Np = D::Np, KJ = D::KJ;
  constexpr int E = SfShape<N, LOCAL>::E, NT = SfShape<N, LOCAL>::THREADS;
  constexpr int CREG = D::kSeparateC ? D::CC : D::TT;
  __shared__ double sX[E][16];
  __shared__ double sN[E][4][4];   // triangle faces 1..4: unit normal, sJ
  __shared__ double sZ[E][5];      // rho c across each face (own on the boundary)
  __shared__ double sM[E][4];      // kappa, 1/rho, rho c, time-step scale
  __shared__ int sNb[E][5][4];     // neighbour, its index in the workgroup or -1, its face, permutation row
  __shared__ double sUD[E][D::UD];
  __shared__ double sAB[E][D::AB];
  __shared__ double sTT[E][D::TT];
  __shared__ double sCC[D::kSeparateC ? E : 1][D::kSeparateC ? D::CC : 1];
  __shared__ int sPerm[10 * n2];
  __shared__ int sPad[Np];       // position of coefficient n in the padded row layout [kj][i]
  __shared__ int sKJ[KJ];        // (k, j) of a row index kj, packed k | j << 8
  __shared__ int sKJI[Np];       // (k, j, i) of a coefficient index, packed k | j << 8 | i << 16
  __shared__ double sJc[E][4];   // bilinear Jacobian coefficients (1, a, b, ab)
  __shared__ double sLa[D::n3], sDa[D::n3], sLe[2 * n2];
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)(mesh.K - e0 < E ? mesh.K - e0 : E);
  // this workgroup's rows of the state and residual: 32-bit offsets below
  const double* Uw = U + e0 * 4 * Np;
  double* ow = out + e0 * 4 * Np;
  double* Rw = MODE == 1 ? R + e0 * 4 * Np : nullptr;

  // ---- tables: vertices, face neighbours, triangle normals, permutations,
  // one-dimensional factors
  stage_tables<N>(sf, sLa, sDa, sLe, tid, NT);
  for (int x = tid; x < E * 16; x += NT) {
    const int le = x / 16;
    sX[le][x % 16] = le < ne ? mesh.verts[(e0 + le) * 16 + x % 16] : 0.0;
  }
  for (int x = tid; x < E * 4; x += NT) {
    const int le = x / 4;
    sM[le][x % 4] = le < ne ? mesh.mat[(e0 + le) * 4 + x % 4] : 0.0;
  }
  for (int x = tid; x < 10 * n2; x += NT) sPerm[x] = ops.perm[x];
  // the coefficients pass through LDS in rows of N+1 (row kj = (k, j) holds
  // u_ijk at i, zeros beyond i = k), so that the a-direction needs no masks
  for (int n = tid; n < Np; n += NT) {
    int k, j, i;
    kji_split<N>(n, k, j, i);
    sPad[n] = (kjofs(k) + j) * n1 + i;
    sKJI[n] = k | j << 8 | i << 16;
  }
  for (int kj = tid; kj < KJ; kj += NT) {
    int k, j;
    kj_split<N>(kj, k, j);
    sKJ[kj] = k | j << 8;
  }
  for (int x = tid; x < E * D::UD; x += NT) sUD[x / D::UD][x % D::UD] = 0.0;
  __syncthreads();
  for (int x = tid; x < E; x += NT) pyr_jac_coeffs(sX[x], sJc[x]);
  for (int x = tid; x < E * 5; x += NT) {
    const int le = x / 5, f = x % 5;
    int nb = -1, loc = -1, nf = 0, prow = 0;
    double z = 1.0;
    if (le < ne) {
      const int64_t e = e0 + le;
      nb = mesh.conn[e * 8 + f];
      z = mesh.mat[e * 4 + 2];
      if (nb >= 0) {
        const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
        nf = code & 7;
        prow = (f == 0 ? (code >> 3) : 8 + (code >> 3)) * n2;
        loc = (nb >= e0 && nb < e0 + ne) ? (int)(nb - e0) : -1;
        z = mesh.mat[(int64_t)nb * 4 + 2];
      }
      if (f > 0) face_normal_unit(sX[le], f, ops.fa[f * n2], ops.fb[f * n2], sN[le][f - 1]);
    }
    sNb[le][f][0] = nb;
    sNb[le][f][1] = loc;
    sNb[le][f][2] = nf;
    sNb[le][f][3] = prow;
    sZ[le][f] = z;
  }

  // ---- column of this thread: element le, base point (p, m)
  const bool col = tid < ne * n2;
  const int le = col ? tid / n2 : 0;
  const int pm = tid % n2, p = pm % n1, m = pm / n1;
  const int64_t e = e0 + le;
  double adj[9], Jc;
  pyr_metric(sX[le], ops.xg[p], ops.xg[m], adj, &Jc);
  const double wab = 0.25 * ops.wf[pm];  // w_p w_m / 4
  const double ha = 0.5 * (1.0 + ops.xg[p]), hb = 0.5 * (1.0 + ops.xg[m]);
  double bacc[4][n1];  // projection onto g_k(c_r): [field][k]
  double qp[n1];       // w-less divergence of u at c_r
  double tb[4];        // own base trace of each field at (p, m)
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    tb[f] = 0.0;
#pragma unroll
    for (int k = 0; k < n1; ++k) bacc[f][k] = 0.0;
  }
#pragma unroll
  for (int r = 0; r < n1; ++r) qp[r] = 0.0;

  // ---- volume term and own traces, one field at a time: the velocities
  // first (they only add to the pressure row's projection), the pressure
  // last, so that the velocity rows' projections are live in registers only
  // from there on
  // The next field's coefficients are loaded into registers while the current
  // field's a-direction runs and stored into LDS once its readers are past the
  // barrier, so a field costs two barriers and its load latency is hidden.
  constexpr int LD = (E * Np + NT - 1) / NT;  // coefficients each thread stages
  for (int x = tid; x < E * Np; x += NT) {
    const int l = x / Np, n = x % Np;
    sUD[l][sPad[n]] = l < ne ? Uw[(l * 4 + 1) * Np + n] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int fld = (it + 1) & 3;
    double nxt[LD];
    if (it < 3) {
      const int nfld = (it + 2) & 3;
#pragma unroll
      for (int q = 0; q < LD; ++q) {
        const int x = tid + q * NT, l = x / Np, n = x % Np;
        nxt[q] = (x < E * Np && l < ne) ? Uw[(l * 4 + nfld) * Np + n] : 0.0;
      }
    }
    // a-direction: A[kj][p] = sum_i l_i(a_p) u_ijk, A'[kj][p] with l'_i(a_p)
    for (int x = tid; x < ne * KJ * n1; x += NT) {
      const int l = x / (KJ * n1), rem = x % (KJ * n1);
      const int kj = rem / n1, pp = rem % n1;
      const int kjc = sKJ[kj], k = kjc & 255, j = kjc >> 8;
      const double* u = sUD[l] + kj * n1;  // padded row: zeros beyond i = k
      const double* La = sLa + (k * n1 + pp) * n1;
      const double* Da = sDa + (k * n1 + pp) * n1;
      double a = 0.0, ad = 0.0;
#pragma unroll
      for (int i = 0; i < n1; ++i) {
        a += La[i] * u[i];
        ad += Da[i] * u[i];
      }
      sAB[l][kj * n1 + pp] = a;
      sAB[l][KJ * n1 + kj * n1 + pp] = ad;
      // Ae[kj][s] = sum_i l_i(-1 or +1) u_ijk, by the items p = 0 and 1 (p = 0
      // takes both when N = 0)
      for (int sd = pp; sd < 2; sd += n1) {
        const double* Le = sLe + (k * 2 + sd) * n1;
        double ae = 0.0;
#pragma unroll
        for (int i = 0; i < n1; ++i) ae += Le[i] * u[i];
        sAB[l][2 * KJ * n1 + kj * 2 + sd] = ae;
      }
    }
    __syncthreads();
    if (it < 3) {
#pragma unroll
      for (int q = 0; q < LD; ++q) {
        const int x = tid + q * NT;
        if (x < E * Np) sUD[x / Np][sPad[x % Np]] = nxt[q];
      }
    }
    // b- and c-directions, metric and projection along c, per column
    if (col) {
      double s0[n1], sa[n1], sb[n1];
#pragma unroll
      for (int k = 0; k < n1; ++k) {
        const double* La_m = sLa + (k * n1 + m) * n1;
        const double* Da_m = sDa + (k * n1 + m) * n1;
        double x0 = 0.0, xa = 0.0, xb = 0.0;
#pragma unroll
        for (int j = 0; j <= k; ++j) {
          const double A = sAB[le][(kjofs(k) + j) * n1 + p];
          const double Ad = sAB[le][KJ * n1 + (kjofs(k) + j) * n1 + p];
          x0 += La_m[j] * A;
          xa += La_m[j] * Ad;
          xb += Da_m[j] * A;
        }
        s0[k] = x0;
        sa[k] = xa;
        sb[k] = xb;
        tb[fld] += sf.Gb[k] * x0;
      }
      if (fld == 0) {
#pragma unroll
        for (int r = 0; r < n1; ++r) {
          double dr = 0.0, ds = 0.0, dtp = 0.0;
#pragma unroll
          for (int k = 0; k < n1; ++k) {
            dr += sf.Gt[r * n1 + k] * sa[k];
            ds += sf.Gt[r * n1 + k] * sb[k];
            dtp += sf.Gp[r * n1 + k] * s0[k];
          }
          const double dtt = dtp + ha * dr + hb * ds;
          // Q_{u_d} = w sum_rho adj[rho][d] d_rho p, projected onto g_k(c_r)
          const double w = wab * sf.wc[r];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double q = w * (adj[d] * dr + adj[3 + d] * ds + adj[6 + d] * dtt);
#pragma unroll
            for (int k = 0; k < n1; ++k) bacc[1 + d][k] += sf.G[r * n1 + k] * q;
          }
        }
      } else {
        // the d-th term of div u, sum_rho adj[rho][d] d_rho u_d with
        // d_t = d_t' + (1+a)/2 d_r + (1+b)/2 d_s, folded into the column's
        // constants before the c-direction: one combined c-contraction
        const int d = fld - 1;
        const double ca = adj[d] + ha * adj[6 + d], cb = adj[3 + d] + hb * adj[6 + d];
        const double ct = adj[6 + d];
        double tk[n1];
#pragma unroll
        for (int k = 0; k < n1; ++k) tk[k] = ca * sa[k] + cb * sb[k];
#pragma unroll
        for (int r = 0; r < n1; ++r) {
          double g1 = 0.0, g2 = 0.0;
#pragma unroll
          for (int k = 0; k < n1; ++k) {
            g1 += sf.Gt[r * n1 + k] * tk[k];
            g2 += sf.Gp[r * n1 + k] * s0[k];
          }
          qp[r] += g1 + ct * g2;
        }
      }
    }
    // triangle traces of this field from the a-direction results, item
    // (element, face, edge point p), at the face points (p, c_m):
    //   a = -1, +1 (faces 1, 2): sum_k g_k(c_m) sum_j l_j(b_p) Ae[kj][s],
    //   b = -1, +1 (faces 3, 4): sum_k g_k(c_m) sum_j l_j(-1 or +1) A[kj][p]
    for (int x = tid; x < ne * 4 * n1; x += NT) {
      const int l = x / (4 * n1), rem = x % (4 * n1);
      const int ft = rem / n1, pp = rem % n1, f = ft + 1;
      const int sd = (f == 2 || f == 4) ? 1 : 0;
      const bool afc = f <= 2;
      double val[n1];
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) val[mm] = 0.0;
#pragma unroll
      for (int k = 0; k <= N; ++k) {
        // weights and values of row j: (l_j(b_p), Ae[kj][s]) or (l_j(+-1), A[kj][p])
        const double* w = afc ? sLa + (k * n1 + pp) * n1 : sLe + (k * 2 + sd) * n1;
        const double* X = afc ? sAB[l] + 2 * KJ * n1 + kjofs(k) * 2 + sd
                              : sAB[l] + kjofs(k) * n1 + pp;
        const int xs = afc ? 2 : n1;
        double Y = 0.0;
#pragma unroll
        for (int j = 0; j <= k; ++j) Y += w[j] * X[j * xs];
#pragma unroll
        for (int mm = 0; mm < n1; ++mm) val[mm] += sf.Gf[mm * n1 + k] * Y;
      }
      double* tt = sTT[l] + ft * 2 * n2;
      const double nd = fld == 0 ? 0.0 : sN[l][ft][fld - 1];
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) {
        const int pt = pp + n1 * mm;
        if (fld == 0) tt[pt] = val[mm];
        else if (fld == 1) tt[n2 + pt] = nd * val[mm];
        else tt[n2 + pt] += nd * val[mm];
      }
    }
    __syncthreads();
  }

  // ---- base face: flux at (p, m) from the own traces and the neighbour's
  if (col) {
#pragma unroll
    for (int r = 0; r < n1; ++r) {
      const double w = wab * sf.wc[r] * qp[r];
#pragma unroll
      for (int k = 0; k < n1; ++k) bacc[0][k] += sf.G[r * n1 + k] * w;
    }
    double nr[4];
    face_normal_unit(sX[le], 0, ops.xg[p], ops.xg[m], nr);
    const double pmv = tb[0];
    const double unm = nr[0] * tb[1] + nr[1] * tb[2] + nr[2] * tb[3];
    const int nb = sNb[le][0][0];
    double nbp = 0.0, nbun = 0.0;
    if (nb >= 0) {
      const int q2 = sPerm[sNb[le][0][3] + pm];
      if constexpr (LOCAL) {  // (p, u.n') pairs
        const double* tp = T2 + ((int64_t)nb * n2 + q2) * 2;
        nbp = tp[0];
        nbun = tp[1];
      } else {  // pairs of all five faces
        const double* tp = T2 + ((int64_t)nb * D::Nfc + sNb[le][0][2] * n2 + q2) * 2;
        nbp = tp[0];
        nbun = tp[1];
      }
    }
    double pp, unp, Fp, Pu;
    exterior(nb >= 0, nbp, nbun, pmv, unm, mesh.bc, pp, unp);
    jump_flux(pp - pmv, unp - unm, mesh.mat[e * 4 + 2], sZ[le][0], mesh.alpha,
              ops.wf[pm] * nr[3], Fp, Pu);
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const double g = sf.Gb[k];
      bacc[0][k] += g * Fp;
      bacc[1][k] += g * nr[0] * Pu;
      bacc[2][k] += g * nr[1] * Pu;
      bacc[3][k] += g * nr[2] * Pu;
    }
  }

  // ---- triangle faces: fluxes along each edge-point line, folded onto g_k(c)
  {
    double cp[n1], cu[n1];
    int item = -1;
    for (int x = tid; x < ne * 4 * n1; x += NT) {
      const int l = x / (4 * n1), rem = x % (4 * n1);
      const int ft = rem / n1, pp = rem % n1, f = ft + 1;
      const double* nrm = sN[l][ft];
      const int nb = sNb[l][f][0], nf = sNb[l][f][2], prow = sNb[l][f][3];
      const int loc = LOCAL ? sNb[l][f][1] : -1;
      const double zm = mesh.mat[(e0 + l) * 4 + 2], zp = sZ[l][f];
      const double* tt = sTT[l] + ft * 2 * n2;
#pragma unroll
      for (int k = 0; k < n1; ++k) cp[k] = cu[k] = 0.0;
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) {
        const int pt = pp + n1 * mm;
        const double pmv = tt[pt], unm = tt[n2 + pt];
        double nbp = 0.0, nbun = 0.0;
        if (nb >= 0) {
          const int q2 = sPerm[prow + pt];
          if constexpr (LOCAL) {  // the sibling pyramid is in this workgroup
            nbp = sTT[loc][(nf - 1) * 2 * n2 + q2];
            nbun = sTT[loc][(nf - 1) * 2 * n2 + n2 + q2];
          } else {
            const double* tp = T2 + ((int64_t)nb * D::Nfc + nf * n2 + q2) * 2;
            nbp = tp[0];
            nbun = tp[1];
          }
        }
        double ppv, unp, Fp, Pu;
        exterior(nb >= 0, nbp, nbun, pmv, unm, mesh.bc, ppv, unp);
        jump_flux(ppv - pmv, unp - unm, zm, zp, mesh.alpha, ops.wf[f * n2 + pt] * nrm[3], Fp, Pu);
#pragma unroll
        for (int k = 0; k < n1; ++k) {
          cp[k] += sf.Gf[mm * n1 + k] * Fp;
          cu[k] += sf.Gf[mm * n1 + k] * Pu;
        }
      }
      if (D::kSeparateC) {
        double* cc = (double*)sCC[l] + ft * 2 * n2;
#pragma unroll
        for (int k = 0; k < n1; ++k) {
          cc[k * n1 + pp] = cp[k];
          cc[n2 + k * n1 + pp] = cu[k];
        }
      } else {
        item = x;  // at most one item per thread (4 n1 <= n2 <= columns)
      }
    }
    if (!D::kSeparateC) {
      __syncthreads();  // every trace read before the folded fluxes replace them
      if (item >= 0) {
        const int l = item / (4 * n1), rem = item % (4 * n1);
        const int ft = rem / n1, pp = rem % n1;
        double* cc = sTT[l] + ft * 2 * n2;
#pragma unroll
        for (int k = 0; k < n1; ++k) {
          cc[k * n1 + pp] = cp[k];
          cc[n2 + k * n1 + pp] = cu[k];
        }
      }
    }
  }

  // ---- lift sums of the folded triangle fluxes, shared by the coefficients
  // of a row: Tl[ty][face][kj] = sum_p l^k_r(x_p) cc[face][ty][k][p] with r = j
  // for the a = -1, +1 faces and r = i for the b = -1, +1 faces (both the row
  // index of kj = (k, r)); ty 0 lifts the pressure flux, 1 the velocity one.
  // They replace the folded fluxes in the trace region.
  __syncthreads();
  {
    constexpr int TI = 8 * KJ;                   // sums per element
    constexpr int LT = (E * TI + NT - 1) / NT;  // sums per thread
    double tv[LT];
#pragma unroll
    for (int q = 0; q < LT; ++q) {
      const int x = tid + q * NT;
      tv[q] = 0.0;
      if (x < ne * TI) {
        const int l = x / TI, rem = x % TI;
        const int tf = rem / KJ, kj = rem % KJ, ty = tf / 4, face = tf % 4;
        const int kjc = sKJ[kj], k = kjc & 255, r = kjc >> 8;
        const double* cc = (D::kSeparateC ? (const double*)sCC[l] : (const double*)sTT[l]) +
                           face * 2 * n2 + ty * n2 + k * n1;
        const double* Lr = sLa + k * n2 + r;  // l^k_r(x_p) at p * n1
        double acc = 0.0;
#pragma unroll
        for (int pp = 0; pp < n1; ++pp) acc += Lr[pp * n1] * cc[pp];
        tv[q] = acc;
      }
    }
    __syncthreads();  // every folded flux read before the sums replace them
#pragma unroll
    for (int q = 0; q < LT; ++q) {
      const int x = tid + q * NT;
      if (x < ne * TI) sTT[x / TI][x % TI] = tv[q];
    }
  }

  // ---- projection, one field at a time: b-direction, then a-direction with
  // the triangle lifts, inverse mass, material and the RK stage.  The inverse
  // mass diagonal of this thread's coefficients is evaluated once for the
  // four fields.
  double minv[LD];
#pragma unroll
  for (int q = 0; q < LD; ++q) {
    const int x = tid + q * NT, l = x / Np, n = x % Np;
    minv[q] = x < ne * Np ? 1.0 / (pyr_jac_eval(sJc[l], ops.na[n], ops.nb[n]) * ops.wwc[n]) : 0.0;
  }
#pragma unroll
  for (int fld = 0; fld < 4; ++fld) {
    // in RK mode this field's state and residual are loaded here, ahead of
    // the b-direction pass, and used by the update at its end
    double uo[LD], ro[LD];
    if constexpr (MODE == 1) {
#pragma unroll
      for (int q = 0; q < LD; ++q) {
        const int x = tid + q * NT;
        uo[q] = ro[q] = 0.0;
        if (x < ne * Np) {
          const int idx = (x / Np * 4 + fld) * Np + x % Np;
          uo[q] = ow[idx];
          if (ra != 0.0) ro[q] = Rw[idx];
        }
      }
    }
    if (col) {
#pragma unroll
      for (int k = 0; k < n1; ++k) sAB[le][k * n2 + m * n1 + p] = bacc[fld][k];
    }
    __syncthreads();
    // D[kj][p] = sum_m l_j(b_m) B[k][m][p]
    for (int x = tid; x < ne * KJ * n1; x += NT) {
      const int l = x / (KJ * n1), rem = x % (KJ * n1);
      const int kj = rem / n1, pp = rem % n1;
      const int kjc = sKJ[kj], k = kjc & 255, j = kjc >> 8;
      const double* B = sAB[l] + k * n2 + pp;
      double acc = 0.0;
#pragma unroll
      for (int mm = 0; mm < n1; ++mm) acc += sLa[(k * n1 + mm) * n1 + j] * B[mm * n1];
      sUD[l][kj * n1 + pp] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LD; ++q) {
      const int x = tid + q * NT;
      if (x >= ne * Np) continue;
      const int l = x / Np, n = x % Np;
      const int kc = sKJI[n], k = kc & 255, j = (kc >> 8) & 255, i = kc >> 16;
      const double* La_k = sLa + k * n2;  // [p][i]
      const double* Dk = sUD[l] + (kjofs(k) + j) * n1;
      const double* Tl = sTT[l] + (fld == 0 ? 0 : 4 * KJ) + kjofs(k);
      double v = 0.0;
#pragma unroll
      for (int pp = 0; pp < n1; ++pp) v += La_k[pp * n1 + i] * Dk[pp];
      const double t1 = Tl[j], t2 = Tl[KJ + j], t3 = Tl[2 * KJ + i], t4 = Tl[3 * KJ + i];
      const double* Le_k = sLe + k * 2 * n1;  // [side][i]
      double s1 = 1.0, s2 = 1.0, s3 = 1.0, s4 = 1.0;
      if (fld > 0) {
        s1 = sN[l][0][fld - 1];
        s2 = sN[l][1][fld - 1];
        s3 = sN[l][2][fld - 1];
        s4 = sN[l][3][fld - 1];
      }
      v += s1 * Le_k[i] * t1 + s2 * Le_k[n1 + i] * t2 + s3 * Le_k[j] * t3 + s4 * Le_k[n1 + j] * t4;
      const int64_t el = e0 + l;
      if (fld == 0) v -= source_term<Np>(mesh, el, n);
      const int idx = (l * 4 + fld) * Np + n;
      const double rhs = -sM[l][fld == 0 ? 0 : 1] * minv[q] * v;
      if constexpr (MODE == 0) {
        ow[idx] = rhs;
      } else {  // R <- ra R + dt rhs, U <- U + rb R (finish_coeff with the loads above)
        const double rn = ra * ro[q] + dt * sM[l][3] * rhs;
        Rw[idx] = rn;
        ow[idx] = uo[q] + rb * rn;
      }
    }
    __syncthreads();
  }
  (void)CREG;
}

// Resources of a kernel against the device's limits and this file's budgets
// (checked at setup, before any launch).
dgpyr_status check_kernel(const void* fn, int threads, const char* name, std::string& msg) {
  hipFuncAttributes a;
  hipError_t err = hipFuncGetAttributes(&a, fn);
  if (err != hipSuccess) {
    msg = std::string("hipFuncGetAttributes(") + name + "): " + hipGetErrorString(err);
    return DGPYR_E_HIP;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  err = hipGetDevice(&dev);
  if (err == hipSuccess) err = hipGetDeviceProperties(&prop, dev);
  if (err != hipSuccess) {
    msg = std::string("device properties: ") + hipGetErrorString(err);
    return DGPYR_E_HIP;
  }
  if (a.sharedSizeBytes > (size_t)kLdsBudget || a.sharedSizeBytes > prop.sharedMemPerBlock ||
      a.localSizeBytes > kPrivateBudget || a.maxThreadsPerBlock < threads) {
    msg = std::string(name) + ": " + std::to_string(a.sharedSizeBytes) + " bytes of LDS (device " +
          std::to_string(prop.sharedMemPerBlock) + "), " + std::to_string(a.localSizeBytes) +
          " bytes of private memory per lane, " + std::to_string(threads) + " threads (at most " +
          std::to_string(a.maxThreadsPerBlock) + ")";
    return DGPYR_E_UNSUPPORTED;
  }
  return DGPYR_OK;
}

template <int N>
dgpyr_status check_n(const dgpyr_ctx& c, std::string& msg) {
  dgpyr_status st;
  if constexpr (SfDims<N>::hex_elems() > 0) {
    if (c.sf_local) {
      if ((st = check_kernel((const void*)k_sf_trace<N, 1>, TraceShape<N, 1>::THREADS,
                             "k_sf_trace", msg)))
        return st;
      if ((st = check_kernel((const void*)k_sf_stage<N, 0, true>, SfShape<N, true>::THREADS,
                             "k_sf_stage", msg)))
        return st;
      return check_kernel((const void*)k_sf_stage<N, 1, true>, SfShape<N, true>::THREADS,
                          "k_sf_stage", msg);
    }
  }
  if ((st = check_kernel((const void*)k_sf_trace_all<N>, TraceAllShape<N>::THREADS,
                         "k_sf_trace_all", msg)))
    return st;
  if ((st = check_kernel((const void*)k_sf_stage<N, 0, false>, SfShape<N, false>::THREADS,
                         "k_sf_stage", msg)))
    return st;
  return check_kernel((const void*)k_sf_stage<N, 1, false>, SfShape<N, false>::THREADS,
                      "k_sf_stage", msg);
}

template <int N>
hipError_t trace_n(const dgpyr_ctx& c, const double* U, double* T2, hipStream_t s) {
  if (c.sf_local) {
    if constexpr (SfDims<N>::hex_elems() > 0) {
      using TS = TraceShape<N, 1>;
      hipLaunchKernelGGL((k_sf_trace<N, 1>), dim3((unsigned)((c.K + TS::E - 1) / TS::E)),
                         dim3(TS::THREADS), 0, s, U, T2, c.sf, c.ops, c.mesh.verts, c.K);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    using TA = TraceAllShape<N>;
    hipLaunchKernelGGL((k_sf_trace_all<N>), dim3((unsigned)((c.K + TA::E - 1) / TA::E)),
                       dim3(TA::THREADS), 0, s, U, T2, c.sf, c.ops, c.mesh.verts, c.K);
  }
  return hipGetLastError();
}

template <int N, bool LOCAL>
hipError_t stage_nl(const dgpyr_ctx& c, int mode, const double* U, const double* T2, double* out,
                    double* R, double ra, double rb, double dt, hipStream_t s) {
  using SS = SfShape<N, LOCAL>;
  const dim3 grid((unsigned)((c.K + SS::E - 1) / SS::E)), block(SS::THREADS);
  if (mode == 0)
    hipLaunchKernelGGL((k_sf_stage<N, 0, LOCAL>), grid, block, 0, s, U, T2, c.sf, c.ops, c.mesh,
                       out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_sf_stage<N, 1, LOCAL>), grid, block, 0, s, U, T2, c.sf, c.ops, c.mesh,
                       out, R, ra, rb, dt);
  return hipGetLastError();
}

template <int N>
hipError_t stage_n(const dgpyr_ctx& c, int mode, const double* U, const double* T2, double* out,
                   double* R, double ra, double rb, double dt, hipStream_t s) {
  if constexpr (SfDims<N>::hex_elems() > 0) {
    if (c.sf_local) return stage_nl<N, true>(c, mode, U, T2, out, R, ra, rb, dt, s);
  }
  if (c.sf_local) return hipErrorInvalidValue;
  return stage_nl<N, false>(c, mode, U, T2, out, R, ra, rb, dt, s);
}

template <int N>
bool local_possible() {
  return SfDims<N>::hex_elems() > 0;
}

}  // namespace

#define DGPYR_DISPATCH_SF(fn, fail, ...) \
  switch (c.N) {                        \
    case 0: return fn<0>(__VA_ARGS__);  \
    case 1: return fn<1>(__VA_ARGS__);  \
    case 2: return fn<2>(__VA_ARGS__);  \
    case 3: return fn<3>(__VA_ARGS__);  \
    case 4: return fn<4>(__VA_ARGS__);  \
    case 5: return fn<5>(__VA_ARGS__);  \
    case 6: return fn<6>(__VA_ARGS__);  \
    case 7: return fn<7>(__VA_ARGS__);  \
    case 8: return fn<8>(__VA_ARGS__);  \
    default: return fail;               \
  }

bool sf_local_possible(const dgpyr_ctx& c) { DGPYR_DISPATCH_SF(local_possible, false, ) }

dgpyr_status sf_check_resources(const dgpyr_ctx& c, std::string& msg) {
  DGPYR_DISPATCH_SF(check_n, DGPYR_E_ORDER, c, msg)
}

hipError_t launch_sf_trace(const dgpyr_ctx& c, const double* U, double* T2, hipStream_t s) {
  DGPYR_DISPATCH_SF(trace_n, hipErrorInvalidValue, c, U, T2, s)
}

hipError_t launch_sf_stage(const dgpyr_ctx& c, int mode, const double* U, const double* T2,
                           double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  DGPYR_DISPATCH_SF(stage_n, hipErrorInvalidValue, c, mode, U, T2, out, R, ra, rb, dt, s)
}

}  // namespace dgpyr
