// FP64 CPU reference ("oracle") for the lattice Boltzmann hot path of
// Geller, Uphoff & Krafczyk, "Turbulent jet computations based on MRT and
// Cascaded Lattice Boltzmann models" (arXiv:1206.0389).
//
// TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library. The GPU library never
// links, includes or calls it; the two share no code, header or table.
//
// Everything is plain double precision, written from the definitions:
//   velocity sets, weights           Section 2, the D3Q19/D3Q27 tables
//   incompressible equilibrium       Eq. (2), deviation form (no rest term)
//   macroscopic moments              Eqs. (3)-(5) incompressible,
//                                    Eqs. (6)-(8) compressible
//   MRT collision                    Eq. (12) with m_eq = M f_eq, Table 1
//   relaxation time                  Eq. (13): tau = 3 nu + 1/2
//   Smagorinsky closure              Eqs. (16)-(21), closed form Eq. (20)
//   central moments / FCLB           Eqs. (14)-(15), Table 2 equilibria
//   streaming                        left side of Eq. (1), two-lattice pull
// Where the printed formulas are garbled, the readings used are listed in
// the design notes of the repository; each is flagged at its use below.
//
// Build: g++ -O3 -fopenmp -ffp-contract=off -shared -fPIC (no FMA
// contraction, so results do not depend on the host compiler's choices).

#include <cmath>
#include <omp.h>
#include <cstdint>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

extern "C" {

enum { ORC_MRT19 = 1, ORC_FCLB27 = 2, ORC_CLB27 = 3 };
enum { ORC_BASIS_TABLE1 = 0, ORC_BASIS_DHUMIERES = 1 };
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_INLET = 2, ORC_OUTFLOW = 3, ORC_FREESLIP = 4,
       ORC_PRESSURE = 5 };

// Must match the ctypes structure in oracle/__init__.py.
typedef struct orc_params {
  int32_t model;        // ORC_MRT19, ORC_FCLB27 or ORC_CLB27
  int32_t nx, ny, nz;   // lattice (or window) extent
  double nu;            // lattice kinematic viscosity -> tau0 = 3 nu + 1/2
  double cs_smag;       // Smagorinsky constant (MRT only; 0 = off)
  int32_t mrt_basis;    // ORC_BASIS_TABLE1 or ORC_BASIS_DHUMIERES
  int32_t pad0;
  double rates[8];      // non-shear rates, meaning set by the basis
  int32_t face_type[6]; // x-, x+, y-, y+, z-, z+
  double face_u[6][3];  // wall velocity of WALL faces
  const double* inlet_u;      // [3][nb][na] velocity on the INLET face
  const uint8_t* inlet_mask;  // [nb][na] 1 = perturbed node (may be null)
  double inlet_amp;           // perturbation amplitude
  uint64_t seed;              // perturbation seed
  int32_t origin[3];          // global coordinate of local node (0,0,0)
  int32_t inlet_na, inlet_nb; // global extent of the inlet face arrays
  const uint8_t* solid;       // [N] nonzero = solid node (may be null)
  double face_drho[6];        // density deviation of PRESSURE faces
  const double* link_q;       // [Q][N] wall distance of the link from node x
                              // towards the solid x + e_i, as a fraction of
                              // the link (0 or null: halfway)
} orc_params;

}  // extern "C"

namespace {

// D3Q27 velocities in the order of the tables of Section 2; the first 19
// entries are the D3Q19 set, printed identically there.
const int E[27][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}, {1, 1, 1},
    {-1, 1, 1},  {1, -1, 1},  {1, 1, -1},  {-1, -1, 1}, {-1, 1, -1},
    {1, -1, -1}, {-1, -1, -1}};

int nq(int model) { return model == ORC_MRT19 ? 19 : 27; }

// Weights quoted in Section 2: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27,
// 1/54, 1/216, chosen by the number of non-zero velocity components.
double weight(int Q, int i) {
  int n = std::abs(E[i][0]) + std::abs(E[i][1]) + std::abs(E[i][2]);
  if (Q == 19) {
    const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    return w[n];
  }
  const double w[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  return w[n];
}

int opposite(int Q, int i) {
  for (int j = 0; j < Q; ++j)
    if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2])
      return j;
  return -1;
}

// Forward-mode dual number (value, derivative along one direction): exact
// Jacobian-vector products of the oracle's own double-precision code.
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
// Square root; at 0 the derivative is taken as 0 (the strain magnitude of
// Eq. (19) is not differentiable at zero strain: this picks the subgradient
// 0 there).
inline Dual sqrt(Dual a) {
  const double r = std::sqrt(a.v);
  return Dual(r, r > 0.0 ? a.d / (2.0 * r) : 0.0);
}
inline double value_of(double x) { return x; }
inline double value_of(Dual x) { return x.v; }
inline bool is_zero(double x) { return x == 0.0; }
inline bool is_zero(Dual x) { return x.v == 0.0 && x.d == 0.0; }

template <typename T>
T ipow(T x, int k) {
  T r = 1.0;
  for (int j = 0; j < k; ++j) r = r * x;
  return r;
}

// Gaussian elimination with partial pivoting: solves A x = b in place
// (A is n x n row-major and is destroyed; b becomes x). Pivots are chosen
// on values, so a dual-number solve follows the same elimination.
template <typename T>
void dense_solve(int n, T* A, T* b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(value_of(A[k * n + k]));
    for (int r = k + 1; r < n; ++r) {
      double v = std::fabs(value_of(A[r * n + k]));
      if (v > best) { best = v; p = r; }
    }
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[p * n + c]);
      std::swap(b[k], b[p]);
    }
    for (int r = k + 1; r < n; ++r) {
      T l = A[r * n + k] / A[k * n + k];
      if (is_zero(l)) continue;
      for (int c = k; c < n; ++c) A[r * n + c] -= l * A[k * n + c];
      b[r] -= l * b[k];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    T s = b[r];
    for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * b[c];
    b[r] = s / A[r * n + r];
  }
}

void dense_inverse(int n, const double* A, double* Ainv) {
  std::vector<double> work(n * n), col(n);
  for (int j = 0; j < n; ++j) {
    std::memcpy(work.data(), A, sizeof(double) * n * n);
    for (int r = 0; r < n; ++r) col[r] = (r == j) ? 1.0 : 0.0;
    dense_solve(n, work.data(), col.data());
    for (int r = 0; r < n; ++r) Ainv[r * n + j] = col[r];
  }
}

// ---------------------------------------------------------------------------
// Eq. (2): He-Luo incompressible equilibrium, deviation form (rho0 = 1, the
// lattice speed c = 1 so the printed c_s denominators read as c).
template <typename T>
void feq_incomp(int Q, T drho, const T u[3], T* feq) {
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    const T eu = T(E[i][0]) * u[0] + T(E[i][1]) * u[1] + T(E[i][2]) * u[2];
    feq[i] = T(weight(Q, i)) * (drho + T(3.0) * eu + T(4.5) * eu * eu - T(1.5) * uu);
  }
}

// One-dimensional factor of the D3Q27 product equilibrium: its moments
// about u are 1, 0, 1/3 (the Gaussian values the FCLB equilibria of
// Table 2 are built from).
double phi(int e, double u) {
  if (e == 0) return 2.0 / 3.0 - u * u;
  return 0.5 * (1.0 / 3.0 + u * u + e * u);
}

// ---------------------------------------------------------------------------
// MRT moment bases (rows = moments, columns = populations of D3Q19).
double basis_row(int basis, int k, const int* e) {
  const double x = e[0], y = e[1], z = e[2];
  const double x2 = x * x, y2 = y * y, z2 = z * z, e2 = x2 + y2 + z2;
  if (basis == ORC_BASIS_TABLE1) {
    // Table 1 groups in moment notation mu_{x^i y^j z^k}.
    switch (k) {
      case 0: return 1.0;
      case 1: return x;
      case 2: return y;
      case 3: return z;
      case 4: return x * y;            // s1: mu_12
      case 5: return x * z;            // s1: mu_13
      case 6: return y * z;            // s1: mu_23
      case 7: return x2 - y2;          // s1: mu_11 - mu_22
      case 8: return x2 - z2;          // s1: mu_11 - mu_33
      case 9: return e2;               // s2: mu_11 + mu_22 + mu_33
      case 10: return x * y2 + x * z2; // s3: mu_122 + mu_133
      case 11: return x2 * y + y * z2; // s3: mu_112 + mu_233
      case 12: return x2 * z + y2 * z; // s3: mu_113 + mu_223 (printed garbled)
      case 13: return x * y2 - x * z2; // s4
      case 14: return x2 * y - y * z2; // s4
      case 15: return x2 * z - y2 * z; // s4 (printed garbled)
      case 16: return x2 * y2 - 2 * x2 * z2 + y2 * z2;  // 4th order
      case 17: return x2 * y2 + x2 * z2 - 2 * y2 * z2;  // 4th order
      case 18: return x2 * y2 + x2 * z2 + y2 * z2;      // 4th order
    }
  } else {
    // d'Humieres et al. (2002) orthogonal D3Q19 basis.
    switch (k) {
      case 0: return 1.0;
      case 1: return 19.0 * e2 - 30.0;
      case 2: return 0.5 * (21.0 * e2 * e2 - 53.0 * e2 + 24.0);
      case 3: return x;
      case 4: return (5.0 * e2 - 9.0) * x;
      case 5: return y;
      case 6: return (5.0 * e2 - 9.0) * y;
      case 7: return z;
      case 8: return (5.0 * e2 - 9.0) * z;
      case 9: return 3.0 * x2 - e2;
      case 10: return (3.0 * e2 - 5.0) * (3.0 * x2 - e2);
      case 11: return y2 - z2;
      case 12: return (3.0 * e2 - 5.0) * (y2 - z2);
      case 13: return x * y;
      case 14: return y * z;
      case 15: return x * z;
      case 16: return (y2 - z2) * x;
      case 17: return (z2 - x2) * y;
      case 18: return (x2 - y2) * z;
    }
  }
  return 0.0;
}

struct MrtBasis {
  double M[19 * 19];
  double Minv[19 * 19];
};

const MrtBasis& get_basis(int basis) {
  static MrtBasis b[2];
  static bool ready[2] = {false, false};
  #pragma omp critical(orc_basis)
  {
    if (!ready[basis]) {
      for (int k = 0; k < 19; ++k)
        for (int i = 0; i < 19; ++i) b[basis].M[k * 19 + i] = basis_row(basis, k, E[i]);
      dense_inverse(19, b[basis].M, b[basis].Minv);
      ready[basis] = true;
    }
  }
  return b[basis];
}

// Relaxation rate of each moment row; shear rows get 1/tau_total.
template <typename T>
void mrt_rates(int basis, const double* rates, T s_shear, T* s) {
  for (int k = 0; k < 19; ++k) s[k] = T(0.0);
  if (basis == ORC_BASIS_TABLE1) {
    for (int k = 4; k <= 8; ++k) s[k] = s_shear;  // s1
    s[9] = rates[0];                               // s2
    for (int k = 10; k <= 12; ++k) s[k] = rates[1];  // s3
    for (int k = 13; k <= 15; ++k) s[k] = rates[2];  // s4
    for (int k = 16; k <= 18; ++k) s[k] = rates[3];  // s7 (both 4th-order rows)
  } else {
    s[1] = rates[0];                   // energy
    s[2] = rates[1];                   // energy squared
    s[4] = s[6] = s[8] = rates[2];     // heat flux
    s[9] = s[11] = s[13] = s[14] = s[15] = s_shear;  // viscous stress
    s[10] = s[12] = rates[3];          // 4th-order stress
    s[16] = s[17] = s[18] = rates[4];  // 3rd-order antisymmetric
  }
}

// Eqs. (3)-(5), (16)-(21): strain-rate-dependent total relaxation time.
template <typename T>
T smagorinsky_tau(const T* f, double tau0, double cs, T* Q_out) {
  using std::sqrt;
  T drho = 0.0, u[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    for (int a = 0; a < 3; ++a) u[a] += f[i] * T(E[i][a]);
  }
  T feq[19];
  feq_incomp(19, drho, u, feq);
  T pi2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T p = 0.0;
      for (int i = 0; i < 19; ++i) p += T(E[i][a] * E[i][b]) * (f[i] - feq[i]);
      pi2 += p * p;
    }
  const T Q = sqrt(T(2.0) * pi2);
  if (Q_out) *Q_out = Q;
  return T(0.5) * (T(tau0) + sqrt(T(tau0 * tau0) + T(18.0 * cs * cs) * Q));
}

// Eq. (12), read with the sign of a relaxation: f* = f - M^-1 S (M f - M f_eq).
template <typename T>
void mrt_collide(const T* f, double tau0, double cs, int basis, const double* rates, T* fout,
                 T* tau_out) {
  const MrtBasis& B = get_basis(basis);
  T drho = 0.0, u[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    for (int a = 0; a < 3; ++a) u[a] += f[i] * T(E[i][a]);
  }
  T feq[19];
  feq_incomp(19, drho, u, feq);
  const T tau = smagorinsky_tau(f, tau0, cs, (T*)nullptr);
  if (tau_out) *tau_out = tau;
  T s[19];
  mrt_rates(basis, rates, T(1.0) / tau, s);
  T d[19];
  for (int k = 0; k < 19; ++k) {
    T m = 0.0, meq = 0.0;
    for (int i = 0; i < 19; ++i) {
      m += T(B.M[k * 19 + i]) * f[i];
      meq += T(B.M[k * 19 + i]) * feq[i];
    }
    d[k] = s[k] * (m - meq);
  }
  for (int i = 0; i < 19; ++i) {
    T c = 0.0;
    for (int k = 0; k < 19; ++k) c += T(B.Minv[i * 19 + k]) * d[k];
    fout[i] = f[i] - c;
  }
}

// Eqs. (14)-(15) per unit mass: kappa_abc = (1/rho) sum_i F_i (e_x-u_x)^a
// (e_y-u_y)^b (e_z-u_z)^c, a,b,c in {0,1,2}; index 9a + 3b + c.
template <typename T>
void central_moments(const T* F, T* rho_out, T* u, T* kappa) {
  T rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 27; ++i) {
    rho += F[i];
    for (int a = 0; a < 3; ++a) j[a] += F[i] * T(E[i][a]);
  }
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        T s = 0.0;
        for (int i = 0; i < 27; ++i)
          s += F[i] * ipow(T(E[i][0]) - u[0], a) * ipow(T(E[i][1]) - u[1], b) *
               ipow(T(E[i][2]) - u[2], c);
        kappa[9 * a + 3 * b + c] = s / rho;
      }
  *rho_out = rho;
}

// FCLB collision (Section 2, Table 1 groups applied to central moments,
// Table 2 equilibria, all rates except the shear rate equal to 1). With
// gaussian set, the cascaded scheme before the factorization (the CLB the
// paper starts from, Section 2): the fourth- and sixth-order central moments
// relax to those of the Gaussian whose variance is the squared speed of
// sound (1/9, 0 and 1/27 per unit mass) instead of to products of the
// relaxed second order.
template <typename T>
void fclb_collide(const T* f, double omega, T* fout, bool gaussian = false) {
  T F[27];
  for (int i = 0; i < 27; ++i) F[i] = T(weight(27, i)) + f[i];
  T rho, u[3], k[27];
  central_moments(F, &rho, u, k);
  auto K = [&](int a, int b, int c) { return k[9 * a + 3 * b + c]; };
  T ks[27];
  for (int m = 0; m < 27; ++m) ks[m] = 0.0;  // orders 1, 3, 5 relax to 0
  ks[0] = 1.0;
  const T T3 = K(2, 0, 0) + K(0, 2, 0) + K(0, 0, 2);
  const T third = 1.0 / 3.0, omc = 1.0 - omega;
  // second order: trace to 1 (rate s2 = 1), deviatoric part at omega
  const T k200 = third + omc * (K(2, 0, 0) - T3 * third);
  const T k020 = third + omc * (K(0, 2, 0) - T3 * third);
  const T k002 = third + omc * (K(0, 0, 2) - T3 * third);
  const T k110 = omc * K(1, 1, 0);
  const T k101 = omc * K(1, 0, 1);
  const T k011 = omc * K(0, 1, 1);
  ks[9 * 2 + 0 + 0] = k200;
  ks[0 + 3 * 2 + 0] = k020;
  ks[0 + 0 + 2] = k002;
  ks[9 + 3 + 0] = k110;
  ks[9 + 0 + 1] = k101;
  ks[0 + 3 + 1] = k011;
  // fourth order: factorized equilibria from the relaxed second order
  ks[9 * 2 + 3 * 2 + 0] = k200 * k020;
  ks[9 * 2 + 0 + 2] = k200 * k002;
  ks[0 + 3 * 2 + 2] = k020 * k002;
  ks[9 * 2 + 3 + 1] = k200 * k011;
  ks[9 + 3 * 2 + 1] = k020 * k101;
  ks[9 + 3 + 2] = k002 * k110;
  // sixth order
  ks[9 * 2 + 3 * 2 + 2] = k200 * k020 * k002;
  if (gaussian) {
    ks[9 * 2 + 3 * 2 + 0] = ks[9 * 2 + 0 + 2] = ks[0 + 3 * 2 + 2] = 1.0 / 9.0;
    ks[9 * 2 + 3 + 1] = ks[9 + 3 * 2 + 1] = ks[9 + 3 + 2] = 0.0;
    ks[9 * 2 + 3 * 2 + 2] = 1.0 / 27.0;
  }
  // back to populations: sum_i F*_i prod_a (e_ia - u_a)^{n_a} = rho kappa*
  T A[27 * 27], b[27];
  for (int a = 0; a < 3; ++a)
    for (int bb = 0; bb < 3; ++bb)
      for (int c = 0; c < 3; ++c) {
        const int m = 9 * a + 3 * bb + c;
        for (int i = 0; i < 27; ++i)
          A[m * 27 + i] = ipow(T(E[i][0]) - u[0], a) * ipow(T(E[i][1]) - u[1], bb) *
                          ipow(T(E[i][2]) - u[2], c);
        b[m] = rho * ks[m];
      }
  dense_solve(27, A, b);
  for (int i = 0; i < 27; ++i) fout[i] = b[i] - T(weight(27, i));
}

void collide_node(const orc_params* p, const double* f, double* fout) {
  const double tau0 = 3.0 * p->nu + 0.5;
  if (p->model == ORC_MRT19)
    mrt_collide(f, tau0, p->cs_smag, p->mrt_basis, p->rates, fout, (double*)nullptr);
  else
    fclb_collide(f, 1.0 / tau0, fout, p->model == ORC_CLB27);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): one output for a state.
uint64_t splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Uniform [0,1) draw for inlet node (a, b), component c at time step t.
double inlet_uniform(uint64_t seed, int64_t t, int a, int b, int c) {
  const uint64_t key = seed ^ (((uint64_t)t << 32) | ((uint64_t)c << 28) |
                               ((uint64_t)b << 14) | (uint64_t)a);
  return (double)(splitmix64(key) >> 11) * (1.0 / 9007199254740992.0);
}

// Inlet velocity of the node at local (x,y,z) on face `face` at step t.
void inlet_velocity(const orc_params* p, int face, int x, int y, int z,
                    int64_t t, double u[3]) {
  const int g[3] = {x + p->origin[0], y + p->origin[1], z + p->origin[2]};
  const int axis = face / 2;
  const int ta = (axis == 0) ? 1 : 0;
  const int tb = (axis == 2) ? 1 : 2;
  const int a = g[ta], b = g[tb];
  const long idx = (long)b * p->inlet_na + a;
  const long nface = (long)p->inlet_na * p->inlet_nb;
  for (int c = 0; c < 3; ++c) {
    u[c] = p->inlet_u[c * nface + idx];
    if (p->inlet_mask && p->inlet_mask[idx])
      u[c] += p->inlet_amp * (2.0 * inlet_uniform(p->seed, t, a, b, c) - 1.0);
  }
}

inline long node_index(const orc_params* p, int x, int y, int z) {
  return ((long)z * p->ny + y) * p->nx + x;
}

// Where the pull-streamed population i of node (x,y,z) comes from:
//  * periodic faces wrap;
//  * a source beyond a WALL face: halfway bounce-back with the wall's
//    velocity, f_i = f*_opp(i)(x) + 6 w_i (e_i . u_w);
//  * beyond an INLET face: the same with the inlet velocity at the node;
//  * beyond OUTFLOW faces only: the post-collision value of the nearest
//    boundary node (a ghost layer copying the last plane);
//  * a solid node inside the domain: bounce-back off a wall at rest. With
//    no link distance (or q = 1/2) halfway, f_i = f*_opp(i)(x), the same
//    rule as a WALL face with u_w = 0; otherwise Bouzidi's linear
//    interpolation along the link (k = opp(i), the direction from x to the
//    wall, q its distance fraction):
//      q < 1/2:  f_i(x) = 2q f*_k(x) + (1 - 2q) f*_k(x - e_k)
//      q >= 1/2: f_i(x) = f*_k(x) / (2q) + (2q - 1)/(2q) f*_i(x)
//    where x - e_k must be a fluid node inside the domain (periodic axes
//    wrap); where it is not, the halfway rule stays;
//  * beyond FREESLIP faces (and possibly OUTFLOW faces): halfway specular
//    reflection, f_i = f*_k(s) with k = i mirrored across every crossed
//    FREESLIP face (its normal component reversed) and s = x - e_i with
//    every crossed coordinate kept (the node the mirrored population left);
//  * beyond a PRESSURE face (fixed pressure): anti-bounce-back, f_i =
//    -f*_opp(i)(x) + feq_i + feq_opp(i), the model's equilibrium at the
//    face's density and the node's own velocity (of its state at t).
// When a source lies beyond several faces, WALL wins over INLET over
// PRESSURE over FREESLIP over OUTFLOW.
enum { SRC_NORMAL = 0, SRC_WALL = 1, SRC_INLET = 2, SRC_OUTFLOW = 3, SRC_SOLID = 4,
       SRC_FREESLIP = 5, SRC_PRESSURE = 6 };
struct Source {
  int kind;
  long node;  // source node (NORMAL/OUTFLOW/FREESLIP) or the node itself
  int face;   // crossed WALL/INLET face; the mirrored direction (FREESLIP)
};

// Index of the velocity (ex, ey, ez) in the table (-1 if absent).
int velocity_index(int Q, int ex, int ey, int ez) {
  for (int k = 0; k < Q; ++k)
    if (E[k][0] == ex && E[k][1] == ey && E[k][2] == ez) return k;
  return -1;
}

Source classify(const orc_params* p, int i, int x, int y, int z) {
  const int n[3] = {p->nx, p->ny, p->nz};
  int s[3] = {x - E[i][0], y - E[i][1], z - E[i][2]};
  int crossed[6] = {0, 0, 0, 0, 0, 0};
  bool any = false;
  for (int d = 0; d < 3; ++d) {
    int face = -1;
    if (s[d] < 0) face = 2 * d;
    else if (s[d] >= n[d]) face = 2 * d + 1;
    if (face < 0) continue;
    if (p->face_type[face] == ORC_PERIODIC) {
      s[d] = (s[d] + n[d]) % n[d];
    } else {
      crossed[face] = 1;
      any = true;
    }
  }
  if (!any) {
    const long src = node_index(p, s[0], s[1], s[2]);
    if (p->solid && p->solid[src]) return {SRC_SOLID, node_index(p, x, y, z), -1};
    return {SRC_NORMAL, src, -1};
  }
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_WALL)
      return {SRC_WALL, node_index(p, x, y, z), face};
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_INLET)
      return {SRC_INLET, node_index(p, x, y, z), face};
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_PRESSURE)
      return {SRC_PRESSURE, node_index(p, x, y, z), face};
  for (int d = 0; d < 3; ++d) {
    if (s[d] < 0) s[d] = 0;
    if (s[d] >= n[d]) s[d] = n[d] - 1;
  }
  int e[3] = {E[i][0], E[i][1], E[i][2]};
  bool mirrored = false;
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_FREESLIP) {
      e[face / 2] = -e[face / 2];
      mirrored = true;
    }
  if (mirrored)
    return {SRC_FREESLIP, node_index(p, s[0], s[1], s[2]),
            velocity_index(nq(p->model), e[0], e[1], e[2])};
  return {SRC_OUTFLOW, node_index(p, s[0], s[1], s[2]), -1};
}

// Pull-streamed value of population i at node (x,y,z) at t+1 from the
// post-collision field fpost of step t (rules in classify()).
double pull(const orc_params* p, const double* fpost, int Q, int i, int x, int y, int z,
            int64_t t) {
  const long N = (long)p->nx * p->ny * p->nz;
  const Source src = classify(p, i, x, y, z);
  if (src.kind == SRC_NORMAL || src.kind == SRC_OUTFLOW) return fpost[i * N + src.node];
  if (src.kind == SRC_FREESLIP) return fpost[src.face * N + src.node];
  const int io = opposite(Q, i);
  if (src.kind == SRC_SOLID) {
    const double fk = fpost[io * N + src.node];
    const double q = p->link_q ? p->link_q[io * N + src.node] : 0.0;
    if (!(q > 0.0 && q <= 1.0) || q == 0.5) return fk;
    // the fluid node behind x along the link (x - e_k = x + e_i)
    const int n[3] = {p->nx, p->ny, p->nz};
    int b[3] = {x + E[i][0], y + E[i][1], z + E[i][2]};
    for (int d = 0; d < 3; ++d) {
      if (b[d] >= 0 && b[d] < n[d]) continue;
      const int face = b[d] < 0 ? 2 * d : 2 * d + 1;
      if (p->face_type[face] != ORC_PERIODIC) return fk;
      b[d] = (b[d] + n[d]) % n[d];
    }
    const long behind = node_index(p, b[0], b[1], b[2]);
    if (p->solid && p->solid[behind]) return fk;
    if (q < 0.5) return 2.0 * q * fk + (1.0 - 2.0 * q) * fpost[io * N + behind];
    return fk / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fpost[i * N + src.node];
  }
  if (src.kind == SRC_PRESSURE) {
    // the node's velocity: momentum and mass are those of its state at t
    double d = 0.0, j[3] = {0, 0, 0};
    for (int k = 0; k < Q; ++k) {
      const double v = fpost[k * N + src.node];
      d += v;
      for (int a = 0; a < 3; ++a) j[a] += v * E[k][a];
    }
    const double rho = (p->model == ORC_MRT19) ? 1.0 : 1.0 + d;
    const double ub[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double drho = p->face_drho[src.face];
    double feq[27];
    if (p->model == ORC_MRT19) {
      feq_incomp(19, drho, ub, feq);
    } else {
      for (int k = 0; k < 27; ++k)
        feq[k] = (1.0 + drho) * phi(E[k][0], ub[0]) * phi(E[k][1], ub[1]) * phi(E[k][2], ub[2]) -
                 weight(27, k);
    }
    return -fpost[io * N + src.node] + feq[i] + feq[io];
  }
  double u[3];
  if (src.kind == SRC_WALL) {
    for (int c = 0; c < 3; ++c) u[c] = p->face_u[src.face][c];
  } else {
    inlet_velocity(p, src.face, x, y, z, t, u);
  }
  const double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
  return fpost[io * N + src.node] + 6.0 * weight(Q, i) * eu;
}

// Exact Jacobian-vector product of the FCLB or MRT-LES collision of one node,
// by forward-mode dual numbers through the same code as the collision (for
// MRT-LES with the strain-dependent relaxation time of Eqs. (16)-(21); at zero
// strain the derivative of the strain magnitude is taken as 0).
void collide_jvp(const orc_params* p, const double* f, const double* v, double* out) {
  const double tau0 = 3.0 * p->nu + 0.5;
  const int Q = nq(p->model);
  Dual a[27], b[27];
  for (int i = 0; i < Q; ++i) a[i] = Dual(f[i], v[i]);
  if (p->model == ORC_MRT19)
    mrt_collide(a, tau0, p->cs_smag, p->mrt_basis, p->rates, b, (Dual*)nullptr);
  else
    fclb_collide(a, 1.0 / tau0, b);
  for (int i = 0; i < Q; ++i) out[i] = b[i].d;
}

}  // namespace

extern "C" {

// OpenMP team size of the oracle's parallel loops (timing only: the
// results do not depend on it, every loop writes disjoint entries).
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads() { return omp_get_max_threads(); }

int orc_stencil(int Q, int* e, double* w, int* opp) {
  if (Q != 19 && Q != 27) return -1;
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < 3; ++a) e[3 * i + a] = E[i][a];
    w[i] = weight(Q, i);
    opp[i] = opposite(Q, i);
  }
  return 0;
}

void orc_feq_incomp(int Q, double drho, const double* u, double* feq) {
  feq_incomp(Q, drho, u, feq);
}

// Full (not deviation) D3Q27 product equilibrium rho prod_a phi(e_ia, u_a).
void orc_feq_product(double rho, const double* u, double* F) {
  for (int i = 0; i < 27; ++i)
    F[i] = rho * phi(E[i][0], u[0]) * phi(E[i][1], u[1]) * phi(E[i][2], u[2]);
}

void orc_mrt_basis(int basis, double* M) {
  const MrtBasis& B = get_basis(basis);
  std::memcpy(M, B.M, sizeof(B.M));
}

double orc_smagorinsky_tau(const double* f19, double tau0, double cs, double* Q) {
  return smagorinsky_tau(f19, tau0, cs, Q);
}

void orc_mrt_collide(const double* f, double tau0, double cs, int basis,
                     const double* rates, double* fout, double* tau_out) {
  mrt_collide(f, tau0, cs, basis, rates, fout, tau_out);
}

void orc_central_moments(const double* F, double* rho, double* u, double* kappa) {
  central_moments(F, rho, u, kappa);
}

void orc_clb_collide(const double* f, double omega, double* fout) {
  fclb_collide(f, omega, fout, true);
}

void orc_fclb_collide(const double* f, double omega, double* fout) {
  fclb_collide(f, omega, fout);
}

uint64_t orc_splitmix64(uint64_t state) { return splitmix64(state); }

double orc_inlet_uniform(uint64_t seed, int64_t t, int a, int b, int c) {
  return inlet_uniform(seed, t, a, b, c);
}

// Collide every node of a lattice (no streaming): populations [Q][N].
void orc_collide_lattice(const orc_params* p, const double* f, double* fout) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double a[27], b[27];
    for (int i = 0; i < Q; ++i) a[i] = f[i * N + n];
    collide_node(p, a, b);
    for (int i = 0; i < Q; ++i) fout[i * N + n] = b[i];
  }
}

// Advance the lattice state f ([Q][nz][ny][nx], pre-collision deviations at
// step t0) by nsteps collide-and-stream updates, in place.
int orc_run(const orc_params* p, double* f, int64_t t0, int64_t nsteps) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  std::vector<double> post((size_t)Q * N);
  for (int64_t t = t0; t < t0 + nsteps; ++t) {
    orc_collide_lattice(p, f, post.data());
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const long self = node_index(p, x, y, z);
          if (p->solid && p->solid[self]) continue;  // solid nodes are not updated
          for (int i = 0; i < Q; ++i)
            f[i * N + self] = pull(p, post.data(), Q, i, x, y, z, t);
        }
  }
  return 0;
}

// Eqs. (3)-(5) (MRT, rho0 = 1) or (6)-(8) (FCLB, rho = 1 + sum f).
void orc_macroscopic(const orc_params* p, const double* f, double* drho, double* u) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double d = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double v = f[i * N + n];
      d += v;
      for (int a = 0; a < 3; ++a) j[a] += v * E[i][a];
    }
    const double rho = (p->model == ORC_MRT19) ? 1.0 : 1.0 + d;
    drho[n] = d;
    for (int a = 0; a < 3; ++a) u[a * N + n] = j[a] / rho;
  }
}

// Equilibrium populations of the model for given (drho, u) fields:
// MRT: Eq. (2); FCLB: the product equilibrium whose central moments are the
// Table 2 equilibria. Output deviations f = F - w.
void orc_init_equilibrium(const orc_params* p, const double* drho, const double* u,
                          double* f) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    const double uu[3] = {u[n], u[N + n], u[2 * N + n]};
    double g[27];
    if (p->model == ORC_MRT19) {
      feq_incomp(19, drho[n], uu, g);
    } else {
      for (int i = 0; i < 27; ++i)
        g[i] = (1.0 + drho[n]) * phi(E[i][0], uu[0]) * phi(E[i][1], uu[1]) *
                   phi(E[i][2], uu[2]) - weight(27, i);
    }
    for (int i = 0; i < Q; ++i) f[i * N + n] = g[i];
  }
}

// Sums over the lattice: mass deviation, momentum (3), kinetic energy
// (|j|^2 / (2 rho), rho = 1 for the incompressible model).
void orc_reduce(const orc_params* p, const double* f, double* out) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  double s[5] = {0, 0, 0, 0, 0};
  for (long n = 0; n < N; ++n) {
    double d = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double v = f[i * N + n];
      d += v;
      for (int a = 0; a < 3; ++a) j[a] += v * E[i][a];
    }
    const double rho = (p->model == ORC_MRT19) ? 1.0 : 1.0 + d;
    s[0] += d;
    for (int a = 0; a < 3; ++a) s[1 + a] += j[a];
    s[4] += 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
  }
  for (int k = 0; k < 5; ++k) out[k] = s[k];
}

}  // extern "C"

// ===========================================================================
// Nested time refinement on a hierarchical block grid (Section 1: block grid
// with a nested time step and Yu et al.'s interpolation and rescaling of the
// non-equilibrium part; Section 3: refinement levels, constant CFL number).
// The paper cites the interface method and prints no formulas; the readings
// used here are:
//  * Levels l = 0 .. L-1. Level l has spacing and time step 2^-l of level 0
//    (the velocity scale, hence the CFL number, is the same on every level),
//    lattice viscosity 2^l nu_0 (tau_l - 1/2 = 2^l (tau_0 - 1/2)); the
//    Smagorinsky constant acts in each level's own lattice units.
//  * A map over the level-0 blocks (B^3 nodes) names the finest level of
//    each block; R_l is the union of the blocks whose entry is >= l.
//  * Cell-centred 2:1 nesting: level-(l+1) node j lies at level-l coordinate
//    j/2 - 1/4 (node i's cell holds the children 2i, 2i+1 on each axis), so
//    the halfway walls and faces of all levels coincide.
//  * Every level stores post-collision populations; a level step pulls and
//    collides.
//  * Level-(l+1) ghost nodes (the layer just outside R_{l+1}) receive
//    level-l post-collision values interpolated in space (tensor 4-point
//    cubic Lagrange; windows kept inside non-periodic domains) and in time
//    (three-point quadratic over the level-l states at t-1, t, t+1 for the
//    half step, weights -1/8, 3/4, 3/8; linear for the first step after a
//    state change, when t-1 is unknown), then rescaled.
//  * Covered level-l nodes (inside R_{l+1}, read by no ghost stencil)
//    receive the mean of their 8 children, rescaled back, once the two
//    level-(l+1) substeps are done.
//  * Rescaling of the non-equilibrium part from a parent level c to its
//    child f (Chapman-Enskog: the post-collision non-equilibrium of a moment
//    relaxed at 1/tau scales as (tau - 1) dt): FCLB/CLB one ratio
//    r = (tau_f - 1) / (2 (tau_c - 1)); MRT per moment group with tau = 1/s
//    (non-shear rates are the same on both levels: r = 1/2, and 0 where the
//    rate is 1, whose post-collision non-equilibrium vanishes), the shear
//    group with the total relaxation times of Eq. (20): tau_c,tot recovered
//    from the post-collision traceless stress of the interpolated state (the
//    stress taken traceless before the collision), tau_f,tot = tau0_f +
//    (tau_c,tot - tau0_c) / 2 (the eddy viscosity halves in fine lattice
//    units). Back from f to c: the inverse ratios, tau_c,tot = tau0_c +
//    2 (tau_f,tot - tau0_f).
// Every level is held over its whole domain here (plain, not memory-lean).
// ===========================================================================

namespace {

enum { T_UNUSED = 0, T_FLUID = 1, T_BAND = 2, T_COVERED = 3, T_GHOST = 4, T_SOLID = 5 };

struct MLevel {
  orc_params p;                   // this level's lattice over its whole domain
  int n[3];
  long N;
  std::vector<uint8_t> type;      // [N]
  std::vector<double> f, g;       // post-collision state and a work array [Q][N]
  std::vector<long> ghosts;       // node indices of the ghost layer (l >= 1)
  std::vector<double> G[3];       // parent values at the ghosts at t-1, t, t+1
  bool have_cur = false, have_prev = false;
  std::vector<uint8_t> solid;
  std::vector<double> link_q, inlet_u;
  std::vector<uint8_t> inlet_mask;
  int box_lo[3], box_hi[3];       // bounding box of the non-unused nodes
  long bad_pull = 0;              // pulls from unused nodes (geometry error)
};

struct MLRefine {
  int L, B, Q, nb[3];
  std::vector<uint8_t> map;
  std::vector<MLevel> lev;
};

int block_level(const MLRefine& R, int bx, int by, int bz) {
  return R.map[((long)bz * R.nb[1] + by) * R.nb[0] + bx];
}

// Is node x of level l inside R_m (m <= l)?
bool in_region(const MLRefine& R, int l, int m, const int x[3]) {
  const MLevel& V = R.lev[l];
  int b[3];
  for (int d = 0; d < 3; ++d) {
    if (x[d] < 0 || x[d] >= V.n[d]) return false;
    b[d] = x[d] / (R.B << l);
  }
  return block_level(R, b[0], b[1], b[2]) >= m;
}

long lidx(const MLevel& V, const int x[3]) {
  return ((long)x[2] * V.n[1] + x[1]) * V.n[0] + x[0];
}

void lcoords(const MLevel& V, long k, int x[3]) {
  x[0] = (int)(k % V.n[0]);
  x[1] = (int)((k / V.n[0]) % V.n[1]);
  x[2] = (int)(k / ((long)V.n[0] * V.n[1]));
}

// Neighbour of x by offset d inside the level's domain (periodic axes wrap);
// false beyond a non-periodic face.
bool neighbour(const MLevel& V, const int x[3], const int d[3], int y[3]) {
  for (int a = 0; a < 3; ++a) {
    y[a] = x[a] + d[a];
    if (y[a] >= 0 && y[a] < V.n[a]) continue;
    if (V.p.face_type[2 * a] != ORC_PERIODIC) return false;
    y[a] = (y[a] + V.n[a]) % V.n[a];
  }
  return true;
}

// 4-point Lagrange weights at position p on nodes s..s+3.
void lagrange4(double p, int s, double w[4]) {
  for (int a = 0; a < 4; ++a) {
    double v = 1.0;
    for (int b = 0; b < 4; ++b)
      if (b != a) v *= (p - (s + b)) / (double)(a - b);
    w[a] = v;
  }
}

// Level-l window of the cubic interpolant at child coordinate j: nodes
// s..s+3 (wrapped if periodic) and Lagrange weights at p = j/2 - 1/4.
void child_stencil(const MLevel& parent, int d, int j, int idx[4], double w[4]) {
  const double p = 0.5 * j - 0.25;
  int s = (int)std::floor(p) - 1;
  const int n = parent.n[d];
  const bool periodic = parent.p.face_type[2 * d] == ORC_PERIODIC;
  if (!periodic) s = std::max(0, std::min(s, n - 4));
  lagrange4(p, s, w);
  for (int a = 0; a < 4; ++a) idx[a] = periodic ? (((s + a) % n) + n) % n : s + a;
}

// Raw spatial interpolation of the parent state at every ghost of level l.
void interp_ghosts(const MLRefine& R, int l, const std::vector<double>& fp,
                   std::vector<double>& out) {
  const MLevel& V = R.lev[l];
  const MLevel& P = R.lev[l - 1];
  const long ng = (long)V.ghosts.size();
  out.assign((size_t)R.Q * ng, 0.0);
  #pragma omp parallel for schedule(static)
  for (long gi = 0; gi < ng; ++gi) {
    int x[3];
    lcoords(V, V.ghosts[gi], x);
    int idx[3][4];
    double w[3][4];
    for (int d = 0; d < 3; ++d) child_stencil(P, d, x[d], idx[d], w[d]);
    for (int q = 0; q < R.Q; ++q) {
      double s = 0.0;
      for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
          for (int a = 0; a < 4; ++a) {
            const int y[3] = {idx[0][a], idx[1][b], idx[2][c]};
            s += w[0][a] * w[1][b] * w[2][c] * fp[(size_t)q * P.N + lidx(P, y)];
          }
      out[(size_t)q * ng + gi] = s;
    }
  }
}

// The model's equilibrium (deviation form) for the moments of f.
void equilibrium_of(int model, const double* f, double* feq) {
  const int Q = nq(model);
  double d = 0.0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    for (int a = 0; a < 3; ++a) j[a] += f[i] * E[i][a];
  }
  if (model == ORC_MRT19) {
    feq_incomp(19, d, j, feq);
  } else {
    const double rho = 1.0 + d;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    for (int i = 0; i < 27; ++i)
      feq[i] = rho * phi(E[i][0], u[0]) * phi(E[i][1], u[1]) * phi(E[i][2], u[2]) -
               weight(27, i);
  }
}

bool mrt_shear_row(int basis, int k) {
  if (basis == ORC_BASIS_TABLE1) return k >= 4 && k <= 8;
  return k == 9 || k == 11 || k == 13 || k == 14 || k == 15;
}

bool mrt_conserved_row(int basis, int k) {
  if (basis == ORC_BASIS_TABLE1) return k <= 3;
  return k == 0 || k == 3 || k == 5 || k == 7;
}

// Total relaxation time of a post-collision state of the MRT-LES model:
// the traceless stress T of its non-equilibrium part gives Qp = sqrt(2 T:T)
// = Q |1 - 1/tau| with Q the pre-collision value of Eq. (21); with Eq. (20)
// (tau^2 - tau0 tau = 9/2 C_S^2 Q) this is the root that tends to tau0 as
// Qp -> 0: tau = (1 + tau0 -+ sqrt((1 - tau0)^2 -+ 18 C_S^2 Qp)) / 2 (upper
// signs for tau0 < 1; a negative radicand, out of reach of a collision's
// output, is clamped to 0).
double tau_from_post(const double* neq, double tau0, double cs) {
  double P[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int i = 0; i < 19; ++i) s += E[i][a] * E[i][b] * neq[i];
      P[a][b] = s;
    }
  const double tr = (P[0][0] + P[1][1] + P[2][2]) / 3.0;
  double t2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double v = P[a][b] - (a == b ? tr : 0.0);
      t2 += v * v;
    }
  const double Qp = std::sqrt(2.0 * t2);
  const double k = 18.0 * cs * cs * Qp;
  if (tau0 < 1.0) {
    const double rad = std::max(0.0, (1.0 - tau0) * (1.0 - tau0) - k);
    return 0.5 * (1.0 + tau0 - std::sqrt(rad));
  }
  return 0.5 * (1.0 + tau0 + std::sqrt((tau0 - 1.0) * (tau0 - 1.0) + k));
}

// Non-equilibrium rescaling of one node between a parent level c and its
// child f: dir > 0 maps a parent state to the child, dir < 0 back. Returns
// the shear ratio used (child over parent).
double rescale_node(const orc_params* pc, const orc_params* pf, const double* in, int dir,
                    double* out) {
  const int model = pc->model;
  const int Q = nq(model);
  double feq[27], neq[27];
  equilibrium_of(model, in, feq);
  for (int i = 0; i < Q; ++i) neq[i] = in[i] - feq[i];
  const double t0c = 3.0 * pc->nu + 0.5, t0f = 3.0 * pf->nu + 0.5;
  if (model != ORC_MRT19) {
    const double r = (t0f - 1.0) / (2.0 * (t0c - 1.0));
    const double s = dir > 0 ? r : 1.0 / r;
    for (int i = 0; i < Q; ++i) out[i] = feq[i] + s * neq[i];
    return r;
  }
  double tc, tf;
  if (dir > 0) {
    tc = tau_from_post(neq, t0c, pc->cs_smag);
    tf = t0f + 0.5 * (tc - t0c);
  } else {
    tf = tau_from_post(neq, t0f, pf->cs_smag);
    tc = t0c + 2.0 * (tf - t0f);
  }
  const double r_shear = (tf - 1.0) / (2.0 * (tc - 1.0));
  const MrtBasis& Bm = get_basis(pc->mrt_basis);
  double s[19];
  mrt_rates(pc->mrt_basis, pc->rates, 0.0, s);
  double m[19];
  for (int k = 0; k < 19; ++k) {
    double v = 0.0;
    for (int i = 0; i < 19; ++i) v += Bm.M[k * 19 + i] * neq[i];
    double r;
    if (mrt_conserved_row(pc->mrt_basis, k)) r = 0.0;  // no non-equilibrium part
    else if (mrt_shear_row(pc->mrt_basis, k)) r = dir > 0 ? r_shear : 1.0 / r_shear;
    else if (s[k] == 1.0) r = 0.0;                      // relaxed to equilibrium
    else r = dir > 0 ? 0.5 : 2.0;                       // same rate on both levels
    m[k] = r * v;
  }
  for (int i = 0; i < 19; ++i) {
    double v = 0.0;
    for (int k = 0; k < 19; ++k) v += Bm.Minv[i * 19 + k] * m[k];
    out[i] = feq[i] + v;
  }
  return r_shear;
}

// Ghosts of level l := rescale(c0 G[0] + c1 G[1] + c2 G[2]).
void fill_ghosts(MLRefine& R, int l, double c0, double c1, double c2) {
  MLevel& V = R.lev[l];
  const MLevel& P = R.lev[l - 1];
  const long ng = (long)V.ghosts.size();
  #pragma omp parallel for schedule(static)
  for (long gi = 0; gi < ng; ++gi) {
    double a[27], b[27];
    for (int q = 0; q < R.Q; ++q) {
      const size_t k = (size_t)q * ng + gi;
      a[q] = c1 * V.G[1][k] + c2 * V.G[2][k];
      if (c0 != 0.0) a[q] += c0 * V.G[0][k];
    }
    rescale_node(&P.p, &V.p, a, +1, b);
    for (int q = 0; q < R.Q; ++q) V.f[(size_t)q * V.N + V.ghosts[gi]] = b[q];
  }
}

// Time weights of the parent states at t-1, t, t+1 for the child's half
// step t + 1/2: three-point quadratic Lagrange (-1/8, 3/4, 3/8), or linear
// (0, 1/2, 1/2) while the state at t-1 is unknown.
void half_step_weights(bool have_prev, double w[3]) {
  w[0] = have_prev ? -0.125 : 0.0;
  w[1] = have_prev ? 0.75 : 0.5;
  w[2] = have_prev ? 0.375 : 0.5;
}

// Covered nodes of level l := the rescaled mean of their 8 children.
void inject(MLRefine& R, int l) {
  MLevel& V = R.lev[l];
  const MLevel& C = R.lev[l + 1];
  #pragma omp parallel for schedule(static)
  for (long k = 0; k < V.N; ++k) {
    if (V.type[k] != T_COVERED) continue;
    int x[3];
    lcoords(V, k, x);
    double a[27], b[27];
    for (int q = 0; q < R.Q; ++q) a[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int y[3] = {2 * x[0] + (c & 1), 2 * x[1] + ((c >> 1) & 1), 2 * x[2] + (c >> 2)};
      const long kc = lidx(C, y);
      for (int q = 0; q < R.Q; ++q) a[q] += C.f[(size_t)q * C.N + kc];
    }
    for (int q = 0; q < R.Q; ++q) a[q] *= 0.125;
    rescale_node(&V.p, &C.p, a, -1, b);
    for (int q = 0; q < R.Q; ++q) V.f[(size_t)q * V.N + k] = b[q];
  }
}

// One step of level l at its step index t: f := C(pull(f)) on fluid and
// band nodes; the others keep their values.
void level_step(MLevel& V, int Q, int64_t t) {
  long bad = 0;
  #pragma omp parallel for schedule(static) reduction(+ : bad)
  for (long k = 0; k < V.N; ++k) {
    const uint8_t ty = V.type[k];
    if (ty != T_FLUID && ty != T_BAND) {
      for (int q = 0; q < Q; ++q) V.g[(size_t)q * V.N + k] = V.f[(size_t)q * V.N + k];
      continue;
    }
    int x[3];
    lcoords(V, k, x);
    for (int i = 0; i < Q; ++i) {  // every in-domain source must hold a state
      const int d[3] = {-E[i][0], -E[i][1], -E[i][2]};
      int y[3];
      if (neighbour(V, x, d, y) && V.type[lidx(V, y)] == T_UNUSED) ++bad;
    }
    double a[27], b[27];
    for (int i = 0; i < Q; ++i) a[i] = pull(&V.p, V.f.data(), Q, i, x[0], x[1], x[2], t);
    collide_node(&V.p, a, b);
    for (int q = 0; q < Q; ++q) V.g[(size_t)q * V.N + k] = b[q];
  }
  V.bad_pull += bad;
  V.f.swap(V.g);
}

// Advance level l by one of its steps (index t); recursively the finer
// levels by two steps each.
void advance(MLRefine& R, int l, int64_t t) {
  MLevel& V = R.lev[l];
  const bool child = l + 1 < R.L;
  if (child && !R.lev[l + 1].have_cur) {
    interp_ghosts(R, l + 1, V.f, R.lev[l + 1].G[1]);
    R.lev[l + 1].have_cur = true;
    R.lev[l + 1].have_prev = false;
  }
  level_step(V, R.Q, t);
  if (!child) return;
  MLevel& C = R.lev[l + 1];
  interp_ghosts(R, l + 1, V.f, C.G[2]);
  fill_ghosts(R, l + 1, 0.0, 1.0, 0.0);
  advance(R, l + 1, 2 * t);
  double w[3];
  half_step_weights(C.have_prev, w);
  fill_ghosts(R, l + 1, w[0], w[1], w[2]);
  advance(R, l + 1, 2 * t + 1);
  inject(R, l);
  C.G[0].swap(C.G[1]);
  C.G[1].swap(C.G[2]);
  C.have_prev = true;
}

bool build_levels(MLRefine& R, const orc_params* coarse, const double* const* inlet_u,
                  const uint8_t* const* inlet_mask, const uint8_t* const* solid,
                  const double* const* link_q) {
  const int L = R.L, Q = R.Q;
  // nesting: the neighbours of a block at level m >= 2 are at level >= m - 1
  for (int bz = 0; bz < R.nb[2]; ++bz)
    for (int by = 0; by < R.nb[1]; ++by)
      for (int bx = 0; bx < R.nb[0]; ++bx) {
        const int m = block_level(R, bx, by, bz);
        if (m >= L) return false;
        if (m < 2) continue;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int b[3] = {bx + dx, by + dy, bz + dz};
              bool inside = true;
              for (int d = 0; d < 3; ++d) {
                if (b[d] >= 0 && b[d] < R.nb[d]) continue;
                if (coarse->face_type[2 * d] != ORC_PERIODIC) inside = false;
                b[d] = (b[d] + R.nb[d]) % R.nb[d];
              }
              if (inside && block_level(R, b[0], b[1], b[2]) < m - 1) return false;
            }
      }
  // a refined region on a periodic axis spans it or keeps off its ends
  for (int l = 1; l < L; ++l)
    for (int d = 0; d < 3; ++d) {
      if (coarse->face_type[2 * d] != ORC_PERIODIC) continue;
      int lo = R.nb[d], hi = -1;
      for (int bz = 0; bz < R.nb[2]; ++bz)
        for (int by = 0; by < R.nb[1]; ++by)
          for (int bx = 0; bx < R.nb[0]; ++bx)
            if (block_level(R, bx, by, bz) >= l) {
              const int b3[3] = {bx, by, bz};
              lo = std::min(lo, b3[d]);
              hi = std::max(hi, b3[d]);
            }
      if (hi < 0) continue;
      const bool full = lo == 0 && hi == R.nb[d] - 1;
      if (!full && (lo == 0 || hi == R.nb[d] - 1)) return false;
    }
  R.lev.resize(L);
  for (int l = 0; l < L; ++l) {
    MLevel& V = R.lev[l];
    V.p = *coarse;
    V.p.nx = coarse->nx << l;
    V.p.ny = coarse->ny << l;
    V.p.nz = coarse->nz << l;
    V.p.nu = coarse->nu * (double)(1 << l);
    V.p.seed = coarse->seed + (uint64_t)l;
    for (int d = 0; d < 3; ++d) V.p.origin[d] = 0;
    V.n[0] = V.p.nx;
    V.n[1] = V.p.ny;
    V.n[2] = V.p.nz;
    V.N = (long)V.n[0] * V.n[1] * V.n[2];
    for (int face = 0; face < 6; ++face)
      if (coarse->face_type[face] == ORC_INLET) {
        const int d = face / 2;
        V.p.inlet_na = V.n[d == 0 ? 1 : 0];
        V.p.inlet_nb = V.n[d == 2 ? 1 : 2];
        if (l > 0) {
          const long nf = (long)V.p.inlet_na * V.p.inlet_nb;
          if (!inlet_u || !inlet_u[l]) return false;
          V.inlet_u.assign(inlet_u[l], inlet_u[l] + 3 * nf);
          V.p.inlet_u = V.inlet_u.data();
          if (inlet_mask && inlet_mask[l]) {
            V.inlet_mask.assign(inlet_mask[l], inlet_mask[l] + nf);
            V.p.inlet_mask = V.inlet_mask.data();
          } else {
            V.p.inlet_mask = nullptr;
          }
        }
      }
    V.p.solid = nullptr;
    V.p.link_q = nullptr;
    if (solid && solid[l]) {
      V.solid.assign(solid[l], solid[l] + V.N);
      V.p.solid = V.solid.data();
    }
    if (link_q && link_q[l]) {
      V.link_q.assign(link_q[l], link_q[l] + (size_t)Q * V.N);
      V.p.link_q = V.link_q.data();
    }
    const double tau = 3.0 * V.p.nu + 0.5;
    if (L > 1 && std::fabs(tau - 1.0) < 1e-6) return false;
    // node types
    V.type.assign(V.N, T_UNUSED);
    for (long k = 0; k < V.N; ++k) {
      int x[3];
      lcoords(V, k, x);
      if (in_region(R, l, l, x)) {
        V.type[k] = (l + 1 < L && in_region(R, l, l + 1, x)) ? T_COVERED : T_FLUID;
        continue;
      }
      for (int c = 0; c < 27 && V.type[k] == T_UNUSED; ++c) {
        const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
        int y[3];
        if (neighbour(V, x, d, y) && in_region(R, l, l, y)) V.type[k] = T_GHOST;
      }
    }
    V.ghosts.clear();
    if (l > 0)
      for (long k = 0; k < V.N; ++k)
        if (V.type[k] == T_GHOST) V.ghosts.push_back(k);
  }
  // band: parent nodes read by a child's ghost stencils stay parent-updated
  for (int l = 1; l < L; ++l) {
    MLevel& V = R.lev[l];
    MLevel& P = R.lev[l - 1];
    for (long gk : V.ghosts) {
      int x[3];
      lcoords(V, gk, x);
      int idx[3][4];
      double w[3][4];
      for (int d = 0; d < 3; ++d) child_stencil(P, d, x[d], idx[d], w[d]);
      for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
          for (int a = 0; a < 4; ++a) {
            const int y[3] = {idx[0][a], idx[1][b], idx[2][c]};
            uint8_t& t = P.type[lidx(P, y)];
            if (t == T_COVERED) t = T_BAND;
            if (t != T_FLUID && t != T_BAND) return false;  // stencil off the parent's state
          }
    }
  }
  // solids: off the interface (ghosts, ghost stencils, covered nodes that a
  // parent-updated node pulls from, and their children)
  for (int l = 0; l < L; ++l) {
    MLevel& V = R.lev[l];
    if (V.solid.empty()) continue;
    for (long k = 0; k < V.N; ++k) {
      if (!V.solid[k]) continue;
      const uint8_t t = V.type[k];
      if (t == T_GHOST || t == T_BAND) return false;
      if (t == T_FLUID) V.type[k] = T_SOLID;
      if (t == T_COVERED) V.type[k] = T_SOLID;
    }
  }
  for (int l = 0; l + 1 < L; ++l) {
    MLevel& V = R.lev[l];
    const MLevel& C = R.lev[l + 1];
    for (long k = 0; k < V.N; ++k) {
      if (V.type[k] != T_FLUID && V.type[k] != T_BAND) continue;
      int x[3];
      lcoords(V, k, x);
      for (int i = 1; i < Q; ++i) {
        const int d[3] = {-E[i][0], -E[i][1], -E[i][2]};
        int y[3];
        if (!neighbour(V, x, d, y)) continue;
        const uint8_t t = V.type[lidx(V, y)];
        if (t == T_SOLID && in_region(R, l, l + 1, y)) return false;
        if (t != T_COVERED) continue;
        if (C.solid.empty()) continue;
        for (int c = 0; c < 8; ++c) {
          const int z[3] = {2 * y[0] + (c & 1), 2 * y[1] + ((c >> 1) & 1), 2 * y[2] + (c >> 2)};
          if (C.solid[lidx(C, z)]) return false;
        }
      }
    }
  }
  for (int l = 1; l < L; ++l) {  // children of every stencil or covered read: fluid
    const MLevel& V = R.lev[l];
    if (V.solid.empty()) continue;
    for (long gk : V.ghosts)
      for (int c = 0; c < 27; ++c) {
        int x[3], y[3];
        lcoords(V, gk, x);
        const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
        if (neighbour(V, x, d, y) && V.solid[lidx(V, y)]) return false;
      }
  }
  for (int l = 0; l < L; ++l) {
    MLevel& V = R.lev[l];
    for (int d = 0; d < 3; ++d) {
      V.box_lo[d] = V.n[d];
      V.box_hi[d] = 0;
    }
    for (long k = 0; k < V.N; ++k)
      if (V.type[k] != T_UNUSED) {
        int x[3];
        lcoords(V, k, x);
        for (int d = 0; d < 3; ++d) {
          V.box_lo[d] = std::min(V.box_lo[d], x[d]);
          V.box_hi[d] = std::max(V.box_hi[d], x[d] + 1);
        }
      }
    V.f.assign((size_t)Q * V.N, 0.0);
    V.g.assign((size_t)Q * V.N, 0.0);
  }
  return true;
}

}  // namespace

extern "C" {

// Build the levels. coarse: level-0 lattice parameters (faces, inlet, seed,
// model, viscosity); block: block edge B in level-0 nodes (divides nx, ny,
// nz); nlevels >= 1; map: [nz/B][ny/B][nx/B] finest level of each block (<
// nlevels). Per-level arrays (entry l for level l; the arrays and entries may
// be null): inlet_u [3][nb][na] and inlet_mask [nb][na] at the level's
// resolution (levels >= 1; level 0 takes coarse's own), solid [N_l] and
// link_q [Q][N_l] over the level's whole domain. Returns null on a bad
// configuration (nesting, periodic extent, solids on the interface, tau = 1).
void* orc_mlref_create(const orc_params* coarse, int block, int nlevels, const uint8_t* map,
                       const double* const* inlet_u, const uint8_t* const* inlet_mask,
                       const uint8_t* const* solid, const double* const* link_q) {
  if (block < 2 || nlevels < 1 || nlevels > 8) return nullptr;
  if (coarse->nx % block || coarse->ny % block || coarse->nz % block) return nullptr;
  const int n3[3] = {coarse->nx, coarse->ny, coarse->nz};
  for (int d = 0; d < 3; ++d)  // the one-sided windows need 4 nodes
    if (coarse->face_type[2 * d] != ORC_PERIODIC && n3[d] < 4) return nullptr;
  MLRefine* R = new MLRefine();
  R->L = nlevels;
  R->B = block;
  R->Q = nq(coarse->model);
  R->nb[0] = coarse->nx / block;
  R->nb[1] = coarse->ny / block;
  R->nb[2] = coarse->nz / block;
  R->map.assign(map, map + (long)R->nb[0] * R->nb[1] * R->nb[2]);
  if (!build_levels(*R, coarse, inlet_u, inlet_mask, solid, link_q)) {
    delete R;
    return nullptr;
  }
  return R;
}

void orc_mlref_destroy(void* h) { delete (MLRefine*)h; }

// Level l: domain n[3]; box [lo, hi) of its used nodes; counts = {fluid,
// band, covered, ghost, solid, unused}.
void orc_mlref_info(void* h, int l, int32_t* n, int32_t* box, int64_t* counts) {
  const MLevel& V = ((MLRefine*)h)->lev[l];
  for (int d = 0; d < 3; ++d) {
    n[d] = V.n[d];
    box[d] = V.box_lo[d];
    box[3 + d] = V.box_hi[d];
  }
  for (int k = 0; k < 6; ++k) counts[k] = 0;
  for (uint8_t t : V.type) {
    const int slot = t == T_FLUID ? 0 : t == T_BAND ? 1 : t == T_COVERED ? 2
                     : t == T_GHOST ? 3 : t == T_SOLID ? 4 : 5;
    ++counts[slot];
  }
}

void orc_mlref_types(void* h, int l, uint8_t* type) {
  const MLevel& V = ((MLRefine*)h)->lev[l];
  std::memcpy(type, V.type.data(), V.type.size());
}

// Post-collision state of level l over its whole domain, [Q][N_l]. Setting
// any level forgets the interface history (the next step rebuilds it).
void orc_mlref_set_state(void* h, int l, const double* f) {
  MLRefine& R = *(MLRefine*)h;
  MLevel& V = R.lev[l];
  std::memcpy(V.f.data(), f, sizeof(double) * V.f.size());
  for (MLevel& W : R.lev) W.have_cur = W.have_prev = false;
}

void orc_mlref_get_state(void* h, int l, double* f) {
  const MLevel& V = ((MLRefine*)h)->lev[l];
  std::memcpy(f, V.f.data(), sizeof(double) * V.f.size());
}

// Advance n level-0 steps from level-0 time t0 (level l takes step indices
// t 2^l + k). Returns the number of pulls from unused nodes (0 for a valid
// geometry).
int64_t orc_mlref_run(void* h, int64_t t0, int64_t n) {
  MLRefine& R = *(MLRefine*)h;
  for (int64_t t = t0; t < t0 + n; ++t) advance(R, 0, t);
  int64_t bad = 0;
  for (const MLevel& V : R.lev) bad += V.bad_pull;
  return bad;
}

int64_t orc_mlref_ghost_count(void* h, int l) {
  return (int64_t)((MLRefine*)h)->lev[l].ghosts.size();
}

// Ghost coordinates of level l >= 1 ([ng][3]) and, if parent is given (a
// level l-1 field [Q][N_{l-1}]), its raw spatial interpolation at them
// ([Q][ng]).
void orc_mlref_ghosts(void* h, int l, int32_t* coords, const double* parent, double* g) {
  const MLRefine& R = *(MLRefine*)h;
  const MLevel& V = R.lev[l];
  for (size_t gi = 0; gi < V.ghosts.size(); ++gi) {
    int x[3];
    lcoords(V, V.ghosts[gi], x);
    for (int d = 0; d < 3; ++d) coords[3 * gi + d] = x[d];
  }
  if (parent && g) {
    const MLevel& P = R.lev[l - 1];
    std::vector<double> fp(parent, parent + (size_t)R.Q * P.N), out;
    interp_ghosts(R, l, fp, out);
    std::memcpy(g, out.data(), out.size() * sizeof(double));
  }
}

// Rescale one node between level l-1 and level l (dir > 0: parent state to
// the child level; dir < 0: back). Returns the shear ratio used.
double orc_mlref_rescale(void* h, int l, const double* f, int dir, double* out) {
  const MLRefine& R = *(MLRefine*)h;
  return rescale_node(&R.lev[l - 1].p, &R.lev[l].p, f, dir, out);
}

// The half-step ghost values of level l >= 1 that a step fills from raw
// parent interpolations at t-1, t, t+1 (each [Q][ng]; gm1 ignored unless
// have_prev): time weights, then the rescaling, as in a refined step. out:
// [Q][ng]. The level's stored interface history is left as it was.
void orc_mlref_half_step(void* h, int l, const double* gm1, const double* g0, const double* gp1,
                         int have_prev, double* out) {
  MLRefine& R = *(MLRefine*)h;
  MLevel& V = R.lev[l];
  const size_t n = (size_t)R.Q * V.ghosts.size();
  std::vector<double> keep[3] = {V.G[0], V.G[1], V.G[2]};
  V.G[0].assign(have_prev ? gm1 : g0, (have_prev ? gm1 : g0) + n);
  V.G[1].assign(g0, g0 + n);
  V.G[2].assign(gp1, gp1 + n);
  std::vector<double> fsave = V.f;
  double w[3];
  half_step_weights(have_prev != 0, w);
  fill_ghosts(R, l, w[0], w[1], w[2]);
  for (int q = 0; q < R.Q; ++q)
    for (size_t gi = 0; gi < V.ghosts.size(); ++gi)
      out[(size_t)q * V.ghosts.size() + gi] = V.f[(size_t)q * V.N + V.ghosts[gi]];
  V.f.swap(fsave);
  for (int k = 0; k < 3; ++k) V.G[k].swap(keep[k]);
}

// FP64 sums over the domain: the fluid nodes of every level that no finer
// level covers, weighted by their volume 8^-l in level-0 cells: sum of
// rho - 1, momentum, |j|^2 / (2 rho) (rho = 1 for the MRT).
void orc_mlref_reduce(void* h, double* out) {
  const MLRefine& R = *(MLRefine*)h;
  for (int k = 0; k < 5; ++k) out[k] = 0.0;
  for (int l = 0; l < R.L; ++l) {
    const MLevel& V = R.lev[l];
    const double w = std::ldexp(1.0, -3 * l);
    for (long k = 0; k < V.N; ++k) {
      if (V.type[k] != T_FLUID) continue;
      double d = 0.0, j[3] = {0, 0, 0};
      for (int q = 0; q < R.Q; ++q) {
        const double v = V.f[(size_t)q * V.N + k];
        d += v;
        for (int a = 0; a < 3; ++a) j[a] += v * E[q][a];
      }
      const double rho = V.p.model == ORC_MRT19 ? 1.0 : 1.0 + d;
      out[0] += w * d;
      for (int a = 0; a < 3; ++a) out[1 + a] += w * j[a];
      out[4] += w * 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
    }
  }
}

}  // extern "C"

// ===========================================================================
// Discrete adjoint of the FCLB and MRT-LES collide-and-stream maps (used to
// check the GPU's hand-written adjoint): step t maps the pre-collision state f_t to
// f_{t+1} = S(C(f_t), u_in); for an objective J(f_T) the adjoint runs
// lambda_t = J_C(f_t)^T S^T lambda_{t+1}, and the inlet velocity's gradient
// collects the bounce-back terms 6 w_i e_i lambda_{t+1,i}.
// ===========================================================================
extern "C" {

void orc_collide_jvp(const orc_params* p, const double* f, const double* v, double* out) {
  collide_jvp(p, f, v, out);
}

// Tangent of one step: out = S(J_C(f_t) v) (the inlet velocity held fixed).
void orc_tangent_step(const orc_params* p, const double* f, const double* v, double* out) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  std::vector<double> dpost((size_t)Q * N);
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double a[27], b[27], c[27];
    for (int i = 0; i < Q; ++i) {
      a[i] = f[i * N + n];
      b[i] = v[i * N + n];
    }
    collide_jvp(p, a, b, c);
    for (int i = 0; i < Q; ++i) dpost[i * N + n] = c[i];
  }
  #pragma omp parallel for schedule(static)
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const long self = node_index(p, x, y, z);
        for (int i = 0; i < Q; ++i) {
          const Source src = classify(p, i, x, y, z);
          const int k = (src.kind == SRC_WALL || src.kind == SRC_INLET) ? opposite(Q, i) : i;
          out[i * N + self] = dpost[k * N + src.node];
        }
      }
}

// One adjoint step. f: pre-collision state at t; lam_next: adjoint at t+1;
// lam: output adjoint at t; grad: [3][nb][na] inlet-velocity gradient,
// accumulated (the inlet face's tangential layout of the forward inlet).
void orc_adjoint_step(const orc_params* p, const double* f, const double* lam_next, double* lam,
                      double* grad) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  std::vector<double> mu((size_t)Q * N, 0.0);
  // S^T: scatter every pulled population back to where it came from
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const long self = node_index(p, x, y, z);
        for (int i = 0; i < Q; ++i) {
          const double v = lam_next[i * N + self];
          const Source src = classify(p, i, x, y, z);
          if (src.kind == SRC_NORMAL || src.kind == SRC_OUTFLOW) {
            mu[i * N + src.node] += v;
          } else {
            mu[opposite(Q, i) * N + src.node] += v;
            if (src.kind == SRC_INLET && grad) {
              const int g[3] = {x + p->origin[0], y + p->origin[1], z + p->origin[2]};
              const int axis = src.face / 2;
              const int a = g[axis == 0 ? 1 : 0], b = g[axis == 2 ? 1 : 2];
              const long nf = (long)p->inlet_na * p->inlet_nb;
              for (int c = 0; c < 3; ++c)
                grad[c * nf + (long)b * p->inlet_na + a] += 6.0 * weight(Q, i) * E[i][c] * v;
            }
          }
        }
      }
  // J_C^T per node: column j of J_C is the JVP with the unit vector e_j
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double a[27], e[27], c[27];
    for (int i = 0; i < Q; ++i) a[i] = f[i * N + n];
    for (int j = 0; j < Q; ++j) {
      for (int i = 0; i < Q; ++i) e[i] = (i == j) ? 1.0 : 0.0;
      collide_jvp(p, a, e, c);
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += c[i] * mu[i * N + n];
      lam[j * N + n] = s;
    }
  }
}

// Mean kinetic energy |j|^2 / (2 rho) over the probe box [lo, hi) of the
// pre-collision state f, and (if lam is not null) its gradient dJ/df.
double orc_probe_ke(const orc_params* p, const double* f, const int32_t* lo, const int32_t* hi,
                    double* lam) {
  const int Q = nq(p->model);
  const long N = (long)p->nx * p->ny * p->nz;
  const double np = (double)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  if (lam)
    for (long k = 0; k < (long)Q * N; ++k) lam[k] = 0.0;
  double J = 0.0;
  for (int z = lo[2]; z < hi[2]; ++z)
    for (int y = lo[1]; y < hi[1]; ++y)
      for (int x = lo[0]; x < hi[0]; ++x) {
        const long n = node_index(p, x, y, z);
        double d = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
          d += f[i * N + n];
          for (int a = 0; a < 3; ++a) j[a] += f[i * N + n] * E[i][a];
        }
        const bool comp = p->model == ORC_FCLB27;
        const double rho = comp ? 1.0 + d : 1.0;
        const double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        J += 0.5 * jj / rho / np;
        if (lam)
          for (int i = 0; i < Q; ++i) {
            const double ej = E[i][0] * j[0] + E[i][1] * j[1] + E[i][2] * j[2];
            lam[i * N + n] = (ej / rho - (comp ? 0.5 * jj / (rho * rho) : 0.0)) / np;
          }
      }
  return J;
}

}  // extern "C"
