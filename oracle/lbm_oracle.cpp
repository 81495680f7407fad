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
void feq_incomp(int Q, double drho, const double u[3], double* feq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    const double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
    feq[i] = weight(Q, i) * (drho + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
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
void mrt_rates(int basis, const double* rates, double s_shear, double* s) {
  for (int k = 0; k < 19; ++k) s[k] = 0.0;
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
double smagorinsky_tau(const double* f, double tau0, double cs, double* Q_out) {
  double drho = 0, u[3] = {0, 0, 0};
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    for (int a = 0; a < 3; ++a) u[a] += f[i] * E[i][a];
  }
  double feq[19];
  feq_incomp(19, drho, u, feq);
  double pi2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double p = 0.0;
      for (int i = 0; i < 19; ++i) p += E[i][a] * E[i][b] * (f[i] - feq[i]);
      pi2 += p * p;
    }
  const double Q = std::sqrt(2.0 * pi2);
  if (Q_out) *Q_out = Q;
  return 0.5 * (tau0 + std::sqrt(tau0 * tau0 + 18.0 * cs * cs * Q));
}

// Eq. (12), read with the sign of a relaxation: f* = f - M^-1 S (M f - M f_eq).
void mrt_collide(const double* f, double tau0, double cs, int basis,
                 const double* rates, double* fout, double* tau_out) {
  const MrtBasis& B = get_basis(basis);
  double drho = 0, u[3] = {0, 0, 0};
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    for (int a = 0; a < 3; ++a) u[a] += f[i] * E[i][a];
  }
  double feq[19];
  feq_incomp(19, drho, u, feq);
  const double tau = smagorinsky_tau(f, tau0, cs, nullptr);
  if (tau_out) *tau_out = tau;
  double s[19];
  mrt_rates(basis, rates, 1.0 / tau, s);
  double d[19];
  for (int k = 0; k < 19; ++k) {
    double m = 0.0, meq = 0.0;
    for (int i = 0; i < 19; ++i) {
      m += B.M[k * 19 + i] * f[i];
      meq += B.M[k * 19 + i] * feq[i];
    }
    d[k] = s[k] * (m - meq);
  }
  for (int i = 0; i < 19; ++i) {
    double c = 0.0;
    for (int k = 0; k < 19; ++k) c += B.Minv[i * 19 + k] * d[k];
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
    mrt_collide(f, tau0, p->cs_smag, p->mrt_basis, p->rates, fout, nullptr);
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

// Exact Jacobian-vector product of the FCLB collision of one node, by
// forward-mode dual numbers through the same code as the collision.
void collide_jvp(const orc_params* p, const double* f, const double* v, double* out) {
  const double tau0 = 3.0 * p->nu + 0.5;
  Dual a[27], b[27];
  for (int i = 0; i < 27; ++i) a[i] = Dual(f[i], v[i]);
  fclb_collide(a, 1.0 / tau0, b);
  for (int i = 0; i < 27; ++i) out[i] = b[i].d;
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
// Two-level nested time refinement (Section 1: hierarchical block grid with a
// nested time step, Yu et al.'s interpolation and rescaling; Section 3:
// refinement levels, constant CFL). The paper cites the method and prints no
// formulas; this follows the readings recorded in the design notes:
//  * 2:1 vertex-centred nesting: fine node j sits at coarse coordinate j/2;
//    a refined coarse block of B^3 nodes carries (2B)^3 fine nodes;
//    dt_f = dt_c / 2, so in lattice units nu_f = 2 nu_c (tau_f - 1/2 =
//    2 (tau_c - 1/2)) and velocities are equal on both levels.
//  * Both levels store post-collision values and advance by pull + collide.
//  * Fine ghost nodes (outside the refined region, next to it) hold coarse
//    post-collision populations interpolated in space (tensor 4-point cubic
//    Lagrange, one-sided near non-periodic domain faces) and in time (linear
//    between the coarse states at t and t+1 for the half step), rescaled
//    f_f = f_eq + r (f_c - f_eq), r = (tau_f - 1) / (2 (tau_c - 1)).
//  * Covered coarse nodes (refined, outside every ghost stencil) receive
//    f_c = f_eq + (f_f - f_eq) / r from the coincident fine node after each
//    coarse step.
// ===========================================================================

namespace {

struct Refine {
  orc_params c;      // coarse lattice (full domain)
  orc_params f;      // fine level: global fine extent 2N, fine viscosity
  int B;             // block size (coarse nodes)
  int nb[3];         // blocks per axis
  std::vector<uint8_t> mask;
  int lo[3], M[3];   // fine box origin (global fine coords) and extent
  std::vector<uint8_t> ctype;  // 0 outside R, 1 refined (band), 2 covered
  std::vector<uint8_t> ftype;  // 0 inactive, 1 fluid, 2 ghost
  std::vector<long> ghosts;    // fine box indices of ghost nodes
  double r;
  int Q;
  std::vector<double> g0, g1;  // interpolated coarse values at ghosts [Q][ng]
  bool have_g0 = false;
};

bool refined_block(const Refine& R, int bx, int by, int bz) {
  return R.mask[((long)bz * R.nb[1] + by) * R.nb[0] + bx] != 0;
}

bool coarse_in_R(const Refine& R, int x, int y, int z) {
  return refined_block(R, x / R.B, y / R.B, z / R.B);
}

bool fine_in_R(const Refine& R, int jx, int jy, int jz) {
  const int n2[3] = {2 * R.c.nx, 2 * R.c.ny, 2 * R.c.nz};
  if (jx < 0 || jy < 0 || jz < 0 || jx >= n2[0] || jy >= n2[1] || jz >= n2[2]) return false;
  return refined_block(R, jx / (2 * R.B), jy / (2 * R.B), jz / (2 * R.B));
}

long fidx(const Refine& R, int lx, int ly, int lz) {
  return ((long)lz * R.M[1] + ly) * R.M[0] + lx;
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

// Stencil of fine coordinate j along an axis of n coarse nodes: nodes and
// weights (1 node if j is even, 4 otherwise; indices wrapped if periodic).
int stencil1d(int j, int n, bool periodic, int idx[4], double w[4]) {
  if (j % 2 == 0) {
    int c = j / 2;
    if (periodic) c = ((c % n) + n) % n;
    idx[0] = c;
    w[0] = 1.0;
    return 1;
  }
  const double p = 0.5 * j;
  int s = (j - 1) / 2 - 1;
  if (!periodic) {
    if (s < 0) s = 0;
    if (s > n - 4) s = n - 4;
  }
  lagrange4(p, s, w);
  for (int a = 0; a < 4; ++a) idx[a] = periodic ? (((s + a) % n) + n) % n : s + a;
  return 4;
}

void ghost_global(const Refine& R, long gi, int j[3]) {
  const long l = R.ghosts[gi];
  const int lx = (int)(l % R.M[0]), ly = (int)((l / R.M[0]) % R.M[1]),
            lz = (int)(l / ((long)R.M[0] * R.M[1]));
  j[0] = lx + R.lo[0];
  j[1] = ly + R.lo[1];
  j[2] = lz + R.lo[2];
}

// Spatial interpolation of coarse post-collision values at every ghost.
void interp_ghosts(const Refine& R, const double* fc, std::vector<double>& out) {
  const long ng = (long)R.ghosts.size();
  const long Nc = (long)R.c.nx * R.c.ny * R.c.nz;
  const int n3[3] = {R.c.nx, R.c.ny, R.c.nz};
  out.assign((size_t)R.Q * ng, 0.0);
  #pragma omp parallel for schedule(static)
  for (long gi = 0; gi < ng; ++gi) {
    int j[3];
    ghost_global(R, gi, j);
    int idx[3][4];
    double w[3][4];
    int cnt[3];
    for (int d = 0; d < 3; ++d)
      cnt[d] = stencil1d(j[d], n3[d], R.c.face_type[2 * d] == ORC_PERIODIC, idx[d], w[d]);
    for (int q = 0; q < R.Q; ++q) {
      double s = 0.0;
      for (int c = 0; c < cnt[2]; ++c)
        for (int b = 0; b < cnt[1]; ++b)
          for (int a = 0; a < cnt[0]; ++a) {
            const long n = ((long)idx[2][c] * R.c.ny + idx[1][b]) * R.c.nx + idx[0][a];
            s += w[0][a] * w[1][b] * w[2][c] * fc[q * Nc + n];
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

// f_eq + s (f - f_eq) for one node.
void rescale_node(int model, const double* f, double s, double* out) {
  double feq[27];
  equilibrium_of(model, f, feq);
  for (int i = 0; i < nq(model); ++i) out[i] = feq[i] + s * (f[i] - feq[i]);
}

void fill_ghosts(const Refine& R, const std::vector<double>& g, double* ff) {
  const long ng = (long)R.ghosts.size();
  const long Nf = (long)R.M[0] * R.M[1] * R.M[2];
  #pragma omp parallel for schedule(static)
  for (long gi = 0; gi < ng; ++gi) {
    double a[27], b[27];
    for (int q = 0; q < R.Q; ++q) a[q] = g[(size_t)q * ng + gi];
    rescale_node(R.c.model, a, R.r, b);
    for (int q = 0; q < R.Q; ++q) ff[q * Nf + R.ghosts[gi]] = b[q];
  }
}

void inject(const Refine& R, double* fc, const double* ff) {
  const long Nc = (long)R.c.nx * R.c.ny * R.c.nz;
  const long Nf = (long)R.M[0] * R.M[1] * R.M[2];
  #pragma omp parallel for schedule(static)
  for (long n = 0; n < Nc; ++n) {
    if (R.ctype[n] != 2) continue;
    const int x = (int)(n % R.c.nx), y = (int)((n / R.c.nx) % R.c.ny),
              z = (int)(n / ((long)R.c.nx * R.c.ny));
    const long l = fidx(R, 2 * x - R.lo[0], 2 * y - R.lo[1], 2 * z - R.lo[2]);
    double a[27], b[27];
    for (int q = 0; q < R.Q; ++q) a[q] = ff[q * Nf + l];
    rescale_node(R.c.model, a, 1.0 / R.r, b);
    for (int q = 0; q < R.Q; ++q) fc[q * Nc + n] = b[q];
  }
}

// Coarse step in post-collision storage: out = C(pull(in)) on nodes that
// are not covered (covered nodes are left as they are).
void coarse_step(const Refine& R, const double* in, double* out, int64_t t) {
  const orc_params* p = &R.c;
  const long N = (long)p->nx * p->ny * p->nz;
  const int Q = R.Q;
  #pragma omp parallel for schedule(static)
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const long n = node_index(p, x, y, z);
        if (R.ctype[n] == 2) continue;
        double a[27], b[27];
        for (int i = 0; i < Q; ++i) a[i] = pull(p, in, Q, i, x, y, z, t);
        collide_node(p, a, b);
        for (int i = 0; i < Q; ++i) out[i * N + n] = b[i];
      }
}

// Pull on the fine level: sources inside the box come from the box (fluid
// or ghost nodes); sources beyond a domain face follow the boundary rules on
// the fine level (R.f: global fine extent, fine inlet arrays).
double fine_pull(const Refine& R, const double* in, int i, int lx, int ly, int lz, int64_t t) {
  const orc_params* p = &R.f;
  const int j[3] = {lx + R.lo[0], ly + R.lo[1], lz + R.lo[2]};
  const int n[3] = {p->nx, p->ny, p->nz};
  int s[3] = {j[0] - E[i][0], j[1] - E[i][1], j[2] - E[i][2]};
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
  const long Nf = (long)R.M[0] * R.M[1] * R.M[2];
  const long self = fidx(R, lx, ly, lz);
  const int Q = R.Q;
  if (any) {
    const int io = opposite(Q, i);
    for (int face = 0; face < 6; ++face)
      if (crossed[face] && p->face_type[face] == ORC_WALL) {
        const double* uw = p->face_u[face];
        return in[io * Nf + self] + 6.0 * weight(Q, i) *
                                        (E[i][0] * uw[0] + E[i][1] * uw[1] + E[i][2] * uw[2]);
      }
    for (int face = 0; face < 6; ++face)
      if (crossed[face] && p->face_type[face] == ORC_INLET) {
        double uin[3];
        inlet_velocity(p, face, j[0], j[1], j[2], t, uin);
        return in[io * Nf + self] +
               6.0 * weight(Q, i) * (E[i][0] * uin[0] + E[i][1] * uin[1] + E[i][2] * uin[2]);
      }
    // PRESSURE and FREESLIP faces: the rules of classify() and pull() on the
    // fine level's box
    for (int face = 0; face < 6; ++face)
      if (crossed[face] && p->face_type[face] == ORC_PRESSURE) {
        double d = 0.0, jm[3] = {0, 0, 0};
        for (int k = 0; k < Q; ++k) {
          const double v = in[k * Nf + self];
          d += v;
          for (int a = 0; a < 3; ++a) jm[a] += v * E[k][a];
        }
        const double rho = (p->model == ORC_MRT19) ? 1.0 : 1.0 + d;
        const double ub[3] = {jm[0] / rho, jm[1] / rho, jm[2] / rho};
        const double drho = p->face_drho[face];
        double feq[27];
        if (p->model == ORC_MRT19) {
          feq_incomp(19, drho, ub, feq);
        } else {
          for (int k = 0; k < 27; ++k)
            feq[k] = (1.0 + drho) * phi(E[k][0], ub[0]) * phi(E[k][1], ub[1]) *
                         phi(E[k][2], ub[2]) -
                     weight(27, k);
        }
        return -in[io * Nf + self] + feq[i] + feq[io];
      }
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
      return in[velocity_index(Q, e[0], e[1], e[2]) * Nf +
                fidx(R, s[0] - R.lo[0], s[1] - R.lo[1], s[2] - R.lo[2])];
  }
  return in[i * Nf + fidx(R, s[0] - R.lo[0], s[1] - R.lo[1], s[2] - R.lo[2])];
}

void fine_step(const Refine& R, const double* in, double* out, int64_t t) {
  const long Nf = (long)R.M[0] * R.M[1] * R.M[2];
  const int Q = R.Q;
  #pragma omp parallel for schedule(static)
  for (int lz = 0; lz < R.M[2]; ++lz)
    for (int ly = 0; ly < R.M[1]; ++ly)
      for (int lx = 0; lx < R.M[0]; ++lx) {
        const long l = fidx(R, lx, ly, lz);
        if (R.ftype[l] != 1) continue;
        double a[27], b[27];
        for (int i = 0; i < Q; ++i) a[i] = fine_pull(R, in, i, lx, ly, lz, t);
        collide_node(&R.f, a, b);
        for (int i = 0; i < Q; ++i) out[i * Nf + l] = b[i];
      }
}

}  // namespace

extern "C" {

// Build the two-level geometry. coarse: full-domain lattice parameters;
// block: block edge in coarse nodes (must divide nx, ny, nz); mask:
// [nz/B][ny/B][nx/B], 1 = refined; fine inlet arrays at fine resolution
// ([3][2 nb][2 na], may be null if there is no inlet). Returns null on a
// bad configuration.
void* orc_refine_create(const orc_params* coarse, int block, const uint8_t* mask,
                        const double* fine_inlet_u, const uint8_t* fine_inlet_mask) {
  if (block < 2 || coarse->nx % block || coarse->ny % block || coarse->nz % block) return nullptr;
  Refine* R = new Refine();
  R->c = *coarse;
  R->c.solid = nullptr;  // the refined lattice has no interior solids
  R->B = block;
  R->Q = nq(coarse->model);
  R->nb[0] = coarse->nx / block;
  R->nb[1] = coarse->ny / block;
  R->nb[2] = coarse->nz / block;
  const long nblk = (long)R->nb[0] * R->nb[1] * R->nb[2];
  R->mask.assign(mask, mask + nblk);
  // fine level parameters
  R->f = *coarse;
  R->f.nx = 2 * coarse->nx;
  R->f.ny = 2 * coarse->ny;
  R->f.nz = 2 * coarse->nz;
  R->f.nu = 2.0 * coarse->nu;
  R->f.inlet_u = fine_inlet_u;
  R->f.inlet_mask = fine_inlet_mask;
  R->f.inlet_na = 0;
  R->f.inlet_nb = 0;
  for (int face = 0; face < 6; ++face)
    if (coarse->face_type[face] == ORC_INLET) {
      const int d = face / 2;
      const int n2[3] = {R->f.nx, R->f.ny, R->f.nz};
      R->f.inlet_na = n2[d == 0 ? 1 : 0];
      R->f.inlet_nb = n2[d == 2 ? 1 : 2];
    }
  R->f.seed = coarse->seed + 1;
  R->f.solid = nullptr;  // neither level has interior solids or curved links
  R->f.link_q = nullptr;
  R->c.link_q = nullptr;
  for (int k = 0; k < 3; ++k) R->f.origin[k] = 0;
  const double tc = 3.0 * coarse->nu + 0.5, tf = 3.0 * R->f.nu + 0.5;
  R->r = (tf - 1.0) / (2.0 * (tc - 1.0));
  // fine box: bounding box of the refined blocks, one ghost layer beyond
  // every side that is not a domain face
  int blo[3] = {1 << 30, 1 << 30, 1 << 30}, bhi[3] = {-1, -1, -1};
  for (int bz = 0; bz < R->nb[2]; ++bz)
    for (int by = 0; by < R->nb[1]; ++by)
      for (int bx = 0; bx < R->nb[0]; ++bx)
        if (refined_block(*R, bx, by, bz)) {
          const int b3[3] = {bx, by, bz};
          for (int d = 0; d < 3; ++d) {
            blo[d] = std::min(blo[d], b3[d]);
            bhi[d] = std::max(bhi[d], b3[d] + 1);
          }
        }
  for (int d = 0; d < 3 && bhi[0] >= 0; ++d)
    if (coarse->face_type[2 * d] == ORC_PERIODIC) {
      const bool full = blo[d] == 0 && bhi[d] == R->nb[d];
      const bool inside = blo[d] > 0 && bhi[d] < R->nb[d];
      if (!full && !inside) {  // a wrapped fine pull would leave the box
        delete R;
        return nullptr;
      }
    }
  if (bhi[0] < 0) {  // nothing refined: an empty fine level
    for (int d = 0; d < 3; ++d) {
      R->lo[d] = 0;
      R->M[d] = 0;
    }
  } else {
    const int n2[3] = {R->f.nx, R->f.ny, R->f.nz};
    for (int d = 0; d < 3; ++d) {
      int a = 2 * block * blo[d], b = 2 * block * bhi[d];
      if (a > 0) a -= 1;
      if (b < n2[d]) b += 1;
      R->lo[d] = a;
      R->M[d] = b - a;
    }
  }
  const long Nf = (long)R->M[0] * R->M[1] * R->M[2];
  R->ftype.assign(Nf, 0);
  for (int lz = 0; lz < R->M[2]; ++lz)
    for (int ly = 0; ly < R->M[1]; ++ly)
      for (int lx = 0; lx < R->M[0]; ++lx) {
        const int jx = lx + R->lo[0], jy = ly + R->lo[1], jz = lz + R->lo[2];
        uint8_t t = 0;
        if (fine_in_R(*R, jx, jy, jz)) {
          t = 1;
        } else {
          for (int dz = -1; dz <= 1 && !t; ++dz)
            for (int dy = -1; dy <= 1 && !t; ++dy)
              for (int dx = -1; dx <= 1 && !t; ++dx)
                if (fine_in_R(*R, jx + dx, jy + dy, jz + dz)) t = 2;
        }
        R->ftype[fidx(*R, lx, ly, lz)] = t;
        if (t == 2) R->ghosts.push_back(fidx(*R, lx, ly, lz));
      }
  // coarse types: refined nodes are covered unless a ghost stencil uses them
  const long Nc = (long)coarse->nx * coarse->ny * coarse->nz;
  R->ctype.assign(Nc, 0);
  for (int z = 0; z < coarse->nz; ++z)
    for (int y = 0; y < coarse->ny; ++y)
      for (int x = 0; x < coarse->nx; ++x)
        if (coarse_in_R(*R, x, y, z)) R->ctype[((long)z * coarse->ny + y) * coarse->nx + x] = 2;
  const int n3[3] = {coarse->nx, coarse->ny, coarse->nz};
  for (long gi = 0; gi < (long)R->ghosts.size(); ++gi) {
    int j[3];
    ghost_global(*R, gi, j);
    int idx[3][4];
    double w[3][4];
    int cnt[3];
    for (int d = 0; d < 3; ++d)
      cnt[d] = stencil1d(j[d], n3[d], coarse->face_type[2 * d] == ORC_PERIODIC, idx[d], w[d]);
    for (int c = 0; c < cnt[2]; ++c)
      for (int b = 0; b < cnt[1]; ++b)
        for (int a = 0; a < cnt[0]; ++a) {
          const long n = ((long)idx[2][c] * coarse->ny + idx[1][b]) * coarse->nx + idx[0][a];
          if (R->ctype[n] == 2) R->ctype[n] = 1;
        }
  }
  return R;
}

void orc_refine_destroy(void* h) { delete (Refine*)h; }

// lo[3], M[3]; counts = {fluid, ghost, covered, band}; ratio r.
void orc_refine_geometry(void* h, int32_t* lo, int32_t* M, int64_t* counts, double* r) {
  const Refine& R = *(Refine*)h;
  for (int d = 0; d < 3; ++d) {
    lo[d] = R.lo[d];
    M[d] = R.M[d];
  }
  int64_t nf = 0, ng = 0, nc = 0, nbnd = 0;
  for (uint8_t t : R.ftype) {
    nf += t == 1;
    ng += t == 2;
  }
  for (uint8_t t : R.ctype) {
    nc += t == 2;
    nbnd += t == 1;
  }
  counts[0] = nf;
  counts[1] = ng;
  counts[2] = nc;
  counts[3] = nbnd;
  *r = R.r;
}

void orc_refine_types(void* h, uint8_t* ctype, uint8_t* ftype) {
  const Refine& R = *(Refine*)h;
  std::memcpy(ctype, R.ctype.data(), R.ctype.size());
  std::memcpy(ftype, R.ftype.data(), R.ftype.size());
}

// Ghost fine global coordinates [ng][3] and the raw (not rescaled) spatial
// interpolation of a coarse field fc ([Q][Nc]) at them, [Q][ng].
void orc_refine_ghosts(void* h, int32_t* coords, const double* fc, double* g) {
  const Refine& R = *(Refine*)h;
  for (long gi = 0; gi < (long)R.ghosts.size(); ++gi) {
    int j[3];
    ghost_global(R, gi, j);
    for (int d = 0; d < 3; ++d) coords[3 * gi + d] = j[d];
  }
  if (fc && g) {
    std::vector<double> out;
    interp_ghosts(R, fc, out);
    std::memcpy(g, out.data(), out.size() * sizeof(double));
  }
}

// f_eq + s (f - f_eq) on one node of the refined model.
void orc_refine_rescale(void* h, const double* f, double s, double* out) {
  const Refine& R = *(Refine*)h;
  rescale_node(R.c.model, f, s, out);
}

void orc_refine_inject(void* h, double* fc, const double* ff) {
  inject(*(Refine*)h, fc, ff);
}

// Advance n coarse steps from coarse time t0. fc: coarse post-collision
// state [Q][Nc]; ff: fine box post-collision state [Q][M]; both in place.
// Fine step indices (inlet perturbation) are 2t and 2t+1.
void orc_refine_run(void* h, double* fc, double* ff, int64_t t0, int64_t n) {
  Refine& R = *(Refine*)h;
  const long Nc = (long)R.c.nx * R.c.ny * R.c.nz;
  const long Nf = (long)R.M[0] * R.M[1] * R.M[2];
  std::vector<double> bc(fc, fc + (size_t)R.Q * Nc), bf(ff, ff + (size_t)R.Q * Nf);
  std::vector<double> g0, g1;
  for (int64_t t = t0; t < t0 + n; ++t) {
    interp_ghosts(R, fc, g0);
    fill_ghosts(R, g0, ff);
    coarse_step(R, fc, bc.data(), t);
    fine_step(R, ff, bf.data(), 2 * t);
    interp_ghosts(R, bc.data(), g1);
    for (size_t k = 0; k < g0.size(); ++k) g0[k] = 0.5 * (g0[k] + g1[k]);
    fill_ghosts(R, g0, bf.data());
    fine_step(R, bf.data(), ff, 2 * t + 1);
    std::memcpy(fc, bc.data(), sizeof(double) * R.Q * Nc);
    inject(R, fc, ff);
  }
}

}  // extern "C"

// ===========================================================================
// Discrete adjoint of the FCLB collide-and-stream map (used to check the GPU's
// hand-written adjoint): step t maps the pre-collision state f_t to
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
