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
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

extern "C" {

enum { ORC_MRT19 = 1, ORC_FCLB27 = 2 };
enum { ORC_BASIS_TABLE1 = 0, ORC_BASIS_DHUMIERES = 1 };
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_INLET = 2, ORC_OUTFLOW = 3 };

// Must match the ctypes structure in oracle/__init__.py.
typedef struct orc_params {
  int32_t model;        // ORC_MRT19 or ORC_FCLB27
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

double ipow(double x, int k) {
  double r = 1.0;
  for (int j = 0; j < k; ++j) r *= x;
  return r;
}

// Gaussian elimination with partial pivoting: solves A x = b in place
// (A is n x n row-major and is destroyed; b becomes x).
void dense_solve(int n, double* A, double* b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      double v = std::fabs(A[r * n + k]);
      if (v > best) { best = v; p = r; }
    }
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[p * n + c]);
      std::swap(b[k], b[p]);
    }
    for (int r = k + 1; r < n; ++r) {
      double l = A[r * n + k] / A[k * n + k];
      if (l == 0.0) continue;
      for (int c = k; c < n; ++c) A[r * n + c] -= l * A[k * n + c];
      b[r] -= l * b[k];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
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
void central_moments(const double* F, double* rho_out, double* u, double* kappa) {
  double rho = 0.0, j[3] = {0, 0, 0};
  for (int i = 0; i < 27; ++i) {
    rho += F[i];
    for (int a = 0; a < 3; ++a) j[a] += F[i] * E[i][a];
  }
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int i = 0; i < 27; ++i)
          s += F[i] * ipow(E[i][0] - u[0], a) * ipow(E[i][1] - u[1], b) *
               ipow(E[i][2] - u[2], c);
        kappa[9 * a + 3 * b + c] = s / rho;
      }
  *rho_out = rho;
}

// FCLB collision (Section 2, Table 1 groups applied to central moments,
// Table 2 equilibria, all rates except the shear rate equal to 1).
void fclb_collide(const double* f, double omega, double* fout) {
  double F[27];
  for (int i = 0; i < 27; ++i) F[i] = weight(27, i) + f[i];
  double rho, u[3], k[27];
  central_moments(F, &rho, u, k);
  auto K = [&](int a, int b, int c) { return k[9 * a + 3 * b + c]; };
  double ks[27];
  for (int m = 0; m < 27; ++m) ks[m] = 0.0;  // orders 1, 3, 5 relax to 0
  ks[0] = 1.0;
  const double T = K(2, 0, 0) + K(0, 2, 0) + K(0, 0, 2);
  // second order: trace to 1 (rate s2 = 1), deviatoric part at omega
  const double k200 = 1.0 / 3.0 + (1.0 - omega) * (K(2, 0, 0) - T / 3.0);
  const double k020 = 1.0 / 3.0 + (1.0 - omega) * (K(0, 2, 0) - T / 3.0);
  const double k002 = 1.0 / 3.0 + (1.0 - omega) * (K(0, 0, 2) - T / 3.0);
  const double k110 = (1.0 - omega) * K(1, 1, 0);
  const double k101 = (1.0 - omega) * K(1, 0, 1);
  const double k011 = (1.0 - omega) * K(0, 1, 1);
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
  // back to populations: sum_i F*_i prod_a (e_ia - u_a)^{n_a} = rho kappa*
  double A[27 * 27], b[27];
  for (int a = 0; a < 3; ++a)
    for (int bb = 0; bb < 3; ++bb)
      for (int c = 0; c < 3; ++c) {
        const int m = 9 * a + 3 * bb + c;
        for (int i = 0; i < 27; ++i)
          A[m * 27 + i] = ipow(E[i][0] - u[0], a) * ipow(E[i][1] - u[1], bb) *
                          ipow(E[i][2] - u[2], c);
        b[m] = rho * ks[m];
      }
  dense_solve(27, A, b);
  for (int i = 0; i < 27; ++i) fout[i] = b[i] - weight(27, i);
}

void collide_node(const orc_params* p, const double* f, double* fout) {
  const double tau0 = 3.0 * p->nu + 0.5;
  if (p->model == ORC_MRT19)
    mrt_collide(f, tau0, p->cs_smag, p->mrt_basis, p->rates, fout, nullptr);
  else
    fclb_collide(f, 1.0 / tau0, fout);
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

// Pull-streamed value of population i at node (x,y,z) at t+1 from the
// post-collision field fpost of step t, with the boundary rules:
//  * periodic faces wrap;
//  * a source beyond a WALL face: halfway bounce-back with the wall's
//    velocity, f_i = f*_opp(i) + 6 w_i (e_i . u_w);
//  * beyond an INLET face: the same with the inlet velocity at the node;
//  * beyond OUTFLOW faces only: the post-collision value of the nearest
//    boundary node (a ghost layer copying the last plane).
// When a source lies beyond several faces, WALL wins over INLET over OUTFLOW.
double pull(const orc_params* p, const double* fpost, int Q, int i, int x, int y,
            int z, int64_t t) {
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
  const long N = (long)p->nx * p->ny * p->nz;
  if (!any) return fpost[i * N + node_index(p, s[0], s[1], s[2])];
  const long self = node_index(p, x, y, z);
  const int io = opposite(Q, i);
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_WALL) {
      const double* uw = p->face_u[face];
      const double eu = E[i][0] * uw[0] + E[i][1] * uw[1] + E[i][2] * uw[2];
      return fpost[io * N + self] + 6.0 * weight(Q, i) * eu;
    }
  for (int face = 0; face < 6; ++face)
    if (crossed[face] && p->face_type[face] == ORC_INLET) {
      double uin[3];
      inlet_velocity(p, face, x, y, z, t, uin);
      const double eu = E[i][0] * uin[0] + E[i][1] * uin[1] + E[i][2] * uin[2];
      return fpost[io * N + self] + 6.0 * weight(Q, i) * eu;
    }
  for (int d = 0; d < 3; ++d) {
    if (s[d] < 0) s[d] = 0;
    if (s[d] >= n[d]) s[d] = n[d] - 1;
  }
  return fpost[i * N + node_index(p, s[0], s[1], s[2])];
}

}  // namespace

extern "C" {

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
