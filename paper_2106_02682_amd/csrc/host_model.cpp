// Host-side construction of the fixed data of a problem:
//   * local Hamiltonians H_0 (m x m) and H_0d (n x n) of a translation-invariant
//     pairwise Hamiltonian on a cluster tiling (Sections 2.1, 2.3, 3.3);
//   * the signed-permutation tables of the single-site Pauli collection;
//   * the unique lattice momenta and DFT twiddles of Section 3.3.
#include "host_model.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <stdexcept>

namespace vemb {

using cd = std::complex<double>;

namespace {

// Matrix of a Pauli string on one cluster of L sites: letters[s] in {I,X,Y,Z}
// for local site s (site 0 = most significant bit).
std::vector<cd> cluster_operator(const std::vector<int>& letters, int L) {
  const int m = 1 << L;
  std::vector<cd> op((size_t)m * m, cd(0.0, 0.0));
  for (int u = 0; u < m; ++u) {  // column (input basis state)
    int r = u;
    cd amp(1.0, 0.0);
    for (int s = 0; s < L; ++s) {
      const int bitpos = L - 1 - s;
      const int b = (u >> bitpos) & 1;
      switch (letters[s]) {
        case VEMB_X:
          r ^= 1 << bitpos;
          break;
        case VEMB_Y:  // Y|0> = i|1>, Y|1> = -i|0>
          r ^= 1 << bitpos;
          amp *= (b == 0) ? cd(0.0, 1.0) : cd(0.0, -1.0);
          break;
        case VEMB_Z:
          amp *= (b == 0) ? 1.0 : -1.0;
          break;
        default:
          break;
      }
    }
    op[(size_t)r * m + u] += amp;
  }
  return op;
}

std::vector<cd> kron(const std::vector<cd>& A, const std::vector<cd>& B, int m) {
  const int n = m * m;
  std::vector<cd> out((size_t)n * n);
  for (int x = 0; x < m; ++x)
    for (int xp = 0; xp < m; ++xp)
      for (int y = 0; y < m; ++y)
        for (int yp = 0; yp < m; ++yp)
          out[(size_t)(x * m + y) * n + (xp * m + yp)] = A[(size_t)x * m + xp] * B[(size_t)y * m + yp];
  return out;
}

// coeff (a_p^dag a_q + a_q^dag a_p) on `nsites` sites in Jordan-Wigner order (site 0 the most
// significant bit, occupied = 1), added to the dim x dim matrix H: the hopping moves a particle
// between q and p with the sign (-1)^(number of occupied sites strictly between them).
void add_hopping(std::vector<cd>& H, int nsites, int p, int q, double coeff) {
  const int dim = 1 << nsites;
  const int bp = 1 << (nsites - 1 - p), bq = 1 << (nsites - 1 - q);
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  int between = 0;
  for (int k = lo + 1; k < hi; ++k) between |= 1 << (nsites - 1 - k);
  for (int u = 0; u < dim; ++u) {
    for (int dir = 0; dir < 2; ++dir) {  // a_p^dag a_q, then a_q^dag a_p
      const int from = dir == 0 ? bq : bp, to = dir == 0 ? bp : bq;
      if (!(u & from) || (u & to)) continue;
      const double sign = (__builtin_popcount(u & between) & 1) ? -1.0 : 1.0;
      const int r = u ^ from ^ to;
      H[(size_t)r * dim + u] += coeff * sign;
    }
  }
}

}  // namespace

}  // namespace vemb

// The options' defaults live with their validation (host code only).
extern "C" void vemb_default_options(vemb_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mu = 10.0;
  o->nu = 10.0;
  o->eps = 2.0;
  o->opset = VEMB_OPSET_COMPLETE;
  o->precision = VEMB_FP64;
  o->max_sweeps = 40;
  o->sign = -1;
  o->warm_refresh = 64;
}

namespace vemb {

int normalize_options(const vemb_options* in, vemb_options& o, std::string& err) {
  vemb_default_options(&o);
  if (in) o = *in;
  if (o.max_sweeps <= 0) o.max_sweeps = 40;
  if (o.sign == 0) o.sign = -1;
  if (o.warm_refresh == 0) o.warm_refresh = 64;
  if (!(o.mu > 0 && o.nu > 0 && o.eps > 0)) return err = "mu, nu, eps must be positive", VEMB_E_INVALID;
  if (o.opset != VEMB_OPSET_COMPLETE && o.opset != VEMB_OPSET_PAULI1) return err = "unknown opset", VEMB_E_INVALID;
  if (o.precision < VEMB_FP64 || o.precision > VEMB_FP32) return err = "unknown precision", VEMB_E_INVALID;
  if (o.fermionic != 0 && o.fermionic != 1) return err = "fermionic must be 0 or 1", VEMB_E_INVALID;
  if (o.lb_every < 0) return err = "lb_every must be >= 0", VEMB_E_INVALID;
  if (o.adapt_every < 0) return err = "adapt_every must be >= 0", VEMB_E_INVALID;
  if (o.fermionic && o.opset != VEMB_OPSET_COMPLETE)
    return err = "fermionic problems use the complete operator collection", VEMB_E_UNSUPPORTED;
  return VEMB_OK;
}

int parse_geometry(const vemb_lattice& lat, const vemb_clusters& cl, Geometry& g, std::string& err) {
  if (lat.ndim != 1 && lat.ndim != 2) return err = "ndim must be 1 or 2", VEMB_E_INVALID;
  g = Geometry{};
  g.Nx = lat.extent[0];
  g.Ny = lat.ndim == 2 ? lat.extent[1] : 1;
  g.Lx = cl.shape[0];
  g.Ly = lat.ndim == 2 ? cl.shape[1] : 1;
  if (lat.ndim == 1 && cl.shape[1] > 1) return err = "2D cluster on a 1D lattice", VEMB_E_INVALID;
  if (g.Nx <= 0 || g.Ny <= 0 || g.Lx <= 0 || g.Ly <= 0) return err = "extents must be positive", VEMB_E_INVALID;
  if (!lat.periodic[0] || (lat.ndim == 2 && !lat.periodic[1]))
    return err = "translation invariance needs periodic boundaries", VEMB_E_UNSUPPORTED;
  if (g.Nx % g.Lx || g.Ny % g.Ly) return err = "clusters do not tile the lattice", VEMB_E_INVALID;
  g.Mx = g.Nx / g.Lx;
  g.My = g.Ny / g.Ly;
  // cluster counts beyond 2^20 would not fit the per-offset tables (and overflow int products)
  if ((long long)g.Mx * g.My > (1LL << 20)) return err = "more than 2^20 clusters", VEMB_E_UNSUPPORTED;
  g.M = g.Mx * g.My;
  g.L = g.Lx * g.Ly;
  if (g.M < 2) return err = "at least two clusters are needed (M >= 2)", VEMB_E_UNSUPPORTED;
  if (g.L > 4) return err = "clusters of more than 4 sites are not supported", VEMB_E_UNSUPPORTED;
  g.m = 1 << g.L;
  g.n = g.m * g.m;
  return VEMB_OK;
}

int build_model(const vemb_hamiltonian& H, const Geometry& g, HostModel& out, std::string& err, bool fermionic) {
  const int L = g.L, m = g.m, n = g.n, M = g.M;
  std::vector<cd> H0((size_t)m * m, cd(0, 0));
  std::vector<std::vector<cd>> Hd(M);
  for (int t = 0; t < H.nterms; ++t) {
    const vemb_term& term = H.terms[t];
    if (term.nsites < 1 || term.nsites > 2) {
      err = "only one- and two-site terms are pairwise";
      return VEMB_E_UNSUPPORTED;
    }
    for (int s = 0; s < term.nsites; ++s)
      if (term.pauli[s] < 0 || term.pauli[s] > VEMB_FHOP) {
        err = "Pauli letter out of range";
        return VEMB_E_INVALID;
      }
    const bool hop = term.nsites == 2 && term.pauli[0] == VEMB_FHOP && term.pauli[1] == VEMB_FHOP;
    if (!hop && (term.pauli[0] == VEMB_FHOP || (term.nsites == 2 && term.pauli[1] == VEMB_FHOP))) {
      err = "a hopping term has two VEMB_FHOP ends";
      return VEMB_E_INVALID;
    }
    if (hop && !fermionic) {
      err = "hopping terms need a fermionic problem (vemb_options.fermionic = 1)";
      return VEMB_E_INVALID;
    }
    if (fermionic && !hop)
      for (int s = 0; s < term.nsites; ++s)
        if (term.pauli[s] == VEMB_X || term.pauli[s] == VEMB_Y) {
          err = "fermionic problems take hoppings and Z (1 - 2n) letters only";
          return VEMB_E_UNSUPPORTED;
        }
    for (int x = 0; x < g.Nx; ++x)
      for (int y = 0; y < g.Ny; ++y) {
        int cl[2], loc[2], site[2];
        for (int s = 0; s < term.nsites; ++s) {
          const int sx = ((x + term.offset[s][0]) % g.Nx + g.Nx) % g.Nx;
          const int sy = ((y + term.offset[s][1]) % g.Ny + g.Ny) % g.Ny;
          site[s] = sx * g.Ny + sy;
          cl[s] = (sx / g.Lx) * g.My + (sy / g.Ly);
          loc[s] = (sx % g.Lx) * g.Ly + (sy % g.Ly);
        }
        if (term.nsites == 2 && site[0] == site[1]) {
          err = "a two-site term folds onto one site on this lattice";
          return VEMB_E_UNSUPPORTED;
        }
        const bool touches0 = cl[0] == 0 || (term.nsites == 2 && cl[1] == 0);
        if (!touches0) continue;
        if (hop && cl[0] == cl[1]) {
          // hopping inside cluster 0, in the cluster's Jordan-Wigner order
          add_hopping(H0, L, loc[0], loc[1], term.coeff);
        } else if (hop) {
          // hopping between cluster 0 and cluster d, in the pair's order (cluster 0 first)
          const int s0 = cl[0] == 0 ? 0 : 1;
          const int d = cl[1 - s0];
          if (Hd[d].empty()) Hd[d].assign((size_t)n * n, cd(0, 0));
          add_hopping(Hd[d], 2 * L, loc[s0], L + loc[1 - s0], term.coeff);
        } else if (term.nsites == 1 || cl[0] == cl[1]) {
          // both factors inside cluster 0: product of single-site operators
          std::vector<int> letters(L, VEMB_I);
          std::vector<cd> op;
          for (int s = 0; s < term.nsites; ++s) {
            std::vector<int> one(L, VEMB_I);
            one[loc[s]] = term.pauli[s];
            std::vector<cd> f = cluster_operator(one, L);
            if (op.empty()) {
              op = f;
            } else {
              std::vector<cd> prod((size_t)m * m, cd(0, 0));
              for (int i = 0; i < m; ++i)
                for (int k = 0; k < m; ++k)
                  for (int j = 0; j < m; ++j) prod[(size_t)i * m + j] += op[(size_t)i * m + k] * f[(size_t)k * m + j];
              op = prod;
            }
          }
          for (size_t e = 0; e < op.size(); ++e) H0[e] += term.coeff * op[e];
        } else {
          // one factor in cluster 0 (first tensor factor), the other in cluster d
          const int s0 = cl[0] == 0 ? 0 : 1;
          const int s1 = 1 - s0;
          const int d = cl[s1];
          std::vector<int> l0(L, VEMB_I), l1(L, VEMB_I);
          l0[loc[s0]] = term.pauli[s0];
          l1[loc[s1]] = term.pauli[s1];
          std::vector<cd> op = kron(cluster_operator(l0, L), cluster_operator(l1, L), m);
          if (Hd[d].empty()) Hd[d].assign((size_t)n * n, cd(0, 0));
          for (size_t e = 0; e < op.size(); ++e) Hd[d][e] += term.coeff * op[e];
        }
      }
  }
  // real case only (Section 3): every imaginary part must cancel
  double imax = 0.0;
  for (const cd& v : H0) imax = std::max(imax, std::abs(v.imag()));
  for (const auto& h : Hd)
    for (const cd& v : h) imax = std::max(imax, std::abs(v.imag()));
  if (imax > 1e-12) {
    err = "complex Hamiltonian terms are not supported (real case only)";
    return VEMB_E_UNSUPPORTED;
  }
  out.H0.assign((size_t)m * m, 0.0);
  for (size_t e = 0; e < H0.size(); ++e) out.H0[e] = H0[e].real();
  out.hd_index.assign(M - 1, -1);
  out.Hd.clear();
  int nh = 0;
  for (int d = 1; d < M; ++d) {
    if (Hd[d].empty()) continue;
    out.hd_index[d - 1] = nh++;
    for (const cd& v : Hd[d]) out.Hd.push_back(v.real());
  }
  return VEMB_OK;
}

void build_pauli1_tables(int L, OpTables& T) {
  const int m = 1 << L;
  T.n_op = 3 * L;
  for (int s = 0; s < L; ++s) {
    const int bitpos = L - 1 - s;
    for (int key = 0; key < 3; ++key) {
      const int a = 3 * s + key;
      for (int u = 0; u < m; ++u) {
        const int b = (u >> bitpos) & 1;
        if (key == 0) {  // sigma^x
          T.perm[a][u] = (int8_t)(u ^ (1 << bitpos));
          T.sign[a][u] = 1;
        } else if (key == 1) {  // sigma^z
          T.perm[a][u] = (int8_t)u;
          T.sign[a][u] = (int8_t)(1 - 2 * b);
        } else {  // sigma^x sigma^z: row u has its entry at column u^bit, value 2b - 1
          T.perm[a][u] = (int8_t)(u ^ (1 << bitpos));
          T.sign[a][u] = (int8_t)(2 * b - 1);
        }
      }
    }
  }
}

void build_momenta(const Geometry& g, std::vector<double>& tw, std::vector<double>& wk, int& Ku) {
  const int Mx = g.Mx, My = g.My, M = g.M;
  std::vector<int> ks;
  for (int kx = 0; kx < Mx; ++kx)
    for (int ky = 0; ky < My; ++ky) {
      const int f = kx * My + ky;
      const int nf = ((Mx - kx) % Mx) * My + ((My - ky) % My);
      if (f <= nf) {
        ks.push_back(f);
        wk.push_back(f == nf ? 1.0 : 2.0);
      }
    }
  Ku = (int)ks.size();
  tw.assign((size_t)2 * Ku * M, 0.0);
  const double norm = 1.0 / std::sqrt((double)M);
  for (int ki = 0; ki < Ku; ++ki) {
    const int kx = ks[ki] / My, ky = ks[ki] % My;
    for (int d = 0; d < M; ++d) {
      const int dx = d / My, dy = d % My;
      // angle / 2 pi = (dx kx / Mx + dy ky / My) = ((dx kx My + dy ky Mx) mod M) / M
      const long long num = ((long long)dx * kx * My + (long long)dy * ky * Mx) % M;
      const double ang = 2.0 * M_PI * (double)num / (double)M;
      tw[2 * ((size_t)ki * M + d)] = norm * std::cos(ang);
      tw[2 * ((size_t)ki * M + d) + 1] = -norm * std::sin(ang);
    }
  }
}

int add_site_field(const Geometry& g, int x, int y, int pauli, double coeff, std::vector<double>& Hc,
                   std::string& err) {
  if (pauli != VEMB_X && pauli != VEMB_Z) {
    err = "one-site fields must be X or Z (real)";
    return VEMB_E_UNSUPPORTED;
  }
  if (!std::isfinite(coeff)) {
    err = "non-finite field";
    return VEMB_E_INVALID;
  }
  const int xs = ((x % g.Nx) + g.Nx) % g.Nx, ys = ((y % g.Ny) + g.Ny) % g.Ny;
  const int c = (xs / g.Lx) * g.My + (ys / g.Ly);
  const int loc = (xs % g.Lx) * g.Ly + (ys % g.Ly);
  std::vector<int> letters(g.L, VEMB_I);
  letters[loc] = pauli;
  const std::vector<cd> op = cluster_operator(letters, g.L);
  const size_t mm = (size_t)g.m * g.m;
  for (size_t e = 0; e < mm; ++e) Hc[(size_t)c * mm + e] += coeff * op[e].real();
  return VEMB_OK;
}

}  // namespace vemb
