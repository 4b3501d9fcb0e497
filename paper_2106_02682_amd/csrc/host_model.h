// Host-side fixed data of a problem (see host_model.cpp).
#pragma once

#include <string>
#include <vector>

#include "../../include/vemb.h"
#include "common.h"

namespace vemb {

struct Geometry {
  int Nx, Ny, Lx, Ly, Mx, My, M, L, m, n;
};

struct HostModel {
  std::vector<double> H0;      // m x m
  std::vector<double> Hd;      // compact nonzero H_0d blocks, n x n each
  std::vector<int> hd_index;   // per offset d = 1..M-1: block index or -1
};

// Options with the defaults of vemb_default_options filled in, validated.
int normalize_options(const vemb_options* in, vemb_options& o, std::string& err);
// Periodic lattice tiled by clusters of at most 4 sites, at least two clusters.
int parse_geometry(const vemb_lattice& lat, const vemb_clusters& cl, Geometry& g, std::string& err);
// fermionic: VEMB_FHOP hoppings allowed (Jordan-Wigner order per cluster and per pair), X / Y rejected.
int build_model(const vemb_hamiltonian& H, const Geometry& g, HostModel& out, std::string& err, bool fermionic = false);
void build_pauli1_tables(int L, OpTables& T);
// Adds coeff * (Pauli `pauli` at lattice site (x, y)) to the Hamiltonian of the cluster
// holding that site: Hc is M x m x m.  Real one-site operators only (X, Z).
int add_site_field(const Geometry& g, int x, int y, int pauli, double coeff, std::vector<double>& Hc,
                   std::string& err);
// Unique momenta k (one of each {k, -k}); twiddles M^{-1/2} exp(-2 pi i d.k/M) as
// interleaved complex [Ku][M]; weights 1 for self-conjugate k, 2 otherwise.
void build_momenta(const Geometry& g, std::vector<double>& tw, std::vector<double>& wk, int& Ku);

}  // namespace vemb
