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

int build_model(const vemb_hamiltonian& H, const Geometry& g, HostModel& out, std::string& err);
void build_pauli1_tables(int L, OpTables& T);
// Unique momenta k (one of each {k, -k}); twiddles M^{-1/2} exp(-2 pi i d.k/M) as
// interleaved complex [Ku][M]; weights 1 for self-conjugate k, 2 otherwise.
void build_momenta(const Geometry& g, std::vector<double>& tw, std::vector<double>& wk, int& Ku);

}  // namespace vemb
