// Argument blocks and launchers of nlist.hip (binning, sorting, records,
// neighbour lists).
#pragma once
#include "common.h"

namespace sibfa {

struct BinArgs {
  int n, periodic;
  int nc[3];
  double box[3], ibox[3];
  const double* xyz;     // caller order [n][3]
  const int* mol;        // caller order [n]
  int* cell_of;          // [n]
  int* cell_count;       // [ncell + 1], zeroed
  int* mol_count;        // [n], zeroed
  int* err;              // bit 2: molecule id out of range; bit 8: NaN/Inf position
};

struct RecArgs {
  int n, periodic;
  double box[3], ibox[3];
  const int* perm;       // sorted -> caller
  // caller-order inputs
  const double* xyz; const int* mol;
  const double* q; const double* dip; const double* quad;
  const double* alpha; const double* thole;
  double thole_default;
  // sorted outputs
  double4* sp; double4* sd; double4* sth; double2* sth2;
  float4* sp32; float4* sd32; float4* sth32; float2* sth232;
  double* sa;
  int* mol_s;
  int* inv_perm;
  int* is_pol;
  const int* pol_scan;
  int* polidx; int* polsite;
  double4* pp; float4* pp32; double* pa;
  double* alpha_s; double* ainv_s;
  int* err;              // bit 4: polarizability not positive definite
};

struct NlistArgs {
  int periodic;
  int nc[3];
  double box[3], ibox[3];
  double cutoff2;
  const int* cell_start;
  const double4* sp;
  const int* mol_s;
  const int* polidx;
  const int* mol_count;
  // all: pairs with r^2 < rsplit2 ("near") from the front of the row in
  // candidate order, the others from the back (entry cap - 1 - k holds the
  // k-th far pair); nc_all counts both, nc_near the near ones
  int* nb_all; int* nc_all; int cap_all;
  int* nc_near;
  double rsplit2;
  int* nb_in; int* nc_in; int cap_in;
  int* nb_pol; int* nc_pol; int cap_pol;
  int* nb_ipol; int* nc_ipol; int cap_ipol;
  // [cell] maxima of the four counts over the cell's sites, written by the
  // cell's wavefront (no atomics: one same-address atomic per wavefront
  // costs the launch more than the list build itself)
  int4* cellmax;
  int* err;              // bit 1: a molecule's sites not all within reach
};

void launch_bin(const BinArgs& a, hipStream_t s);
// out[0..3] = the maxima of cellmax over ncell cells
void launch_cellmax_reduce(const int4* cellmax, int ncell, int* out, hipStream_t s);
void launch_scatter(const int* cell_of, const int* cell_start, int* cursor, int* perm,
                    int n, hipStream_t s);
void launch_sort_cells(const int* cell_start, int ncell, int* perm, hipStream_t s);
void launch_sum_ints(const int* v, int n, unsigned long long* out, hipStream_t s);
// positions, multipoles and polarizability records in one pass (after a
// re-sort, when all three change)
void launch_rec_all(const RecArgs& a, hipStream_t s);
// out[0] = largest mean polarizability, out[1] = smallest Thole factor over
// the polarizable sites (after the polarizability records); 0 and +inf
// when none.
void launch_pol_extents(const RecArgs& a, double* out, hipStream_t s);
void launch_rec_mult(const RecArgs& a, hipStream_t s);
void launch_rec_pol(const RecArgs& a, hipStream_t s);
void launch_rec_polsites(const RecArgs& a, hipStream_t s);
void launch_nlist(const NlistArgs& a, int ncell, hipStream_t s);

}  // namespace sibfa
