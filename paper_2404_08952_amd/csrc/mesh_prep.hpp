// Host-side mesh preparation: validation, locality renumbering, partitions.
//
// The finite-volume mesh is face addressed (Sec. 2.1): a cell knows its
// neighbours only through shared faces.  For the device kernels the cells are
// renumbered (reverse Cuthill-McKee or a Hilbert space-filling curve) and cut
// into contiguous partitions of at most B cells.  Each partition owns the list
// of faces ("entries") touching any of its cells; faces on a partition seam
// appear in both partitions.  A cell addresses its faces through "slots":
// (local entry index, side) pairs, side 0 = owner (sigma = +1), 1 = neighbour.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dolinc.h"

namespace dolinc {

struct Prepared {
  int dim = 0;
  int64_t n_cells = 0, n_faces = 0, n_nodes = 0;
  int64_t n_interior = 0;              // caller cells; rows n_interior.. are auxiliary cells
  int part_cells = 256;
  std::vector<int32_t> new_of_old, old_of_new;
  // partitions
  int64_t n_parts = 0;
  std::vector<int32_t> part_ent_ptr;   // [n_parts + 1]
  std::vector<int32_t> ent_face;       // [n_entries] caller face id
  std::vector<int32_t> ent_p, ent_n;   // [n_entries] internal cell ids (owner, neighbour)
  std::vector<int32_t> face_first_ent; // [n_faces] one entry of every face
  std::vector<int32_t> slot_ptr;       // [n_cells + 1] (internal order)
  std::vector<uint16_t> slots;         // local entry | side << 15
  // per slot: 2 * e + side for the face's entry e in the partition across a
  // seam (the same face seen from the other cell's partition), else -1
  std::vector<int32_t> slot_twin;
  int64_t max_entries = 0, max_cell_faces = 0;
};

// A mesh description with non-coupled boundary faces turned into two-cell
// faces: the k-th boundary face (in face order) gets the auxiliary cell
// n_cells + k as its neighbour (zero shift).  Owns the arrays it points to.
struct ExtendedDesc {
  dolinc_mesh_desc d{};
  std::vector<int32_t> nei;
  std::vector<double> shift;
  std::vector<int32_t> bface;  // caller face of auxiliary cell k
  int64_t n_interior = 0;
};
dolinc_status extend_desc(const dolinc_mesh_desc& in, ExtendedDesc& X, std::string& msg);

// Returns DOLINC_OK or an error; msg receives a description.  Cells from
// n_interior on (default: none) are auxiliary cells: they need not be
// closed and keep their indices (after the renumbered interior cells).
dolinc_status prepare_mesh(const dolinc_mesh_desc& d, Prepared& out, std::string& msg, int64_t n_interior = -1);

// Renumbering helpers (exposed for tests through dolinc_mesh_prepare).
void rcm_order(int64_t n, const std::vector<int64_t>& adj_ptr, const std::vector<int32_t>& adj,
               std::vector<int32_t>& new_of_old);
void hilbert_order(int dim, int64_t n, const std::vector<double>& pts, std::vector<int32_t>& new_of_old);

}  // namespace dolinc
