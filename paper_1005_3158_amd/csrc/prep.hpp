// Host preprocessing of the casting step: validation, lumping, boundary
// aggregation, stability bound, locality reordering, colouring and the
// LDS element blocks with private/shared node classes.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/castfem.h"

namespace castfem {

struct Problem {
    int nen = 0;
    int64_t N = 0, E = 0;
    std::vector<double> xyz;
    std::vector<int32_t> conn, emat;
    std::vector<fem_material> mats;
    std::vector<int32_t> dir_nodes;
    std::vector<double> dir_T;
    int npf = 3;
    std::vector<int32_t> flux_faces;
    std::vector<double> flux_q, flux_h, flux_Tinf;
    std::vector<int32_t> if_a, if_b;
    std::vector<double> if_h;
    std::vector<int32_t> contact_faces, contact_side;   // non-matching contact: triangles and their side
    std::vector<double> contact_h;
    std::vector<double> T0;
    int32_t n_scen = 1;
    std::vector<int32_t> mat_scen;    // scenario of every material (empty: all in scenario 0)
    int32_t scen_of_mat(int32_t m) const { return mat_scen.empty() ? 0 : mat_scen[m]; }
};

// node flag bits stored next to the material id; NODE_XTRA: a shared node in
// more than PARTIAL_SLOTS blocks (it has partials beyond the slot-major ones)
enum : uint32_t { NODE_FIXED = 1u << 31, NODE_BC = 1u << 30, NODE_XTRA = 1u << 29, NODE_MAT_MASK = 0xFFFFu };

// partial residuals per shared node held slot-major (the rest go to a list)
constexpr int PARTIAL_SLOTS = 4;

struct BlockInfo {        // one LDS element block (10 ints, 40 bytes)
    int32_t e_begin;      // first element of the block (blocked element order)
    int32_t n_e;          // elements in the block
    int32_t int_base;     // first global id of its private nodes (contiguous)
    int32_t n_int;        // private nodes: local ids 0..n_int-1
    int32_t sh_begin;     // offset of its shared-node list (and partial slots)
    int32_t n_sh;         // shared nodes: local ids n_int..n_int+n_sh-1
    int32_t pad0, pad1;   // pad0: in the apparent-capacity form, the block's one material or -1
    int32_t v_begin;      // first interface pair of the block (Layout::vconn), with
    int32_t n_v;          // ... the number of them (interface pairs as block elements)
};

struct Layout {
    int nen = 0;
    int64_t N = 0, E = 0;
    // numbering: perm[original] = new id, iperm[new] = original
    std::vector<int32_t> perm, iperm;
    // nodes in new numbering
    std::vector<double> xyz;          // N x 3
    std::vector<uint32_t> nflag;      // material | NODE_FIXED | NODE_BC (Robin or interface terms)
    std::vector<double> m;            // lumped capacitance weights (kg)
    std::vector<double> T_init;       // initial temperature after fixed values
    // elements in new order, node ids in new numbering
    std::vector<int32_t> conn;
    // boundary terms per "bc slot" (all nodes, or shared nodes when blocked):
    // r_i += robin_a - robin_b T_i + sum_k w_k (T_{j_k} - T_i)
    int64_t bc_first = 0;             // node id of slot 0 (0, or the first shared node)
    int64_t n_bc_slots = 0;
    std::vector<double> robin_a, robin_b;  // per slot (empty if no flux faces)
    std::vector<int32_t> link_ptr;    // per slot + 1
    std::vector<int32_t> link_node;
    std::vector<double> link_w;
    // colouring
    std::vector<int32_t> color_ptr;   // elements of colour c: [color_ptr[c], color_ptr[c+1])
    // LDS blocks
    std::vector<BlockInfo> blocks;
    int64_t n_private = 0;            // nodes 0..n_private-1 are private to one block
    int64_t n_inflow = 0;             // node-kernel slots 0..n_inflow-1 may carry boundary inflow
    // node ranges of one scenario each (at most SEG_NODES long) for the
    // deterministic per-scenario state reductions
    std::vector<int32_t> seg_begin;   // n_seg + 1
    std::vector<int32_t> seg_scen;    // n_seg
    std::vector<int32_t> sh_list;     // per block: global ids of its shared nodes
    std::vector<uint16_t> lconn;      // per element: local ids in its block
    // tets in blocks of at most 4096 nodes: the same ids packed 12 bits each, two
    // tets per three 32-bit words (tet 2p in bits 0-47 of words 3p..3p+2, tet
    // 2p+1 in bits 48-95); empty otherwise
    std::vector<uint32_t> lconn12;
    // interface pairs as block elements: six local ids (face a, then face b) and
    // the coupling w per pair, in block order
    std::vector<uint16_t> vconn;
    std::vector<double> vw;
    // partials of shared node s: slot j < PARTIAL_SLOTS at j * nsh + s, the
    // others at PARTIAL_SLOTS * nsh + [comb_ptr[s], comb_ptr[s+1]), all in block order
    std::vector<int32_t> comb_ptr;
    std::vector<int32_t> sh_pos;      // per sh_list entry: where that block writes its partial
    int64_t n_partial_slots = 0;      // size of the partial array (unused slots hold zero)
    std::vector<uint8_t> xtra;        // per node (final numbering): NODE_XTRA
    int64_t max_local = 0;
    // report
    double dt_bound = 0;
    int64_t bw_before = 0, bw_after = 0;
    double setup_seconds = 0;
    int64_t block_elems = 0;
};

constexpr int SEG_NODES = 1024;

struct PrepOptions {
    int ordering = FEM_ORDER_HILBERT;
    int scatter = FEM_SCATTER_LDS_BLOCKED;
    int64_t block_elems = 8192;
    int64_t max_local_nodes = 2600;
    bool color_in_block = true;       // order each block's elements by a local colouring
    // matched interface pairs (fem_set_interface) as six-node elements of the LDS
    // blocks instead of node links of the node kernel (enthalpy step)
    bool interface_in_blocks = false;
};

// Throws std::runtime_error with a message; the C interface maps it to a code.
struct PrepError {
    int code;
    std::string msg;
};

// Validation, lumping, boundary aggregation and the stability bound; the parts
// that do not depend on the ordering.  Fills per-node data in input numbering.
struct Base {
    std::vector<int32_t> nmat;        // material of every node
    std::vector<double> m;            // lumped weights
    std::vector<double> robin_a, robin_b;
    std::vector<uint8_t> fixed;
    std::vector<double> T_init;
    // aggregated interface links in input numbering, CSR by node
    std::vector<int32_t> lptr, lnode;
    std::vector<double> lw;
    // the links of the non-matching contact faces alone (the same form)
    std::vector<int32_t> clptr, clnode;
    std::vector<double> clw;
    // per matched interface pair: its coupling w = h A / 9 of every node pair
    std::vector<double> pair_w;
    double dt_bound = 0;
    bool any_robin = false;
    std::vector<double> dt_scen;      // stability bound of every scenario
    std::vector<double> kabs;         // sum_j |K_ij| of the assembled conduction operator per node
    std::vector<int32_t> sisters;     // per contact face: the closest face of the other side
    double sister_seconds = 0;        // host time of the sister search
    double elem_abs_max = 0;          // max_i sum_{e at i} sum_j |K^e_ij|  (W/K)
    double T_span = 1;                // span of initial, fixed and ambient temperatures (K)
};

// node permutation (perm[original] = rank) and element order of a locality ordering
struct Ordering {
    std::vector<int32_t> perm;
    std::vector<int64_t> eorder;
    // the sort key of every element in eorder (scenario, locality key), and the
    // matched interface pairs in the same order of keys
    std::vector<uint64_t> escen, ekey;
    std::vector<int64_t> porder;
    std::vector<uint64_t> pscen, pkey;
};

void prep_base(const Problem &p, Base &b);                                     // throws PrepError
void prep_order(const Problem &p, const Base &b, int ordering, Ordering &ord);  // throws PrepError
void prep_layout(const Problem &p, const Base &b, const PrepOptions &o, const Ordering &ord,
                 Layout &L);                                                    // throws PrepError
int64_t bandwidth(const Problem &p, const Base &b, const std::vector<int32_t> *perm);

// Sister of every contact face: the face of the other side in the same scenario
// whose centroid is nearest (squared distance in FP64, ties to the lower index).
void contact_sisters(const Problem &p, const std::vector<int32_t> &nmat, std::vector<int32_t> &sister);  // throws

// orderings (exposed for testing through the C interface report)
std::vector<int32_t> order_rcm(const Problem &p, const Base &b);
std::vector<int32_t> order_sfc(const Problem &p, bool hilbert);

}  // namespace castfem
