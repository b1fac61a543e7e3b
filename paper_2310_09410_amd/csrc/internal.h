// Internal declarations shared by the host side (assembly, planning, C ABI)
// and the device side (precompute and sweep kernels) of libldopf.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldopf.h"

namespace ldopf {

// Error carrying an ldopf_code; thrown inside the library, turned into a
// return code (plus thread-local detail text) at the C boundary.
struct Error {
    int code;
    std::string detail;
};
[[noreturn]] void fail(int code, const std::string& detail);

// The consensus LP of OurModel in host memory: globals (c, lo, hi, start
// value), and per subsystem a dense row-major A_s, b_s and its ascending
// global indices. Subsystem s owns copies [loc_off[s], loc_off[s+1]), rows
// [row_off[s], row_off[s+1]) and A words [a_off[s], a_off[s+1]).
struct ConsensusLP {
    int64_t n = 0;
    std::vector<double> c, lo, hi, x_init;
    int64_t S = 0;
    std::vector<int32_t> ns, ms;
    std::vector<int64_t> loc_off, row_off, a_off;
    std::vector<double> A, b;
    std::vector<int64_t> gidx;
    // Load scaling (network path only): for each row, the load whose
    // reference powers it carries (-1: none) and the local column of its
    // squared-voltage coefficient (-1: none). Scaling load l by f multiplies
    // that row's right-hand side and that coefficient by f.
    std::vector<int32_t> row_load, row_wcol;
    int32_t n_load = 0;
    // Optional order in which subsystems sit next to each other in the network
    // (a depth-first walk of the feeder); used to cut the problem into
    // workgroup parts that share few variables. Empty: input order.
    std::vector<int64_t> locality_order;
};

// Network -> consensus LP (Section II-A rows, Section V-A decomposition).
ConsensusLP assemble_network(const ldopf_network& net);
// Check an LP given directly (sizes, B_s invariants, bounds) and fill offsets.
void finish_lp(ConsensusLP& lp);

// Largest subsystem the device path takes (columns per lane of the
// precompute, 12-bit fields of the sweep's packed row words).
constexpr int kMaxSubsystemVars = 1024;

// ---------------------------------------------------------------------------
// Work partition of the persistent sweep kernel. Each part is one workgroup
// that keeps its subsystems' operators and state resident in LDS.

// Per subsystem inside a part (device order). The first 16 bytes are what the
// kernel keeps in LDS; basis/brow are only read while loading the part.
struct SubMeta {
    uint64_t basis;  // global word offset of the subsystem's n x n basis
    uint32_t w0;     // first operator word inside the part
    uint32_t canon;  // canonical subsystem index
    uint32_t brow;   // first basis row taken (0 or rank)
    uint16_t row0;   // first local row (copy) of the subsystem inside the part
    uint16_t n;      // n_s
    uint16_t k;      // K_s rank-form vectors
    uint16_t t0;     // first slot of the subsystem in the part's t buffer
    uint16_t mode;   // 1: y = bbar + v - W'(W v); 0: y = bbar + W'(W v)
    uint16_t pad;
};
static_assert(sizeof(SubMeta) == 32, "SubMeta layout");

struct PartInfo {
    int32_t sub_begin, n_sub;   // into the SubMeta array
    int32_t row_begin, n_row;   // into the row arrays
    int32_t var_begin, n_var;   // into the var arrays
    int32_t tk_begin, n_tk;     // into the (sub, k) task map
    int32_t w_words;            // operator words held in LDS
    int32_t copy_begin;         // into var_copy_rows
    int32_t lds_bytes;          // LDS this part needs
    int32_t coff_begin;         // into var_copy_off (n_var + 1 entries per part)
};

struct Plan {
    int32_t n_parts = 0;
    int32_t block_threads = 0;
    int64_t lds_bytes = 0;      // max over parts
    std::vector<PartInfo> parts;
    std::vector<SubMeta> subs;
    std::vector<int32_t> row_canon;    // canonical copy index of each device row
    std::vector<uint16_t> row_lvar;    // part-local var of each device row
    std::vector<uint16_t> row_sub;     // part-local subsystem of each device row
    std::vector<int32_t> var_gid;      // global id of each part-local var
    std::vector<int32_t> var_slot;     // boundary var: this part's owner index; -1 interior
    std::vector<int32_t> var_slot_lo;  // boundary var: slot base (m^2 slots, reader-major); -1 interior
    std::vector<int32_t> var_slot_hi;  // boundary var: number of owner parts m
    std::vector<uint8_t> var_writer;   // 1 if this part writes the var to the output x
    std::vector<uint16_t> var_copy_off;  // per part: n_var + 1 offsets into var_copy_rows
    std::vector<uint16_t> var_copy_rows; // part-local rows holding a copy, grouped by var
    std::vector<uint16_t> tk_sub;      // part-local subsystem of each (s, k) task
    int32_t n_slots = 0;               // boundary (var, writer part, reader part) slots
    int64_t rank_words = 0;
};

// Build the partition for given ranks (from the device precompute).
Plan make_plan(const ConsensusLP& lp, const std::vector<int32_t>& rank, bool fp32,
               int32_t rows_per_part, int32_t block_threads, int32_t max_parts,
               int64_t max_lds_bytes);

}  // namespace ldopf
