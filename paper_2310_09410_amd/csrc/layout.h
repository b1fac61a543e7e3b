// LDS layout of one workgroup of the persistent sweep kernel. Used by the host
// planner (to size and balance parts) and by the kernel (to carve its dynamic
// shared memory), so both agree byte for byte.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define LDOPF_HD __host__ __device__
#else
#define LDOPF_HD
#endif

namespace ldopf {

struct LdsLayout {
    uint32_t W, bbar, xs[3], lam[3], v, t, xloc[4], ownp, crho, lo, hi, cnt;  // T arrays
    uint32_t slot_lo, slot_hi, slot_own;                                         // int32 per var
    uint32_t row_lvar, row_sub, copy_off, copy_rows, tk_sub, meta;                // index arrays
    uint32_t tk_m, row_m;  // uint2 per task / per row: operator offsets packed at load time
    uint32_t var_r0;       // u16 per var: the row of its first copy
    uint32_t red;                                                                // double [waves][4][8], then [8]
    uint32_t agg;          // double [waves][2]: the aggregated residual sums of each row wave
    uint32_t total;
};

LDOPF_HD inline uint32_t lds_align(uint32_t x) { return (x + 15u) & ~15u; }

// w: bytes of the bulk type (8 FP64, 4 FP32); counts of one part.
LDOPF_HD inline LdsLayout lds_layout(uint32_t w, uint32_t w_words, uint32_t rows, uint32_t tks,
                                     uint32_t vars, uint32_t subs, uint32_t waves) {
    LdsLayout L{};
    uint32_t o = 0;
    auto take = [&](uint32_t bytes) {
        uint32_t at = o;
        o = lds_align(o + bytes);
        return at;
    };
    L.W = take(w * w_words);
    L.bbar = take(w * rows);
    // state of the last sweeps: the test of sweep k is decided during the
    // global update of sweep k + 3, and a stop returns the state of sweep k
    // (x_s, lambda of sweeps k .. k + 2; x of sweeps k .. k + 3)
    for (int b = 0; b < 3; ++b) L.xs[b] = take(w * rows);
    for (int b = 0; b < 3; ++b) L.lam[b] = take(w * rows);
    L.v = take(w * rows);
    L.t = take(w * tks);
    for (int b = 0; b < 4; ++b) L.xloc[b] = take(w * vars);
    L.ownp = take(w * vars);
    L.crho = take(w * vars);
    L.lo = take(w * vars);
    L.hi = take(w * vars);
    L.cnt = take(w * vars);
    L.slot_lo = take(4 * vars);
    L.slot_hi = take(4 * vars);
    L.slot_own = take(4 * vars);
    L.row_lvar = take(2 * rows);
    L.row_sub = take(2 * rows);
    L.copy_off = take(2 * (vars + 1));
    L.copy_rows = take(2 * rows);
    L.tk_sub = take(2 * tks);
    L.meta = take(16 * subs);
    L.tk_m = take(8 * tks);
    L.row_m = take(8 * rows);
    L.var_r0 = take(2 * vars);
    L.red = take(8 * 8 * (4 * waves + 1));  // row sums of each wave's 4 rows, then the grid totals
    L.agg = take(8 * 2 * waves);
    L.total = o;
    return L;
}

}  // namespace ldopf
