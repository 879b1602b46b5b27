// Dispatch table: measured T0 per variant, best-of-N, T1 (pad) and T2 (split + pad) with a plan
// record per grid cell (paper Sec. 7.1).
#pragma once

#include <stdint.h>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/smoothgemm.h"

struct sg_table {
    sg_grid grid{};
    int nvar = 0;
    std::vector<int> variants;      // variant id of each T0 row
    std::vector<double> T0;         // nvar x cells, seconds
    std::vector<double> T0best;     // cells: min over variants
    std::vector<int> best_var;      // cells: argmin variant id
    std::vector<double> T1, T2;     // cells
    std::vector<uint8_t> action;    // cells: SG_ACT_*
    std::vector<int32_t> arg;       // cells: pad target (flat) or split point (steps)
    // fingerprint
    std::string device;             // "<name>|<gcnArchName>" or "host" when built from given T0
    int cus = 0;
    int hip_runtime = 0;
    int c_dtype = -1;               // output type the timings were measured with (-1 unknown)
    // Grouped-launch schedules found by the grouped autotuner, keyed by a hash of the group's
    // problem list: later plans of the same group take the schedule by lookup instead of
    // timing candidates again.  Saved and loaded with the table.
    struct GroupSched { int tile, grid_wgs, order; double seconds; };
    mutable std::mutex group_mu;
    mutable std::unordered_map<uint64_t, GroupSched> group_sched;

    int64_t cells() const { return (int64_t)grid.n_m * grid.n_n * grid.n_k; }
    int64_t cell_index(int m, int n, int k) const {
        return ((int64_t)m * grid.n_n + n) * grid.n_k + k;
    }
    void cell_coords(int64_t c, int* m, int* n, int* k) const {
        *k = (int)(c % grid.n_k);
        *n = (int)((c / grid.n_k) % grid.n_n);
        *m = (int)(c / ((int64_t)grid.n_k * grid.n_n));
    }
    // Whether (M, N, K) is a grid point: every dimension a multiple of the step.
    bool on_grid(int64_t M, int64_t N, int64_t K) const {
        const int64_t g = grid.step;
        return M % g == 0 && N % g == 0 && K % g == 0;
    }
    // Cell whose size covers (M, N, K): ceil(dim / step) - 1 per axis; false if beyond the grid.
    bool covering_cell(int64_t M, int64_t N, int64_t K, int* m, int* n, int* k) const {
        const int64_t g = grid.step;
        int64_t cm = (M + g - 1) / g - 1, cn = (N + g - 1) / g - 1, ck = (K + g - 1) / g - 1;
        if (cm < 0) cm = 0;
        if (cn < 0) cn = 0;
        if (ck < 0) ck = 0;
        if (cm >= grid.n_m || cn >= grid.n_n || ck >= grid.n_k) return false;
        *m = (int)cm; *n = (int)cn; *k = (int)ck;
        return true;
    }
};

namespace sg {
// Fill T0best/best_var/T1/T2/action/arg from T0.
int build_dp(sg_table* t);
// T0 of variant row `row` interpolated at (M, N, K) (trilinear between the bracketing cells,
// clamped to the grid), and the T0 row of a variant id (-1 if the table has none).
double t0_interp(const sg_table* t, int row, int64_t M, int64_t N, int64_t K);
int variant_row(const sg_table* t, int variant);
int measure_t0(struct ::sg_ctx* ctx, const std::vector<sg_shape>& order,
               const std::vector<int64_t>& cells, const int* variants, int nvar, int c_dtype,
               int warmup, int reps, const void* A_pool, const void* B_pool, void* C_pool,
               hipStream_t s, std::vector<double>& T0, int64_t ncells);
}  // namespace sg
