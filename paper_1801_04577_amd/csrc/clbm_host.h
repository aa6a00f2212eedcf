// clbm_host.h -- host-side parameter derivation shared by the single-lattice and
// batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>

#include "../../include/clbm.h"
#include "clbm_device.h"

namespace clbm {

#define CLBM_HIP(call)                                    \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) {                           \
            set_last_hip_error(e_, #call, __FILE__, __LINE__); \
            return CLBM_ERR_HIP;                          \
        }                                                 \
    } while (0)

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line);

constexpr size_t kAlign = 256;   // workspace region alignment, bytes

// Two steps per launch: tiles of kBlock x kTwoStepRows nodes, kTwoStepThreads threads.
constexpr int kTwoStepRows = 14;
constexpr int kTwoStepThreads = 512;
// FP16 storage: taller tiles of 22 rows, three rows (with the halo) per wave of a
// 512-thread workgroup: half the LDS per node, and 4.6% fewer ring nodes recomputed.
constexpr int kTwoStepRowsF16 = 22;

// Tile heights of the two-step kernel (kBlock columns) and their workgroup sizes: the
// rows + 2 halo rows are dealt to the waves, two rows per wave (6, 14, 30 rows: 256, 512,
// 1024 threads) or three (22 rows: 512 threads).
inline bool two_step_rows_ok(int rows) { return rows == 6 || rows == 14 || rows == 22 || rows == 30; }
inline int two_step_threads(int rows) { return rows == 6 ? 256 : rows == 30 ? 1024 : 512; }

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Rates {
    double s_nu, s_b, s_3, s_4, l0, l1, l2;
};

// Relaxation rates: Sec. 2.1 (nu), Eq. (8) defaults, Sec. 3 no-slip rule for s_3,
// Sec. 2.2 (alpha, c_T^2 = 2/5), Sec. 3.1 rule for lambda_2.
clbm_status derive_rates(const clbm_params* p, Rates* r);
// Full validation of a parameter block (sizes, sides, finite values, rates).
clbm_status validate(const clbm_params* p, Rates* r);
// Kernel constant block for a validated parameter block.
LatticeConst make_const(const clbm_params* p, const Rates& r);
// Elements of one stored row (ceil(nx / kBlock) blocks of 14 populations) and of one
// population buffer (ny rows).
size_t row_elems(int nx);
size_t buffer_elems(int nx, int ny);
// One-dimensional grid of blk-shaped blocks covering a lattice, for the per-node kernels
// (grid_node decodes a block index into its nodes).
dim3 node_grid(const LatticeConst& c, dim3 blk);

}  // namespace clbm
