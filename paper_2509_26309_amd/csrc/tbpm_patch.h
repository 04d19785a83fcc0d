// Patch reordering of a sparse Hamiltonian (see tbpm_patch.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace tbpm {

struct PatchPlan {
    std::vector<int32_t> new_of_old;   // [n] new index of each original row
    std::vector<int32_t> old_of_new;   // [n] original row of each new index
    std::vector<int32_t> patch_ptr;    // [npatch+1] first new row of each patch
    std::vector<int64_t> halo_ptr;     // [npatch+1] into halo_rows
    std::vector<int32_t> halo_rows;    // new indices, ascending within a patch
    int max_halo = 0;
    double halo_fraction = 0.0;        // sum of halo sizes / n
};

// Plans patches of at most max_rows rows; false when some halo exceeds
// max_halo (the plan is still filled in for inspection).
bool plan_patches(int64_t n, const int64_t *rp, const int32_t *col, int max_rows, int max_halo, PatchPlan &plan);

}  // namespace tbpm

namespace tbpm {

// Layered halos of a patch plan, for fusing K = depth + 1 Chebyshev terms:
// layer 1 = rows outside the patch referenced by patch rows; layer l + 1 =
// rows outside the patch and layers <= l referenced by layer-l rows.  Per
// patch the halo list holds layer 1 (ascending), then layer 2, ...; the
// key list holds the same rows ascending with their position in the halo
// list, for lookups.
struct LayerPlan {
    int depth = 0;
    std::vector<int64_t> halo_ptr;     // [npatch+1]
    std::vector<int32_t> halo_rows;    // new indices, layer by layer
    std::vector<int32_t> layer_cnt;    // [npatch][depth]
    std::vector<int32_t> key_rows;     // per patch, ascending
    std::vector<int32_t> key_pos;      // position of key_rows[i] in the patch's halo list
    int max_halo = 0;                  // largest halo (all layers) of a patch
    double halo_fraction = 0.0;        // total halo rows / n
};

// Uses the patches of `plan` (computed by plan_patches) and the original CSR.
void plan_layers(int64_t n, const int64_t *rp, const int32_t *col, const PatchPlan &plan, int depth,
                 LayerPlan &out);

}  // namespace tbpm
