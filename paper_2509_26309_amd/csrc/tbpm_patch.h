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
