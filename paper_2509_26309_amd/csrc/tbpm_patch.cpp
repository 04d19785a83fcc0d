// Patch reordering of a sparse Hamiltonian (host side).
//
// Two Chebyshev terms can share one pass over H when the intermediate vector
// of the first term is kept on chip for the rows the second term needs.  For
// that, rows are grouped into patches: a patch is a set of at most S rows
// grown by breadth-first search over the sparsity graph (so on a lattice it
// is a compact region), and its halo is every row outside the patch that a
// patch row references.  Rows are renumbered patch by patch (each patch is a
// contiguous index range; inside it, the rows bordering each neighbouring
// patch are kept together), so the permuted matrix is H' = P H P^T; the
// propagation of P psi0 under H' gives the same C(t).
//
// Seeds: the next patch starts from an unassigned row adjacent to the
// previous patch when there is one (patches then sweep the lattice as a
// front), otherwise from the lowest unassigned row.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "tbpm_patch.h"

namespace tbpm {

// Orders the rows of each patch so that the rows another patch reads as its
// halo are contiguous.  Row i of patch P gets the key (q, d, i): d = 1 and q =
// the lowest other patch adjacent to i; else d = 2 and q = the lowest q of
// i's d = 1 neighbours in P; else d = 3 (interior).  The halo of a
// neighbouring patch Q is then the run of P's rows with q = Q (plus corner
// rows assigned to a lower q), and Q's second layer follows it, so halo reads
// touch few partly used memory lines (on graphene 1.3x the useful bytes at
// 64-byte lines instead of 2.5x in breadth-first order).
static void group_boundary_rows(const int64_t *rp, const int32_t *col, const std::vector<int32_t> &patch_ptr,
                                std::vector<int32_t> &new_of_old, std::vector<int32_t> &old_of_new)
{
    const int64_t n = (int64_t)old_of_new.size();
    const int64_t npatch = (int64_t)patch_ptr.size() - 1;
    std::vector<int32_t> patch_of((size_t)n);
    for (int64_t p = 0; p < npatch; ++p)
        for (int32_t i = patch_ptr[(size_t)p]; i < patch_ptr[(size_t)p + 1]; ++i)
            patch_of[(size_t)i] = (int32_t)p;
    const int64_t none = INT64_MAX;
    std::vector<int64_t> q1((size_t)n, none);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t v = old_of_new[(size_t)i];
        for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
            const int32_t pc = patch_of[(size_t)new_of_old[(size_t)col[k]]];
            if (pc != patch_of[(size_t)i])
                q1[(size_t)i] = std::min<int64_t>(q1[(size_t)i], pc);
        }
    }
    struct Key {
        int64_t q;
        int32_t d, i;
    };
    std::vector<Key> keys;
    std::vector<int32_t> reordered((size_t)n);
    for (int64_t p = 0; p < npatch; ++p) {
        const int32_t b = patch_ptr[(size_t)p], e = patch_ptr[(size_t)p + 1];
        keys.clear();
        for (int32_t i = b; i < e; ++i) {
            if (q1[(size_t)i] != none) {
                keys.push_back({q1[(size_t)i], 1, i});
                continue;
            }
            int64_t q2 = none;
            const int32_t v = old_of_new[(size_t)i];
            for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
                q2 = std::min(q2, q1[(size_t)new_of_old[(size_t)col[k]]]);
            keys.push_back({q2, q2 != none ? 2 : 3, i});
        }
        std::sort(keys.begin(), keys.end(), [](const Key &x, const Key &y) {
            return x.q != y.q ? x.q < y.q : x.d != y.d ? x.d < y.d : x.i < y.i;
        });
        for (int32_t j = b; j < e; ++j)
            reordered[(size_t)j] = old_of_new[(size_t)keys[(size_t)(j - b)].i];
    }
    old_of_new.swap(reordered);
    for (int64_t i = 0; i < n; ++i)
        new_of_old[(size_t)old_of_new[(size_t)i]] = (int32_t)i;
}

bool plan_patches(int64_t n, const int64_t *rp, const int32_t *col, int max_rows, int max_halo, PatchPlan &plan)
{
    plan = PatchPlan();
    if (n <= 0 || max_rows < 1)
        return false;
    std::vector<int32_t> new_of_old((size_t)n, -1);
    std::vector<int32_t> old_of_new;
    old_of_new.reserve((size_t)n);
    std::vector<int32_t> patch_ptr;
    patch_ptr.push_back(0);
    std::vector<int32_t> queue;
    queue.reserve((size_t)max_rows);
    int64_t low = 0;              // lowest possibly unassigned row
    int32_t next_seed = -1;       // unassigned neighbour of the previous patch
    while ((int64_t)old_of_new.size() < n) {
        const int32_t pstart = (int32_t)old_of_new.size();
        int32_t count = 0;
        int32_t seed = next_seed;
        next_seed = -1;
        while (count < max_rows && (int64_t)old_of_new.size() < n) {
            if (seed < 0 || new_of_old[(size_t)seed] >= 0) {
                while (low < n && new_of_old[(size_t)low] >= 0)
                    ++low;
                if (low >= n)
                    break;
                seed = (int32_t)low;
            }
            // breadth-first growth from `seed`
            queue.clear();
            queue.push_back(seed);
            new_of_old[(size_t)seed] = pstart + count;
            old_of_new.push_back(seed);
            ++count;
            for (size_t qi = 0; qi < queue.size(); ++qi) {
                const int32_t v = queue[qi];
                for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
                    const int32_t u = col[k];
                    if (new_of_old[(size_t)u] >= 0)
                        continue;
                    if (count >= max_rows) {
                        if (next_seed < 0)
                            next_seed = u;
                        continue;
                    }
                    new_of_old[(size_t)u] = pstart + count;
                    old_of_new.push_back(u);
                    queue.push_back(u);
                    ++count;
                }
            }
            seed = -1;
        }
        patch_ptr.push_back((int32_t)old_of_new.size());
    }
    const int64_t npatch = (int64_t)patch_ptr.size() - 1;
    group_boundary_rows(rp, col, patch_ptr, new_of_old, old_of_new);

    // halos: rows outside the patch referenced by its rows (new indices, sorted)
    std::vector<int64_t> halo_ptr((size_t)npatch + 1, 0);
    std::vector<int32_t> halo_rows;
    std::vector<int32_t> tmp;
    int64_t halo_total = 0;
    int max_h = 0;
    for (int64_t p = 0; p < npatch; ++p) {
        const int32_t b = patch_ptr[(size_t)p], e = patch_ptr[(size_t)p + 1];
        tmp.clear();
        for (int32_t i = b; i < e; ++i) {
            const int32_t v = old_of_new[(size_t)i];
            for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
                const int32_t c = new_of_old[(size_t)col[k]];
                if (c < b || c >= e)
                    tmp.push_back(c);
            }
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        max_h = std::max(max_h, (int)tmp.size());
        halo_total += (int64_t)tmp.size();
        halo_rows.insert(halo_rows.end(), tmp.begin(), tmp.end());
        halo_ptr[(size_t)p + 1] = (int64_t)halo_rows.size();
    }
    plan.new_of_old = std::move(new_of_old);
    plan.old_of_new = std::move(old_of_new);
    plan.patch_ptr = std::move(patch_ptr);
    plan.halo_ptr = std::move(halo_ptr);
    plan.halo_rows = std::move(halo_rows);
    plan.max_halo = max_h;
    plan.halo_fraction = (double)halo_total / (double)n;
    return max_h <= max_halo;
}

}  // namespace tbpm
