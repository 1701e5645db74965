// Groups of BCSR row blocks that share columns (host, plan time).
//
// Every tile of the BCSR-part gathers one row of the dense operand, and a
// row block's tiles serve only its own B_r rows.  Neighbouring row blocks
// of a mesh or banded matrix need many of the same rows (a 9-point stencil's
// row block shares two of its three grid rows of columns with the row
// blocks above and below it).  The group kernels load each column that two
// or more tiles of a group use once into LDS and let all of those tiles
// read it there; a column used by one tile of the group is gathered
// directly, as before.
#pragma once

#include <cstdint>
#include <vector>

namespace hspmm {

struct GroupParams {
    int u_max = 144;         // most shared columns a group may stage (LDS rows)
    int g_max = 8;           // most row blocks in a group
    int hub_cap = 64;        // columns used by more row blocks do not propose candidates
    double min_share = 0.25; // a candidate must find this share of its tiles' columns in the group
    bool stage_all = true;   // stage every column of the group (else only shared ones)
};

struct Groups {
    std::vector<int32_t> order;    // row-block slots in kernel order (groups contiguous)
    std::vector<int32_t> grp_ptr;  // [ngroups + 1]: groups as ranges of `order`
    std::vector<int32_t> u_ptr;    // [ngroups + 1]: ranges of `ucol`
    std::vector<int32_t> ucol;     // shared columns of each group, ascending
    std::vector<int32_t> bsrc;     // per stored tile (padded layout): >= 0 row of the group's LDS
                                   // stage, < 0 column -(v + 1) gathered directly
    int64_t staged_tiles = 0;      // tiles reading their row from LDS
    int64_t max_u = 0;             // largest group stage
    int64_t ngroups() const { return (int64_t)grp_ptr.size() - 1; }
};

// blk_ptr[s] / blk_cnt[s]: first stored tile and number of real tiles of
// slot s (tiles are padded after blk_cnt up to the next slot's blk_ptr or
// nblk_pad); blk_col: column of every stored tile (padding tiles: any).
// Slots are visited as seeds in increasing order; each grows greedily by the
// unassigned slot with the most columns already in the group (ties: lowest
// slot), while that slot finds at least min_share of its columns there,
// the stage stays within u_max rows and the group within g_max slots.
// The stage holds every column of the group's tiles (stage_all) or only
// the columns two or more of its tiles share (the others are gathered
// directly by their tiles).
void build_groups(const std::vector<int32_t>& blk_ptr, const std::vector<int32_t>& blk_cnt,
                  const std::vector<int32_t>& blk_col, int64_t nblk_pad, int64_t k, const GroupParams& prm,
                  Groups& out);

}  // namespace hspmm
