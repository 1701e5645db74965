// Greedy grouping of BCSR row blocks by shared columns (host arithmetic).
#include "group.h"

#include <algorithm>

namespace hspmm {

void build_groups(const std::vector<int32_t>& blk_ptr, const std::vector<int32_t>& blk_cnt,
                  const std::vector<int32_t>& blk_col, int64_t nblk_pad, int64_t k, const GroupParams& prm,
                  Groups& out) {
    const int64_t ns = (int64_t)blk_cnt.size();
    out = Groups{};
    out.grp_ptr.assign(1, 0);
    out.u_ptr.assign(1, 0);
    out.bsrc.assign((size_t)nblk_pad, -1);
    if (ns == 0) return;

    // the slots that use each column (a counting sort of the real tiles)
    std::vector<int32_t> cptr((size_t)k + 1, 0);
    for (int64_t s = 0; s < ns; ++s)
        for (int32_t t = 0; t < blk_cnt[s]; ++t) ++cptr[(size_t)blk_col[(size_t)blk_ptr[s] + t] + 1];
    for (int64_t c = 0; c < k; ++c) cptr[c + 1] += cptr[c];
    std::vector<int32_t> cslots((size_t)cptr[k]);
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t s = 0; s < ns; ++s)
            for (int32_t t = 0; t < blk_cnt[s]; ++t) cslots[fill[blk_col[(size_t)blk_ptr[s] + t]]++] = (int32_t)s;
    }

    // per column: tiles of the current group using it (stamped by group id);
    // per slot: columns it shares with the current group (stamped)
    std::vector<int32_t> col_stamp((size_t)k, -1), col_cnt((size_t)k, 0), col_local((size_t)k, -1);
    std::vector<int32_t> slot_stamp((size_t)ns, -1), score((size_t)ns, 0);
    std::vector<uint8_t> assigned((size_t)ns, 0);
    std::vector<int32_t> cands, members, shared;
    out.order.reserve((size_t)ns);

    int32_t gid = 0;
    for (int64_t seed = 0; seed < ns; ++seed, ++gid) {
        if (assigned[seed]) {
            --gid;
            continue;
        }
        members.clear();
        cands.clear();
        const int need = prm.stage_all ? 1 : 2;  // tiles of the group that make a column staged
        int64_t U = 0;  // staged columns of the group
        auto add = [&](int64_t s) {
            assigned[s] = 1;
            members.push_back((int32_t)s);
            for (int32_t t = 0; t < blk_cnt[s]; ++t) {
                const int32_t c = blk_col[(size_t)blk_ptr[s] + t];
                const bool fresh = col_stamp[c] != gid;
                if (fresh) {
                    col_stamp[c] = gid;
                    col_cnt[c] = 0;
                }
                if (++col_cnt[c] == need) ++U;
                if (!fresh || cptr[c + 1] - cptr[c] > prm.hub_cap) continue;
                for (int32_t x = cptr[c]; x < cptr[c + 1]; ++x) {
                    const int32_t o = cslots[x];
                    if (assigned[o]) continue;
                    if (slot_stamp[o] != gid) {
                        slot_stamp[o] = gid;
                        score[o] = 0;
                        cands.push_back(o);
                    }
                    ++score[o];
                }
            }
        };
        add(seed);
        // a row block with more columns than the stage holds stays alone,
        // with an empty stage: its tiles gather their rows directly
        const bool oversize = prm.stage_all && U > prm.u_max;
        while (!oversize && (int)members.size() < prm.g_max) {
            int32_t best = -1;
            for (int32_t o : cands) {
                if (assigned[o]) continue;
                if (best < 0 || score[o] > score[best] || (score[o] == score[best] && o < best)) best = o;
            }
            if (best < 0 || blk_cnt[best] == 0) break;
            if ((double)score[best] < prm.min_share * (double)blk_cnt[best]) break;
            int64_t dU = 0;
            for (int32_t t = 0; t < blk_cnt[best]; ++t) {
                const int32_t c = blk_col[(size_t)blk_ptr[best] + t];
                if (prm.stage_all ? col_stamp[c] != gid : (col_stamp[c] == gid && col_cnt[c] == 1)) ++dU;
            }
            if (U + dU > prm.u_max) break;
            add(best);
        }
        // the group's stage, ascending: every column of its tiles
        // (stage_all), or the columns two or more of its tiles use
        shared.clear();
        if (!oversize) {
            for (int32_t s : members)
                for (int32_t t = 0; t < blk_cnt[s]; ++t) {
                    const int32_t c = blk_col[(size_t)blk_ptr[s] + t];
                    if (col_cnt[c] >= need && col_local[c] != -2 - gid) {
                        col_local[c] = -2 - gid;  // collected once
                        shared.push_back(c);
                    }
                }
        }
        std::sort(shared.begin(), shared.end());
        for (size_t u = 0; u < shared.size(); ++u) col_local[shared[u]] = (int32_t)u;
        for (int32_t s : members) {
            const int64_t b0 = blk_ptr[s];
            const int64_t b1 = s + 1 < ns ? blk_ptr[s + 1] : nblk_pad;
            for (int64_t b = b0; b < b1; ++b) {
                if (b - b0 < blk_cnt[s]) {
                    const int32_t c = blk_col[(size_t)b];
                    if (!oversize && col_cnt[c] >= need) {
                        out.bsrc[(size_t)b] = col_local[c];
                        ++out.staged_tiles;
                    } else {
                        out.bsrc[(size_t)b] = -(c + 1);
                    }
                } else {
                    // padding tiles hold zero values: any finite row will do
                    out.bsrc[(size_t)b] = shared.empty() ? -1 : 0;
                }
            }
        }
        for (int32_t c : shared) col_local[c] = -1;
        out.order.insert(out.order.end(), members.begin(), members.end());
        out.grp_ptr.push_back((int32_t)out.order.size());
        out.ucol.insert(out.ucol.end(), shared.begin(), shared.end());
        out.u_ptr.push_back((int32_t)out.ucol.size());
        out.max_u = std::max<int64_t>(out.max_u, (int64_t)shared.size());
    }
}

}  // namespace hspmm
