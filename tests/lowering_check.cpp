// lowering_check.cpp -- host-only driver for the sanitizer test: lowers a
// model (written by the test as the ABI's structs) under several launch
// options, checks the layout invariants, and runs the state-blob checks of
// arb_set_state on a valid blob and on corrupted ones.  Built with g++ and
// AddressSanitizer + UndefinedBehaviorSanitizer together with the library's
// lower.cpp; exits non-zero on any failure.
//
// Model file: int64 counts[6] (cells, branches, synapses, connections,
// events, clamps), then the six struct arrays in that order.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_1901_07454_amd/csrc/lower.hpp"

using namespace arbmi;

namespace {

template <class T>
bool read_array(FILE* f, std::vector<T>& v, int64_t n) {
    v.resize(size_t(n));
    return n == 0 || std::fread(v.data(), sizeof(T), size_t(n), f) == size_t(n);
}

int fails = 0;

void expect(bool ok, const std::string& what) {
    if (!ok) {
        std::printf("FAIL %s\n", what.c_str());
        ++fails;
    }
}

// The lowering's order of branches within a depth level: every parent's
// first child in the parents' task order, then every second child, and so
// on, each level numbered in that order (so consecutive threads of a round
// find their children at consecutive task entries).
bool level_order_ok(const Lowered& L) {
    for (const PackDesc& D : L.packs) {
        std::vector<std::vector<int32_t>> by_lev;
        for (int32_t t = 0; t < D.ntk; ++t) {
            const int32_t lev = L.tk_lev[D.tk0 + t];
            if (lev < 0) return false;
            if (size_t(lev) >= by_lev.size()) by_lev.resize(size_t(lev) + 1);
            by_lev[size_t(lev)].push_back(t);
        }
        for (const std::vector<int32_t>& ts : by_lev) {
            int32_t prev = -1;
            for (int32_t k = 0;; ++k) {
                bool any = false;
                for (int32_t t : ts) {
                    const TaskDesc& T = L.tasks[D.tk0 + t];
                    if (T.nch <= k) continue;
                    const int32_t c = L.ch_task[D.ch0 + T.ch0 + k];
                    if (c <= prev) return false;
                    prev = c;
                    any = true;
                }
                if (!any) break;
            }
        }
    }
    return true;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t cnt[6];
    if (std::fread(cnt, 8, 6, f) != 6) return 2;
    std::vector<arb_cell> cells;
    std::vector<arb_branch> br;
    std::vector<arb_synapse> syn;
    std::vector<arb_connection> con;
    std::vector<arb_event> ev;
    std::vector<arb_iclamp> ic;
    if (!read_array(f, cells, cnt[0]) || !read_array(f, br, cnt[1]) || !read_array(f, syn, cnt[2]) ||
        !read_array(f, con, cnt[3]) || !read_array(f, ev, cnt[4]) || !read_array(f, ic, cnt[5]))
        return 2;
    std::fclose(f);

    arb_params p{};
    p.dt_ms = 0.025;
    p.threshold_mV = -10.0;
    p.v_init_mV = -65.0;
    struct Opt {
        int T, mode, slots, len, cells;
        bool grads;
    };
    const Opt opts[] = {{64, 1, 0, 8, 1, false},   {256, 2, 0, 8, 8, false}, {128, 2, 0, 8, 4, true},
                        {64, 3, 2, 8, 1, false},   {128, 3, 2, 8, 4, false}, {256, 3, 3, 8, 64, false},
                        {128, 3, 1, 16, 2, false}, {64, 3, 3, 8, 1, true}};
    int lowered = 0;
    for (const Opt& o : opts) {
        LowerOptions opt;
        opt.block_threads = o.T;
        opt.coef_mode = o.mode;
        opt.reg_slots = o.mode == 3 ? o.slots : 0;
        opt.reg_len = o.len;
        opt.max_cells_per_pack = o.cells;
        opt.grads = o.grads;
        opt.lds_budget = 80 * 1024;
        opt.lds_hard_max = 160 * 1024 - 256;
        Lowered L;
        std::string err;
        const int rc = lower_model(cells.data(), int32_t(cells.size()), br.data(), int64_t(br.size()), syn.data(),
                                   int64_t(syn.size()), con.data(), int64_t(con.size()), ev.data(),
                                   int64_t(ev.size()), ic.data(), int32_t(ic.size()), p, opt, L, err);
        if (rc != ARB_OK) {  // a layout these cells do not fit is an answer, not a failure
            std::printf("option T=%d mode=%d slots=%d: refused (%s)\n", o.T, o.mode, o.slots, err.c_str());
            continue;
        }
        ++lowered;
        expect(verify_layout(L).empty(), "layout invariants: " + verify_layout(L));
        expect(level_order_ok(L), "branch order within depth levels");
        recompute_coefficients(L);

        // state blobs as arb_get_state writes them for this lowering
        StateShape sh;
        sh.net = !L.cr_src.empty();
        sh.K = sh.net ? L.min_delay : 1000;
        sh.bk_cap = sh.net ? int32_t(std::max<int64_t>(64, 4 * L.max_in_per_pack)) : 0;
        sh.sp_cap = uint32_t(std::max<int64_t>(1 << 16, int64_t(L.n_cells) * 64));
        sh.n_hist = sh.net ? 1 + (L.max_delay + sh.K - 1) / sh.K : 1;
        sh.hist_cap = sh.net ? sh.sp_cap : 0;
        int64_t bytes[kStateParts];
        state_part_bytes(L, sh, bytes);
        int64_t total = sizeof(StateHeader), off[kStateParts];
        for (int k = 0; k < kStateParts; ++k) {
            off[k] = total;
            total += bytes[k];
        }
        std::vector<char> blob(size_t(total), 0);
        const int64_t np = int64_t(L.packs.size());
        StateHeader h{kStateMagic, 0, L.n_slots, int64_t(L.hh_cv.size()), int64_t(L.syn_global.size()),
                      np, np, sh.bk_cap, int64_t(sh.sp_cap), 0};
        std::memcpy(blob.data(), &h, sizeof h);
        for (int64_t q = 0; q < np; ++q) std::memcpy(blob.data() + off[5] + 8 * q, &L.packs[q].xe0, 8);
        expect(check_state_blob(L, sh, blob.data(), total).empty(), "valid blob refused: " +
               check_state_blob(L, sh, blob.data(), total));
        auto corrupt = [&](const char* what, auto mutate) {
            std::vector<char> b = blob;
            mutate(b);
            expect(!check_state_blob(L, sh, b.data(), int64_t(b.size())).empty(), std::string("accepted ") + what);
        };
        corrupt("a wrong magic", [&](std::vector<char>& b) { b[0] ^= 1; });
        corrupt("a negative step", [&](std::vector<char>& b) {
            const int64_t v = -1;
            std::memcpy(b.data() + 8, &v, 8);
        });
        if (np > 0)
            corrupt("a cursor past the pack's events", [&](std::vector<char>& b) {
                const int64_t v = L.packs[0].xe1 + 1;
                std::memcpy(b.data() + off[5], &v, 8);
            });
        corrupt("a spike gid out of range", [&](std::vector<char>& b) {
            const Counters c{1, 0, 0, 0};
            std::memcpy(b.data() + off[10], &c, sizeof c);
            const uint32_t g = uint32_t(L.n_cells);
            std::memcpy(b.data() + off[11], &g, 4);
        });
        if (sh.net && np > 0) {
            corrupt("a bucket offset past its capacity", [&](std::vector<char>& b) {
                const uint32_t v = uint32_t(sh.bk_cap) + 1;
                std::memcpy(b.data() + off[6] + 4 * sh.K, &v, 4);
            });
            corrupt("a history gid out of range", [&](std::vector<char>& b) {
                const uint32_t one = 1, g = uint32_t(L.n_cells) + 7;
                std::memcpy(b.data() + off[14], &one, 4);
                std::memcpy(b.data() + off[15], &g, 4);
            });
        }
        expect(!check_state_blob(L, sh, blob.data(), total - 1).empty(), "accepted a truncated blob");
    }
    std::printf("lowered %d option sets, %d failures\n", lowered, fails);
    return (fails == 0 && lowered > 0) ? 0 : 1;
}
