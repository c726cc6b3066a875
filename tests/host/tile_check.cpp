// Host-only check of the tiled matrix format that the products stream.
//
// Builds the format from synthetic CSR matrices with the library's own
// builder (this file includes the library source, so no GPU is touched),
// decodes it independently of the kernels, and checks:
//   * every stored non-padding entry is a CSR entry (row, column, value bits)
//     and every CSR entry is stored exactly once;
//   * padding entries carry value 0 (24-bit lists: column code cb, the zero
//     kept in LDS; 32-bit lists: the spare row rw);
//   * 24-bit lists are lane-owned: no row is held by two lanes of a list, a
//     lane's entries of one row are adjacent, and a lane's padding repeats its
//     last row or takes a row absent from the list;
//   * 32-bit lists hold 64 distinct rows in every group;
//   * the slot table of every tile is a permutation of the row block, present
//     exactly when the rows are dealt to the waves.
// Prints one line per case and "ok" at the end; exits 1 after a failure.
#include "../../paper_1601_08201_amd/csrc/sgtv_api.hip"

#include <cstdio>
#include <map>
#include <set>
#include <tuple>

namespace {

struct Csr {
    int64_t n_rows = 0, n_cols = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<float> v;
};

uint64_t lcg(uint64_t &s) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 33;
}

// rows with about `per_row` entries (some rows empty, some long runs of one
// column block, a few duplicated entries and explicit zeros)
Csr make_csr(int64_t n_rows, int64_t n_cols, int per_row, uint64_t seed, bool runs) {
    Csr m;
    m.n_rows = n_rows;
    m.n_cols = n_cols;
    m.rp.push_back(0);
    uint64_t s = seed;
    for (int64_t r = 0; r < n_rows; ++r) {
        int k = static_cast<int>(lcg(s) % (2 * per_row + 1));
        if (r % 17 == 5) k = 0;                     // empty rows
        for (int e = 0; e < k; ++e) {
            int32_t c = static_cast<int32_t>(lcg(s) % n_cols);
            if (runs && r % 7 == 0) c = static_cast<int32_t>((r * 13 + e) % std::min<int64_t>(n_cols, 40));
            if (c % 101 == 3) c = (c + 1) % n_cols;   // some empty columns
            float val = static_cast<float>(lcg(s) % 1000 + 1) / 997.0f;
            if (e % 29 == 11) val = 0.0f;             // explicit zeros
            m.ci.push_back(c);
            m.v.push_back(val);
            if (e % 31 == 7) {                        // a duplicated entry
                m.ci.push_back(c);
                m.v.push_back(val * 0.5f);
            }
        }
        m.rp.push_back(static_cast<int64_t>(m.ci.size()));
    }
    return m;
}

int failures = 0;

#define CHECK(cond, ...)                                       \
    do {                                                       \
        if (!(cond)) {                                         \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);   \
            std::printf(__VA_ARGS__);                          \
            std::printf("\n");                                 \
            ++failures;                                        \
            return;                                            \
        }                                                      \
    } while (0)

typedef std::tuple<int64_t, int64_t, uint32_t> Entry;   // row, column, value bits

uint32_t bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

void check_case(const char *name, const Csr &m, TileParams t, bool want24, bool want_dealt) {
    std::vector<int32_t> pk, goff, poff;
    std::vector<float> pv;
    std::vector<uint16_t> slot;
    sgtv::TileMap map{};
    const int e = build_tiled(m.n_rows, m.n_cols, m.rp, m.ci, m.v, t, true, pk, pv, goff, poff, slot, map);
    CHECK(e == SGTV_OK, "%s: build failed", name);
    CHECK((map.idx24 != 0) == want24, "%s: index format %d", name, map.idx24);
    CHECK(!slot.empty() == want_dealt, "%s: slot table present %d", name, static_cast<int>(!slot.empty()));
    const int64_t RB = static_cast<int64_t>(t.waves) * t.rw;
    const int ns = map.ns, cbs = map.cbs_max, W = t.waves;
    const int64_t n_tiles = map.n_rb * ns;
    // row offset of every slot (inverse of the slot table)
    std::vector<int64_t> row_of(static_cast<size_t>(n_tiles * RB));
    for (int64_t tile = 0; tile < n_tiles; ++tile) {
        std::vector<uint8_t> seen(static_cast<size_t>(RB), 0);
        for (int64_t i = 0; i < RB; ++i) {
            const int64_t s = slot.empty() ? i : slot[static_cast<size_t>(tile * RB + i)];
            CHECK(s >= 0 && s < RB && !seen[s], "%s: slot table of tile %lld is not a permutation", name,
                  static_cast<long long>(tile));
            seen[s] = 1;
            row_of[static_cast<size_t>(tile * RB + s)] = i;
        }
    }
    std::vector<Entry> stored;
    const int64_t n_lists = map.n_rb * ns * cbs * W;
    CHECK(static_cast<int64_t>(goff.size()) == n_lists + 1, "%s: goff size", name);
    for (int64_t L = 0; L < n_lists; ++L) {
        const int64_t w = L % W, cl = (L / W) % cbs, tile = L / W / cbs;
        const int64_t rb = tile / ns;
        const int slab = static_cast<int>(tile % ns);
        const int64_t cbi = map.slab_begin[slab] + cl;
        const int64_t ng = goff[L + 1] - goff[L], nb4 = ng / 4, nsb = nb4 / 4;
        const int64_t base = static_cast<int64_t>(goff[L]) * 64;
        if (cbi >= map.slab_begin[slab + 1]) {
            CHECK(ng == 0, "%s: list past its slab is not empty", name);
            continue;
        }
        // entry (group g, lane) -> packed index and value
        auto get = [&](int64_t g, int64_t lane, uint32_t &code, float &val) {
            const int64_t b = g / 4, m4 = g % 4;
            const int64_t vpos = g < nb4 * 4 ? base + b * 256 + lane * 4 + m4 : base + nb4 * 256 + (g - nb4 * 4) * 64 + lane;
            val = pv[static_cast<size_t>(vpos)];
            if (!map.idx24) {
                code = static_cast<uint32_t>(pk[static_cast<size_t>(vpos)]);
                return;
            }
            const uint32_t *q = reinterpret_cast<const uint32_t *>(pk.data()) + poff[L];
            if (g >= nb4 * 4) {
                code = q[nb4 * 192 + (g - nb4 * 4) * 64 + lane];
                return;
            }
            uint32_t w0, w1, w2;
            if (b < nsb * 4) {
                const uint32_t *sbp = q + (b / 4) * 768;
                uint32_t W12[12];
                for (int i = 0; i < 12; ++i) W12[i] = sbp[(i / 4) * 256 + lane * 4 + (i % 4)];
                const int64_t t3 = 3 * (b % 4);
                w0 = W12[t3];
                w1 = W12[t3 + 1];
                w2 = W12[t3 + 2];
            } else {
                const uint32_t *bp = q + nsb * 768 + (b - nsb * 4) * 192;
                w0 = bp[lane * 2];
                w1 = bp[lane * 2 + 1];
                w2 = bp[128 + lane];
            }
            const uint32_t e4[4] = {w0 & 0xFFFFFFu, ((w0 >> 24) | (w1 << 8)) & 0xFFFFFFu,
                                    ((w1 >> 16) | (w2 << 16)) & 0xFFFFFFu, w2 >> 8};
            code = e4[m4];
        };
        CHECK(!map.idx24 || map.cbits == (t.rw <= 1024 ? 14 : 13), "%s: column bits %d", name, map.cbits);
        const int sh = map.idx24 ? map.cbits : 16;
        const uint32_t cmask = (1u << sh) - 1;
        std::map<int64_t, int> owner;             // local row -> lane (24-bit lists)
        std::vector<std::vector<int64_t>> lane_rows(64);
        std::vector<std::vector<bool>> lane_pad(64);
        for (int64_t g = 0; g < ng; ++g) {
            std::set<int64_t> group_rows;
            for (int64_t lane = 0; lane < 64; ++lane) {
                uint32_t code;
                float val;
                get(g, lane, code, val);
                const int64_t lr = code >> sh, col = code & cmask;
                const bool pad = map.idx24 ? col == static_cast<int64_t>(t.cb) : lr == t.rw;
                lane_rows[lane].push_back(lr);
                lane_pad[lane].push_back(pad);
                if (pad) {
                    CHECK(bits(val) == 0, "%s: padding with a nonzero value", name);
                    continue;
                }
                CHECK(lr < t.rw && col < t.cb, "%s: index out of range", name);
                if (!map.idx24) CHECK(group_rows.insert(lr).second, "%s: row twice in a group", name);
                const int64_t row = rb * RB + row_of[static_cast<size_t>(tile * RB + w * t.rw + lr)];
                stored.emplace_back(row, cbi * t.cb + col, bits(val));
            }
        }
        if (!map.idx24) continue;
        std::set<int64_t> real_rows;
        for (int lane = 0; lane < 64; ++lane)
            for (size_t i = 0; i < lane_rows[lane].size(); ++i)
                if (!lane_pad[lane][i]) real_rows.insert(lane_rows[lane][i]);
        for (int lane = 0; lane < 64; ++lane) {
            int64_t last = -1;
            bool any = false;
            std::set<int64_t> done;
            for (size_t i = 0; i < lane_rows[lane].size(); ++i) {
                const int64_t lr = lane_rows[lane][i];
                if (lane_pad[lane][i]) {
                    CHECK((any && lr == last) || (!any && !real_rows.count(lr)),
                          "%s: padding row of a lane is neither its last row nor absent", name);
                    continue;
                }
                CHECK(!any || lr == last || !done.count(lr), "%s: a lane's row is not one run", name);
                if (any && lr != last) done.insert(last);
                auto it = owner.find(lr);
                CHECK(it == owner.end() || it->second == lane, "%s: row held by two lanes", name);
                owner[lr] = lane;
                last = lr;
                any = true;
            }
        }
    }
    std::vector<Entry> want;
    for (int64_t r = 0; r < m.n_rows; ++r)
        for (int64_t k = m.rp[r]; k < m.rp[r + 1]; ++k) want.emplace_back(r, m.ci[k], bits(m.v[k]));
    std::sort(stored.begin(), stored.end());
    std::sort(want.begin(), want.end());
    CHECK(stored == want, "%s: stored entries differ from the matrix (%zu stored, %zu in CSR)", name,
          stored.size(), want.size());
    // list lengths: the sum over column blocks of the longest wave list
    int64_t sum_max = 0;
    for (int64_t tile = 0; tile < n_tiles; ++tile)
        for (int cl = 0; cl < cbs; ++cl) {
            int64_t mx = 0;
            for (int w = 0; w < W; ++w) {
                const int64_t L = (tile * cbs + cl) * W + w;
                mx = std::max<int64_t>(mx, goff[L + 1] - goff[L]);
            }
            sum_max += mx;
        }
    std::printf("%s: %zu entries, %lld tiles, %s indices, %s rows, sum of block maxima %lld groups\n", name,
                want.size(), static_cast<long long>(n_tiles), map.idx24 ? "24-bit" : "32-bit",
                slot.empty() ? "contiguous" : "dealt", static_cast<long long>(sum_max));
}

// The packed arrays of one case built with one host thread and with eight.
void check_threads(const char *name, const Csr &m, TileParams t) {
    std::vector<int32_t> pk[2], goff[2], poff[2];
    std::vector<float> pv[2];
    std::vector<uint16_t> slot[2];
    sgtv::TileMap map[2]{};
    const char *counts[2] = {"1", "8"};
    for (int k = 0; k < 2; ++k) {
        setenv("SGTV_HOST_THREADS", counts[k], 1);
        const int e = build_tiled(m.n_rows, m.n_cols, m.rp, m.ci, m.v, t, true, pk[k], pv[k], goff[k], poff[k],
                                  slot[k], map[k]);
        CHECK(e == SGTV_OK, "%s: build with %s threads failed", name, counts[k]);
    }
    unsetenv("SGTV_HOST_THREADS");
    CHECK(pk[0] == pk[1], "%s: packed indices differ between 1 and 8 threads", name);
    CHECK(pv[0].size() == pv[1].size() &&
              std::memcmp(pv[0].data(), pv[1].data(), sizeof(float) * pv[0].size()) == 0,
          "%s: values differ between 1 and 8 threads", name);
    CHECK(goff[0] == goff[1] && poff[0] == poff[1] && slot[0] == slot[1],
          "%s: list offsets or slot tables differ between 1 and 8 threads", name);
    CHECK(std::memcmp(&map[0], &map[1], sizeof(map[0])) == 0, "%s: tile maps differ", name);
    std::printf("%s: identical with 1 and 8 host threads\n", name);
}

}  // namespace

int main() {
    const Csr a = make_csr(5000, 3000, 20, 1, false);
    check_case("24-bit, dealt rows", a, TileParams{64, 4, 1024, 2}, true, true);
    check_case("24-bit, 16 waves, 3 slabs", a, TileParams{128, 16, 256, 3}, true, true);
    check_case("32-bit (odd block width)", a, TileParams{100, 4, 1023, 2}, false, false);
    const Csr b = make_csr(3000, 4000, 24, 2, true);
    check_case("24-bit, long row runs and duplicates", b, TileParams{64, 8, 512, 1}, true, true);
    const Csr c = make_csr(2048, 200000, 30, 3, false);
    check_case("24-bit, counts past 2^24: contiguous rows", c, TileParams{64, 16, 12, 1}, true, false);
    check_threads("threads, 24-bit dealt rows", a, TileParams{64, 4, 1024, 2});
    check_threads("threads, 32-bit", a, TileParams{100, 4, 1023, 2});
    check_threads("threads, long row runs", b, TileParams{64, 8, 512, 1});
    const Csr d = make_csr(40000, 30000, 16, 4, false);
    check_threads("threads, many row blocks", d, TileParams{128, 16, 4096, 4});
    // degenerate matrices: no entries at all, one row, one column
    Csr e;
    e.n_rows = 300;
    e.n_cols = 500;
    e.rp.assign(301, 0);
    check_case("24-bit, no entries", e, TileParams{64, 4, 128, 2}, true, true);
    check_case("32-bit, no entries", e, TileParams{100, 4, 127, 2}, false, false);
    const Csr one_row = make_csr(1, 4000, 900, 5, false);
    check_case("24-bit, one row", one_row, TileParams{64, 4, 1024, 2}, true, true);
    const Csr one_col = make_csr(3000, 1, 1, 6, false);
    check_case("24-bit, one column", one_col, TileParams{64, 4, 4, 1}, true, true);
    // 11-bit rows and 13-bit columns: up to 2048 rows per wave, blocks of at
    // most 8188 columns; wider blocks take the 32-bit format
    const Csr f = make_csr(9000, 20000, 40, 7, true);
    check_case("24-bit, 2048 rows per wave, dealt rows", f, TileParams{2048, 4, 8188, 2}, true, true);
    check_case("24-bit, 1500 rows per wave, dealt rows", f, TileParams{1500, 3, 4000, 3}, true, true);
    check_case("32-bit, 2048 rows per wave, 8192-column blocks", f, TileParams{2048, 2, 8192, 2}, false, false);
    check_threads("threads, 2048 rows per wave", f, TileParams{2048, 4, 8188, 2});
    // seeded random schedules over both index formats and both column splits;
    // the expected format and dealing follow the format's stated limits
    uint64_t rs = 12345;
    for (int k = 0; k < 24 && !failures; ++k) {
        const int64_t n_rows = 1 + static_cast<int64_t>(lcg(rs) % 12000);
        const int64_t n_cols = 1 + static_cast<int64_t>(lcg(rs) % 30000);
        const Csr m = make_csr(n_rows, n_cols, 1 + static_cast<int>(lcg(rs) % 30), 100 + k, k % 3 == 0);
        TileParams t;
        const int rws[] = {64, 100, 512, 1024, 1025, 1536, 2048, 2100};
        t.rw = rws[lcg(rs) % 8];
        t.waves = 1 + static_cast<int>(lcg(rs) % 16);
        const int cbs[] = {12, 1000, 4096, 8188, 8192, 16380, 16384};
        t.cb = cbs[lcg(rs) % 7];
        t.ns = 1 + static_cast<int>(lcg(rs) % 4);
        const int cmax = t.rw <= 1024 ? 16380 : 8188;
        const bool want24 = t.rw >= 64 && t.rw <= 2048 && t.cb % 4 == 0 && t.cb <= cmax;
        const int64_t ncb = (n_cols + t.cb - 1) / t.cb;
        if (t.ns > ncb) t.ns = static_cast<int>(ncb);   // as the schedule chooser caps it
        int64_t cbs_max = 0;
        for (int s2 = 0; s2 < t.ns; ++s2)
            cbs_max = std::max<int64_t>(cbs_max, ((s2 + 1) * ncb) / t.ns - (s2 * ncb) / t.ns);
        const int64_t RB = static_cast<int64_t>(t.waves) * t.rw;
        const bool want_dealt = want24 && t.ns * RB * cbs_max <= (int64_t(1) << 24);
        char name[160];
        std::snprintf(name, sizeof name, "random %d: %lld x %lld, rw %d, waves %d, cb %d, ns %d", k,
                      static_cast<long long>(n_rows), static_cast<long long>(n_cols), t.rw, t.waves, t.cb, t.ns);
        check_case(name, m, t, want24, want_dealt);
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
