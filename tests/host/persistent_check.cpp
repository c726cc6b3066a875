// Host-only check of the order of work of the persistent batched iteration
// (paper_1601_08201_amd/csrc/sgtv_persistent.h), the walk every workgroup of
// the cooperative launch takes.  The G workgroups of a launch run as G CPU
// threads with a real barrier between phases and atomic tile-queue counters,
// as on the GPU, and for grids and work counts around their edge cases:
//   * every workgroup passes the same barriers with targets G, 2G, 3G, ...
//     (four per iteration), so no wait can miss an arrival;
//   * within every iteration each tile and each elementwise block of each
//     phase is done exactly once, by some workgroup (and quarter), and a tile
//     only by a workgroup of its queue (t = wg mod min(G, 8));
//   * each item falls between the right barriers: forward tiles of iteration
//     k after 4k barriers, ratio after 4k + 1, back tiles after 4k + 2, the
//     image update after 4k + 3, and the split of iteration k after 4k + 4
//     (the last iteration's after all of them);
//   * the buffer parities of every phase are those of the launch sequence one
//     iteration at a time (forward from f[fc], image update f[fc] -> f[fc^1]
//     with (v, a) of parity vc, split with the new image and vc -> vc^1).
// Prints one line per case and "ok" at the end; exits 1 after a failure.
#include "../../paper_1601_08201_amd/csrc/sgtv_persistent.h"

#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

using namespace sgtv;

namespace {

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

struct Item {
    int segment, fc, vc;
    uint32_t wg;
};

// A reusable barrier for the simulated workgroups.
struct Barrier {
    std::mutex mu;
    std::condition_variable cv;
    uint32_t n, waiting = 0;
    uint64_t generation = 0;
    explicit Barrier(uint32_t count) : n(count) {}
    void wait() {
        std::unique_lock<std::mutex> lock(mu);
        const uint64_t gen = generation;
        if (++waiting == n) {
            waiting = 0;
            ++generation;
            cv.notify_all();
        } else {
            cv.wait(lock, [&] { return generation != gen; });
        }
    }
};

struct Shared {
    Barrier bar;
    std::atomic<int64_t> queue[2][kMaxQueues];
    std::mutex mu;
    std::map<std::tuple<int, int, int64_t>, std::vector<Item>> seen;
    explicit Shared(uint32_t G) : bar(G) {
        for (auto &q : queue)
            for (auto &c : q) c = 0;
    }
};

struct Recorder {
    const PersistentPlan &P;
    Shared &sh;
    uint32_t wg;
    int segment = 0;
    std::vector<uint32_t> targets;
    std::vector<std::tuple<int, int, int64_t, Item>> log;
    // iteration of a phase from the number of barriers passed
    int iteration(int phase) const { return phase == kPhaseSplit ? segment / 4 - 1 : segment / 4; }
    int64_t grab(int phase, uint32_t q) { return sh.queue[phase == kPhaseForward ? 0 : 1][q].fetch_add(1); }
    void clear(int phase) {
        for (auto &c : sh.queue[phase == kPhaseForward ? 0 : 1]) c = 0;
    }
    void tile(int phase, int64_t t, int fc) { log.emplace_back(phase, iteration(phase), t, Item{segment, fc, -1, wg}); }
    void blocks(int phase, int64_t first, int64_t stride, int64_t n, int fc, int vc) {
        for (int q = 0; q < P.quarters; ++q)
            for (int64_t b = first + q; b < n; b += stride)
                log.emplace_back(phase, iteration(phase), b, Item{segment, fc, vc, wg});
    }
    bool barrier(uint32_t target) {
        targets.push_back(target);
        sh.bar.wait();
        ++segment;
        return true;
    }
};

void check_case(const char *name, PersistentPlan P, uint32_t G) {
    Shared sh(G);
    std::vector<std::vector<uint32_t>> targets(G);
    std::vector<std::thread> pool;
    for (uint32_t wg = 0; wg < G; ++wg)
        pool.emplace_back([&, wg] {
            Recorder r{P, sh, wg};
            persistent_walk(P, wg, G, r);
            std::lock_guard<std::mutex> lock(sh.mu);
            targets[wg] = r.targets;
            for (auto &e : r.log) sh.seen[std::make_tuple(std::get<0>(e), std::get<1>(e), std::get<2>(e))].push_back(std::get<3>(e));
        });
    for (auto &t : pool) t.join();
    const uint32_t nq = persistent_queues(G);
    for (uint32_t wg = 0; wg < G; ++wg) {
        CHECK(static_cast<int64_t>(targets[wg].size()) == persistent_barriers(P), "%s: workgroup %u passed %zu barriers",
              name, wg, targets[wg].size());
        for (size_t i = 0; i < targets[wg].size(); ++i)
            CHECK(targets[wg][i] == static_cast<uint32_t>(i + 1) * G, "%s: barrier %zu of workgroup %u has target %u",
                  name, i, wg, targets[wg][i]);
    }
    const int64_t counts[5] = {P.n_tiles_f, P.n_rblocks, P.n_tiles_b, P.n_vblocks, P.n_sblocks};
    int64_t expected = 0;
    for (int k = 0; k < P.n_iters; ++k) {
        const int fc = (P.fcur0 + k) & 1, vc = (P.vcur0 + k) & 1;
        for (int phase = 0; phase < 5; ++phase)
            for (int64_t i = 0; i < counts[phase]; ++i) {
                ++expected;
                auto it = sh.seen.find(std::make_tuple(phase, k, i));
                CHECK(it != sh.seen.end() && it->second.size() == 1, "%s: phase %d item %lld of iteration %d done %zu times",
                      name, phase, static_cast<long long>(i), k, it == sh.seen.end() ? size_t(0) : it->second.size());
                const Item &x = it->second[0];
                const int want_seg = phase == kPhaseSplit ? 4 * k + 4 : 4 * k + phase;
                CHECK(x.segment == want_seg, "%s: phase %d of iteration %d after %d barriers (want %d)", name, phase,
                      k, x.segment, want_seg);
                if (phase == kPhaseForward || phase == kPhaseBack) {
                    CHECK(x.fc == fc, "%s: product of iteration %d reads f[%d]", name, k, x.fc);
                    CHECK(x.wg % nq == static_cast<uint32_t>(i % nq), "%s: tile %lld done by workgroup %u of another queue",
                          name, static_cast<long long>(i), x.wg);
                }
                if (phase == kPhaseVoxel)
                    CHECK(x.fc == fc && x.vc == vc, "%s: image update parities %d %d", name, x.fc, x.vc);
                if (phase == kPhaseSplit)
                    CHECK(x.fc == (fc ^ 1) && x.vc == vc, "%s: split of iteration %d has parities %d %d", name, k,
                          x.fc, x.vc);
            }
    }
    CHECK(static_cast<int64_t>(sh.seen.size()) == expected, "%s: %zu items done, %lld expected", name, sh.seen.size(),
          static_cast<long long>(expected));
    std::printf("%s: %u workgroups, %d iterations, %lld items, %lld barriers each\n", name, G, P.n_iters,
                static_cast<long long>(expected), static_cast<long long>(persistent_barriers(P)));
}

}  // namespace

int main() {
    // tiles fewer than, equal to and more than the workgroups; empty phases;
    // odd start parities; one iteration and several
    check_case("fewer tiles than workgroups", PersistentPlan{5, 3, 7, 11, 4, 3, 0, 0, 4}, 8);
    check_case("tiles a multiple of the grid", PersistentPlan{16, 24, 40, 64, 33, 2, 1, 0, 4}, 8);
    check_case("uneven tiles, odd parities", PersistentPlan{37, 53, 100, 201, 77, 4, 1, 1, 4}, 16);
    check_case("one iteration", PersistentPlan{9, 9, 9, 9, 9, 1, 0, 1, 2}, 4);
    check_case("empty elementwise phases", PersistentPlan{12, 12, 0, 0, 0, 3, 0, 0, 4}, 8);
    check_case("no iterations", PersistentPlan{12, 12, 5, 5, 5, 0, 0, 0, 4}, 8);
    check_case("one workgroup", PersistentPlan{7, 5, 9, 13, 6, 3, 1, 0, 4}, 1);
    check_case("fewer workgroups than queues", PersistentPlan{23, 17, 9, 13, 6, 3, 0, 1, 4}, 5);
    check_case("256 workgroups, 64-scan-like batch", PersistentPlan{4104, 4312, 600, 1200, 700, 2, 0, 0, 4}, 256);
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
