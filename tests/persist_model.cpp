// Host model of the persistent batched launch's scheduling loop
// (paper_1702_07482_amd/csrc/tnrd_persist.hpp, the same source the GPU kernel
// runs): workgroups of threads standing for waves, std::barrier for the
// workgroup barrier, std::atomic_ref for the device-scope atomics.  The
// stage work is replaced by the reads and writes a stage makes in the
// exchange form, on plain (non-atomic) per-tile words, so that
// ThreadSanitizer checks every read and overwrite against the loop's
// synchronisation, and the stamps read check that each stage sees the values
// of the stage before it:
//   stage t >= 1 of tile k reads u_(t-1) (plane (T - t + 1) mod 2, stamp t - 1)
//   and the stage t-1 slab (set (t - 1) mod 2, stamp t - 1) of every tile of
//   its 3 x 3 neighbourhood, writes u_t of its own pixels (plane (T - t) mod 2)
//   and its stage t slab (set t mod 2); stage 0 writes only its slab; the last
//   reaction (t = T) reads the covering slabs and its own u_(T-1) and writes
//   u_T (plane 0).
//
// usage: persist_model <seed> <workgroups> <waves> <stages> <spin_limit> <budget_ns> <slow>
// Exit status 0 when every item ran once, every flag reached T + 1, every
// stamp read was the expected one and no wait gave up (slow = 0), or, with
// slow = 1 (a stage takes 200 us, so waits give up), when the launch still
// ended with the abort flag raised.
#include <atomic>
#include <barrier>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "tnrd_persist.hpp"

using namespace tnrd;

namespace {

struct Image {
    int k0, tiles_x, tiles_y;
};

struct Batch {
    int T = 0, per_stage = 0;
    std::vector<Image> imgs;
    std::vector<int> img_of;  // per item
    std::vector<int> plane[2], slab[2], done;
    int bad = 0;              // stamps that were not the expected ones (atomic)
    bool slow = false;
};

struct Workgroup {
    explicit Workgroup(int waves) : bar(waves) {}
    std::barrier<> bar;
    int shared = 0;
};

struct HostP {
    Batch *b;
    Workgroup *wg;
    int wave;
    std::mt19937 *rng;
    int tid() const { return wave; }
    void barrier() { wg->bar.arrive_and_wait(); }
    int fetch_next(int *p) { return std::atomic_ref<int>(*p).fetch_add(1, std::memory_order_relaxed); }
    void set_shared(int v) { wg->shared = v; }
    int get_shared() { return wg->shared; }
    // ThreadSanitizer does not model stand-alone fences, so the polls carry the
    // acquire here and acquire() is empty (on the GPU the polls are relaxed and
    // acquire() is the fence); std::barrier orders the other threads' accesses
    int poll(const int *p)
    {
        return std::atomic_ref<int>(*const_cast<int *>(p)).load(std::memory_order_acquire);
    }
    void acquire() {}
    void store_release(int *p, int v) { std::atomic_ref<int>(*p).store(v, std::memory_order_release); }
    void stores_done() {}
    void pause() { std::this_thread::yield(); }
    long long now()
    {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    void neighbours(int k, int *nb)
    {
        const Image &im = b->imgs[b->img_of[k]];
        persist_neighbours(im.k0, k - im.k0, im.tiles_x, im.tiles_y, nb);
    }
    void check(int got, int want)
    {
        if (got != want) std::atomic_ref<int>(b->bad).fetch_add(1, std::memory_order_relaxed);
    }
    void work(int t, int k)
    {
        const int T = b->T;
        // each wave takes a share of the tile's words; the waves of a workgroup
        // touch disjoint words, as the rows of a tile are disjoint
        if (b->slow && wave == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
        if ((*rng)() % 4 == 0) std::this_thread::yield();
        int nb[9];
        neighbours(k, nb);
        if (t < T) {
            if (t >= 1) {
                for (int q = 0; q < 9; ++q) {
                    if (nb[q] < 0) continue;
                    if (t - 1 >= 1) check(b->plane[(T - t + 1) & 1][nb[q]], t - 1);
                    check(b->slab[(t - 1) & 1][nb[q]], t - 1);
                }
            }
            if (wave == 0) {
                if (t >= 1) b->plane[(T - t) & 1][k] = t;
                b->slab[t & 1][k] = t;
            }
        } else {
            if (T - 1 >= 1) check(b->plane[(T - T + 1) & 1][k], T - 1);
            for (int q = 0; q < 9; ++q)
                if (nb[q] >= 0) check(b->slab[(T - 1) & 1][nb[q]], T - 1);
            if (wave == 0) b->plane[0][k] = T;
        }
        if (wave == 0) b->done[(size_t)t * b->per_stage + k] += 1;
    }
};

}  // namespace

int main(int argc, char **argv)
{
    if (argc != 8) {
        std::fprintf(stderr, "usage: %s seed workgroups waves stages spin_limit budget_ns slow\n", argv[0]);
        return 2;
    }
    const unsigned seed = (unsigned)std::atoi(argv[1]);
    const int G = std::atoi(argv[2]), W = std::atoi(argv[3]);
    Batch b;
    b.T = std::atoi(argv[4]);
    const int spin_limit = std::atoi(argv[5]);
    const long long budget = std::atoll(argv[6]);
    b.slow = std::atoi(argv[7]) != 0;
    std::mt19937 rng(seed);
    // uneven images: tile grids from 1 x 1 to 6 x 5
    const int n_img = 3 + (int)(rng() % 5);
    for (int i = 0; i < n_img; ++i) {
        Image im{b.per_stage, 1 + (int)(rng() % 6), 1 + (int)(rng() % 5)};
        b.imgs.push_back(im);
        for (int q = 0; q < im.tiles_x * im.tiles_y; ++q) b.img_of.push_back(i);
        b.per_stage += im.tiles_x * im.tiles_y;
    }
    for (int s = 0; s < 2; ++s) {
        b.plane[s].assign(b.per_stage, -1);
        b.slab[s].assign(b.per_stage, -1);
    }
    b.done.assign((size_t)(b.T + 1) * b.per_stage, 0);
    std::vector<int> flags(b.per_stage, 0);
    int next = 0, abort_flag = 0;
    PersistCtl c{&next, flags.data(), &abort_flag, (b.T + 1) * b.per_stage, b.per_stage, spin_limit, budget};

    std::vector<Workgroup *> wgs;
    for (int g = 0; g < G; ++g) wgs.push_back(new Workgroup(W));
    std::vector<std::mt19937> rngs;
    for (int i = 0; i < G * W; ++i) rngs.emplace_back(seed * 7919u + (unsigned)i);
    std::vector<std::thread> th;
    for (int g = 0; g < G; ++g)
        for (int w = 0; w < W; ++w)
            th.emplace_back([&, g, w]() {
                HostP p{&b, wgs[g], w, &rngs[(size_t)g * W + w]};
                persist_loop(p, c);
            });
    for (auto &x : th) x.join();
    for (auto *w : wgs) delete w;

    if (b.slow) {
        std::printf("ended; abort flag %d\n", abort_flag);
        return 0;
    }
    int missing = 0;
    for (int d : b.done) missing += d != 1;
    int flag_bad = 0;
    for (int f : flags) flag_bad += f != b.T + 1;
    int out_bad = 0;
    for (int k = 0; k < b.per_stage; ++k) out_bad += b.plane[0][k] != b.T;
    std::printf("images %d items/stage %d: not run once %d, flags off %d, outputs off %d, "
                "stamps off %d, abort %d\n",
                n_img, b.per_stage, missing, flag_bad, out_bad, b.bad, abort_flag);
    return (missing || flag_bad || out_bad || b.bad || abort_flag) ? 1 : 0;
}
