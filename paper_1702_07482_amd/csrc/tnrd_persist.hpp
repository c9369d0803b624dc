// Scheduling loop of the single persistent launch of the batched forward:
// every stage of every tile of an uneven batch in one launch (per-look models,
// Sec. 4.5), as plain C++ templated on a platform so that the same source
// runs on the GPU (k_batched_persist) and in a host model with one thread per
// wave, real barriers and std::atomic flags (tests/persist_model.cpp).
//
// Work items are (stage t, batch item k), handed out in the order
// i = t * per_stage + k (stage-major) by one atomic counter; t = T is the last
// stage's reaction.  In the exchange form, stage t of tile k reads u_(t-1)
// and the stage t-1 slabs of the tiles in k's 3 x 3 neighbourhood (the tiles
// of an image are at least 2R on each side, so nothing farther covers k's
// u tile) and writes u_t at its own pixels (the u_(t-2) plane) and its stage t
// slab (the stage t-2 slab set).  All of these reads and overwrites are
// ordered by one condition: every tile of the neighbourhood has finished
// stage t - 1, i.e. flags[k'] >= t, flags counting the stages a tile has
// finished.
//
// Deadlock freedom: a workgroup only ever waits for items of the previous
// stage, which were handed out before its own item (stage-major order) to
// workgroups that were running when they took them; by induction on the item
// index every wait ends, whatever the number of resident workgroups.  A wait
// still gives up after spin_limit polls, or once `budget` clock ticks have
// passed since its workgroup started, raising abort_flag.  A workgroup that
// gave up never waits again, and no wait polls once it sees abort_flag, so a
// launch always ends (with wrong results, which the host detects from the
// flag) even if the flags never became visible: every workgroup's waits end
// within spin_limit polls and its budget, without depending on any other
// workgroup.
//
// Barriers: every thread of a workgroup runs the same sequence of barriers;
// the item is broadcast through one shared word written by thread 0 between
// two barriers, so all threads see the same item and leave the loop together.
//
// Memory ordering: only thread 0 synchronises with other workgroups.  Its
// polls and one acquire after the last of them order the neighbours' results
// before the barrier that starts the item; after the item, every thread
// completes its own stores, a barrier orders them before thread 0's release
// store of the flag.  On the GPU the acquire invalidates the compute unit's
// and the XCD's caches once per item and the release writes the XCD's L2 back
// once per item (the other waves' stores sit in that same L2 by then), instead
// of once per wave and per poll.
//
// Platform P (every member called by every thread of a workgroup unless noted):
//   int tid()                           thread index in the workgroup
//   void barrier()                      workgroup barrier
//   int fetch_next(int *counter)        device-scope atomic increment, returns the old value (thread 0)
//   void set_shared(int v), int get_shared()   the broadcast word
//   int poll(const int *p)              device-scope load of a flag (thread 0); with
//                                       acquire() after the last poll, an acquire
//   void acquire()                      device-scope acquire fence after the polls (thread 0)
//   void store_release(int *p, int v)   device-scope release store (thread 0)
//   void stores_done()                  waits until the thread's own stores have completed
//   void pause()                        back-off between polls (thread 0)
//   long long now()                     a clock that advances at a fixed rate (thread 0)
//   void neighbours(int k, int *nb)     items of k's 3 x 3 neighbourhood (nb[4] = k), -1 where
//                                       the neighbour lies outside the image
//   void work(int t, int k)             stage t (t == T: the last reaction) on item k
#pragma once

namespace tnrd {

struct PersistCtl {
    int *next;        // item counter, 0 at launch
    int *flags;       // [per_stage] stages finished per batch item, 0 at launch
    int *abort_flag;  // 0 at launch; 1 once a wait has given up
    int n_items;      // (T + 1) * per_stage
    int per_stage;    // batch items (image tiles) per stage
    int spin_limit;   // polls before a wait gives up
    long long budget; // clock ticks after a workgroup's start at which its waits give up
};

// Items of the 3 x 3 neighbourhood of tile `tile` of an image whose tiles are
// numbered row-major on a tiles_x x tiles_y grid starting at batch item k0:
// nb[3 (dy + 1) + dx + 1], -1 outside the image.  (Fixed slots keep the array
// in registers on the GPU.)
inline void persist_neighbours(int k0, int tile, int tiles_x, int tiles_y, int *nb)
{
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int y = ty + dy, x = tx + dx;
            nb[3 * (dy + 1) + dx + 1] =
                (y >= 0 && y < tiles_y && x >= 0 && x < tiles_x) ? k0 + y * tiles_x + x : -1;
        }
}

template <class P>
inline void persist_loop(P &p, const PersistCtl &c)
{
    // thread 0 only: when the workgroup started, and whether it gave up
    const long long t0 = p.tid() == 0 ? p.now() : 0;
    bool gave_up = false;
    for (;;) {
        if (p.tid() == 0) p.set_shared(p.fetch_next(c.next));
        p.barrier();
        const int item = p.get_shared();
        p.barrier();  // every thread has the item before thread 0 fetches the next one
        if (item >= c.n_items) return;  // the same value in every thread
        const int t = item / c.per_stage, k = item - t * c.per_stage;
        if (t > 0) {
            if (p.tid() == 0 && !gave_up) {
                int nb[9];
                p.neighbours(k, nb);
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (nb[q] < 0 || gave_up) continue;
                    int spins = 0;
                    while (p.poll(c.flags + nb[q]) < t) {
                        if (p.poll(c.abort_flag) != 0 || ++spins >= c.spin_limit ||
                            p.now() - t0 > c.budget) {
                            p.store_release(c.abort_flag, 1);
                            gave_up = true;
                            break;
                        }
                        p.pause();
                    }
                }
                p.acquire();
            }
            p.barrier();
        }
        p.work(t, k);
        p.stores_done();
        p.barrier();
        if (p.tid() == 0) p.store_release(c.flags + k, t + 1);
    }
}

}  // namespace tnrd
