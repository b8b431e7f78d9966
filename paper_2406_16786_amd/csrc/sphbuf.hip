// MI355X (gfx950, CDNA4) kernels and C ABI of the arbitrary-positioned SPH
// in-/outlet buffer update (arXiv 2406.16786, Section 3, Algorithms 1-3).
//
// Per step of a context (the merged step, the default): a build, then an update.
//   build, count pass: cell key of every particle (FP32 floor) and its rank -- in
//     its cell (k_count: one atomic per run of equal keys in a wave) or in a bucket
//     of consecutive cells (k_bk_count: LDS histogram, one global atomic per
//     workgroup and bucket); the cover cells' particles near a check region are
//     listed as candidates;
//   update, cells pass with the candidates' exact tests beside it (rotation into
//     the buffer frame in FP32 with a hi/lo origin, the decisions inside the guard
//     band redone in FP64 exactly as defined, events appended by ballot/mbcnt wave
//     compaction): k_scan (look-back scan of the cell counts) and k_scatter_cls, or
//     k_bk_scatter_cls and k_bk_sort (a counting sort inside each bucket);
//   k_finalize: status checks before any write, the event lists sorted in LDS,
//     recycle, relabel, hole refill from the tail, append.
// Which build runs is timed and chosen per context (SPH_BUILD_AUTO).  The
// cover-cell walk (SPH_UPDATE_CELLS) classifies the particles of the cover cells
// from the finished cell list (k_classify_local); the full scan (k_filter_full,
// k_classify_cand) tests every particle; batches build by the counting sort.
// Everything reads the live count from device memory, so the whole chain can be
// enqueued without host round trips.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "sphbuf.h"
#include "sphbuf_internal.h"

using sphbuf::BufDev;

namespace {

constexpr int kWave = 64;
constexpr int kBuildBlock = 256;
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kClassifyBlock = 256;
constexpr int kFinBlock = 1024;
constexpr unsigned kMaxEv = SPH_MAX_EVENTS_LIMIT;
static_assert(kMaxEv % kWave == 0, "event lists are sorted in 64-key chunks");
constexpr int kRelPerEvent = 4;
constexpr int kMaxPartBlocks = 8192;  // upper bound on classify / full-scan grid sizes

constexpr unsigned kIn = 1u, kBox = 2u, kFront = 4u, kBack = 8u;
constexpr int kEvNone = 0, kEvGen = 1, kEvDel = 2;

// Cell grid.  Dense: key = ix + dims0 * (iy + dims1 * iz).  Brick-sparse
// (blog2 > 0): cells are grouped in bricks of 2^blog2 cells per axis; an active
// brick with slot s owns keys s * B + local (B cells per brick, local = lx + b *
// (ly + b * lz)); every cell of an inactive brick maps to the single overflow key.
struct Grid {
    float lo[3];
    float inv_cs;
    int32_t dims[3];
    int32_t dim;
    int32_t blog2;
    int32_t bdims[3];
    const int32_t *brick_slot;  // per brick: slot or -1
    uint32_t overflow_key;
};

struct Parts {
    float *pos[3];
    float *car[SPH_MAX_CARRIED];
    int32_t nc;
    int32_t dim;
    int32_t *label;
    int64_t *id;
    int64_t *n_dev;
    int64_t capacity;
};

// Event lists are split into kSeg segments, each with its own counters on a
// 128-byte line of its own: a wave appends to segment (wave index mod kSeg), so
// concurrent waves spread their slot atomics over kSeg addresses instead of
// queueing on one (same-address device atomics serialise at about 12 ns each).
constexpr int kSeg = 16;

struct SegCtr {
    unsigned int n_gen, n_del, n_rel;
    unsigned int pad[29];
};

// Device-resident counters and library state.
struct Ctl {
    SegCtr seg[kSeg];
    unsigned int tile_counter;
    unsigned int nonfinite_build;  // set by the count phase of a build that met a non-finite position
    unsigned int nonfinite_seen;   // the latest completed build's flag (moved there by its scan phase)
    unsigned int nonfinite_full;   // set by a full-scan classify; consumed by its finalize
    unsigned int scan_fault;       // set if a look-back wait ran past its spin limit
    unsigned int fin_ticket;       // finalize blocks that have read the counters
    unsigned int bc_status;        // outcome of the last boundary-condition or rotation pass
    unsigned int cand_overflow;    // the full scan's candidate list overflowed (consumed by its finalize)
    unsigned long long cand_count; // candidates appended by the full scan's filter
    long long next_id;
    long long n_labelled[16];
    unsigned int ident_bad;
    unsigned int pad1;
    unsigned long long ident_count[16];
    int64_t n_built;               // particles of the latest count pass (what its scatter places)
    unsigned int bk_ticket;        // bucketed build: count workgroups that have finished
    unsigned int pad2;
    int32_t run_cnt[16];           // cover runs of each buffer (in its range of the per-buffer run lists)
    int32_t n_runs;                // runs of the compact list the classify and BC kernels walk
    int32_t cover_fault;           // a turned buffer's cover needed more runs than its range holds
};

// ------------------------------------------------------------ device utils --

__device__ __forceinline__ unsigned mbcnt(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Live count clamped to [0, capacity]: a bad count can never send an index out
// of the arrays (the finalize step reports it as an argument error).
__device__ __forceinline__ int64_t live_count(const int64_t *n_dev, int64_t capacity) {
    const int64_t n = *n_dev;
    return n < 0 ? 0 : (n > capacity ? capacity : n);
}

// Blocks are dispatched round-robin over the 8 XCDs; renumber them so that each
// XCD owns a contiguous range of logical blocks (and so of particles).
__device__ __forceinline__ int logical_block() {
    const int b = blockIdx.x, g = gridDim.x;
    if (g & 7) return b;
    return (b & 7) * (g >> 3) + (b >> 3);
}

// Dense cell coordinates: floor(fl32(fl32(x - lo) * inv_cs)) clamped to the grid
// (particles outside the bounds land in edge cells; NaN lands in cell 0).
__device__ __forceinline__ void cell_coords(const Grid &g, float x, float y, float z, uint32_t &ix, uint32_t &iy,
                                            uint32_t &iz) {
    float fx = floorf((x - g.lo[0]) * g.inv_cs);
    float fy = floorf((y - g.lo[1]) * g.inv_cs);
    fx = fminf(fmaxf(fx, 0.0f), (float)(g.dims[0] - 1));
    fy = fminf(fmaxf(fy, 0.0f), (float)(g.dims[1] - 1));
    ix = (uint32_t)fx;
    iy = (uint32_t)fy;
    iz = 0;
    if (g.dim == 3) {
        float fz = floorf((z - g.lo[2]) * g.inv_cs);
        fz = fminf(fmaxf(fz, 0.0f), (float)(g.dims[2] - 1));
        iz = (uint32_t)fz;
    }
}

// Key of the cell with (in-range) coordinates ix, iy, iz: dense row-major, or the
// brick slot and the position inside the brick (cells of inactive bricks share the
// overflow key).
__device__ __forceinline__ uint32_t key_of_cell(const Grid &g, uint32_t ix, uint32_t iy, uint32_t iz) {
    if (g.blog2 == 0) return ix + (uint32_t)g.dims[0] * (iy + (uint32_t)g.dims[1] * iz);
    const uint32_t b = (uint32_t)g.blog2, m = (1u << b) - 1u;
    const uint32_t brick = (ix >> b) + (uint32_t)g.bdims[0] * ((iy >> b) + (uint32_t)g.bdims[1] * (iz >> b));
    const int32_t slot = g.brick_slot[brick];
    if (slot < 0) return g.overflow_key;
    const uint32_t local = (ix & m) + ((iy & m) << b) + (g.dim == 3 ? ((iz & m) << (2 * b)) : 0u);
    return ((uint32_t)slot << (g.dim * b)) + local;
}

__device__ __forceinline__ uint32_t cell_key(const Grid &g, float x, float y, float z) {
    uint32_t ix, iy, iz;
    cell_coords(g, x, y, z, ix, iy, iz);
    return key_of_cell(g, ix, iy, iz);
}

// Exact FP64 decision: local coordinates r' = Q (r - O') evaluated as
// ((q0 d0 + q1 d1) + q2 d2) with every product and sum rounded separately (no
// FMA), then the strict comparisons of the box and the check region.
__device__ __attribute__((noinline)) unsigned classify64(const BufDev &b, int dim, float x, float y, float z) {
#pragma clang fp contract(off)
    const double d0 = __dadd_rn((double)x, -b.o[0]);
    const double d1 = __dadd_rn((double)y, -b.o[1]);
    double l0, l1, l2 = 0.0;
    if (dim == 2) {
        l0 = __dadd_rn(__dmul_rn(b.q[0], d0), __dmul_rn(b.q[1], d1));
        l1 = __dadd_rn(__dmul_rn(b.q[3], d0), __dmul_rn(b.q[4], d1));
    } else {
        const double d2 = __dadd_rn((double)z, -b.o[2]);
        l0 = __dadd_rn(__dadd_rn(__dmul_rn(b.q[0], d0), __dmul_rn(b.q[1], d1)), __dmul_rn(b.q[2], d2));
        l1 = __dadd_rn(__dadd_rn(__dmul_rn(b.q[3], d0), __dmul_rn(b.q[4], d1)), __dmul_rn(b.q[5], d2));
        l2 = __dadd_rn(__dadd_rn(__dmul_rn(b.q[6], d0), __dmul_rn(b.q[7], d1)), __dmul_rn(b.q[8], d2));
    }
    const double a0 = fabs(l0), a1 = fabs(l1), a2 = fabs(l2);
    unsigned bits = 0;
    if (a0 < b.thr[3] && a1 < b.thr[4] && (dim == 2 || a2 < b.thr[5])) bits |= kIn;
    if (a0 < b.thr[0] && a1 < b.thr[1] && (dim == 2 || a2 < b.thr[2])) bits |= kBox;
    if (l0 > b.thr[0]) bits |= kFront;
    if (l0 < -b.thr[0]) bits |= kBack;
    return bits;
}

// Bulk FP32 decision with the FP64 recheck inside the guard band.
__device__ __forceinline__ unsigned classify(const BufDev &b, int dim, float x, float y, float z) {
    const float d0 = (x - b.ohi[0]) - b.olo[0];
    const float d1 = (y - b.ohi[1]) - b.olo[1];
    const float d2 = dim == 3 ? (z - b.ohi[2]) - b.olo[2] : 0.0f;
    if (d0 * d0 + d1 * d1 + d2 * d2 > b.rsq) return 0u;  // outside a sphere holding C_k
    const float l0 = b.qf[0] * d0 + b.qf[1] * d1 + b.qf[2] * d2;
    const float l1 = b.qf[3] * d0 + b.qf[4] * d1 + b.qf[5] * d2;
    const float l2 = b.qf[6] * d0 + b.qf[7] * d1 + b.qf[8] * d2;
    const float a0 = fabsf(l0), a1 = fabsf(l1), a2 = fabsf(l2);
    const float g = b.guard;
    bool near = fabsf(a0 - b.thrf[0]) < g || fabsf(a0 - b.thrf[3]) < g || fabsf(a1 - b.thrf[1]) < g ||
                fabsf(a1 - b.thrf[4]) < g;
    if (dim == 3) near = near || fabsf(a2 - b.thrf[2]) < g || fabsf(a2 - b.thrf[5]) < g;
    if (near) return classify64(b, dim, x, y, z);
    unsigned bits = 0;
    if (a0 < b.thrf[3] && a1 < b.thrf[4] && (dim == 2 || a2 < b.thrf[5])) bits |= kIn;
    if (a0 < b.thrf[0] && a1 < b.thrf[1] && (dim == 2 || a2 < b.thrf[2])) bits |= kBox;
    if (l0 > b.thrf[0]) bits |= kFront;
    if (l0 < -b.thrf[0]) bits |= kBack;
    return bits;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Outcome of one candidate of buffer k (0-based): event kind, label after the
// update (-1: particle not in C_k, untouched).
struct Outcome {
    int ev;
    int newlab;
    bool mine;
};

__device__ __forceinline__ Outcome decide(const BufDev &b, int k, int dim, unsigned bits, int lab, float x,
                                          float y, float z) {
    Outcome o{kEvNone, -1, false};
    if (!(bits & kIn)) return o;
    const int me = k + 1;
    o.mine = (lab == me);
    o.newlab = lab;
    if (b.kind == SPH_INLET) {  // Algorithm 1: labels fixed after identification
        if (o.mine && (bits & kFront)) o.ev = kEvGen;
    } else if (b.kind == SPH_OUTLET) {  // Algorithm 2
        if (bits & kFront) {
            o.ev = kEvDel;
        } else {
            o.newlab = (bits & kBox) ? me : (o.mine ? 0 : lab);
        }
    } else {  // Algorithm 3
        if (o.mine && (bits & kFront)) {
            o.ev = kEvGen;
            // relabel on the recycled position r - a d (FP64, rounded to FP32)
            const float xr = (float)((double)x - b.shift[0]);
            const float yr = (float)((double)y - b.shift[1]);
            const float zr = dim == 3 ? (float)((double)z - b.shift[2]) : 0.0f;
            const unsigned b2 = classify(b, dim, xr, yr, zr);
            if (b2 & kIn) o.newlab = (b2 & kBox) ? me : 0;
        } else if (o.mine && (bits & kBack)) {
            o.ev = kEvDel;
        } else {
            o.newlab = (bits & kBox) ? me : (o.mine ? 0 : lab);
        }
    }
    return o;
}

// Event storage: kSeg segments of cap_ev generation / deletion slots and cap_rel
// relabel slots.  Slot t of segment g is entry g * cap + t of each array; a
// duplicate payload takes 3 + n_carried floats.
struct EventArgs {
    Ctl *ctl;
    uint32_t *gen_idx;         // [kSeg * cap_ev] generated-source index
    float *gen_new;            // [kSeg * cap_ev * 4] its recycled position and density
    float *dup;                // [kSeg * cap_ev * (3 + nc)] its pre-recycle position and carried fields
    uint32_t *del_idx;         // [kSeg * cap_ev] deleted index
    unsigned long long *rel;   // [kSeg * cap_rel] (index << 32) | new label
    unsigned cap_ev;
    unsigned cap_rel;
    unsigned *part;  // label counts, kCountReplicas copies: part[(copy * 16 + k) * 2 + {0: found, 1: post}]
    int32_t rho_field;  // carried index of the density, or -1
};

// Label counts of each buffer: waves add into LDS, then one thread per buffer
// adds the block's total into one of kCountReplicas copies of the global
// counters (picked by block index, so concurrent blocks rarely hit the same
// address); the finalize step sums the copies and clears them.
constexpr int kCountReplicas = 64;

__device__ __forceinline__ void block_counts_init(unsigned *s_cnt) {
    if (threadIdx.x < 2 * SPH_MAX_BUFFERS) s_cnt[threadIdx.x] = 0u;
}
__device__ __forceinline__ void block_counts_store(const EventArgs &e, const unsigned *s_cnt, int nb) {
    if (threadIdx.x < 2 * nb && s_cnt[threadIdx.x])
        atomicAdd(&e.part[(size_t)(blockIdx.x % kCountReplicas) * 2 * SPH_MAX_BUFFERS + threadIdx.x],
                  s_cnt[threadIdx.x]);
}

// Emit the wave's events for buffer k into event segment seg and accumulate its
// label counts.  The three slot atomics are issued together.  A generating lane
// also captures the duplicate's payload (the state before the recycle) and the
// recycled position r - a d (FP64, rounded to FP32): nothing of the caller's
// arrays is written here, so a failed status check can still leave them
// untouched, and the finalize step has no random reads left to do.
template <bool kPrefetched>  // carried fields already in carv, or loaded here
__device__ __forceinline__ void emit(const EventArgs &e, const Parts &p, const BufDev &b, int k, int seg,
                                     bool valid, int64_t i, int lab, const Outcome &o, float x, float y, float z,
                                     const float (&carv)[SPH_MAX_CARRIED], unsigned long long &found,
                                     unsigned long long &post) {
    const bool in = valid && o.newlab >= 0;
    if (in && o.mine) found++;
    if (in && o.ev != kEvDel && o.newlab == k + 1) post++;
    const bool pg = in && o.ev == kEvGen, pd = in && o.ev == kEvDel, pr = in && o.ev != kEvDel && o.newlab != lab;
    const unsigned long long mg = __ballot(pg), md = __ballot(pd), mr = __ballot(pr);
    if ((mg | md | mr) == 0ull) return;
    SegCtr &sc = e.ctl->seg[seg];
    const int lane = lane_id();
    const int lg = mg ? __ffsll((long long)mg) - 1 : 0, ld = md ? __ffsll((long long)md) - 1 : 0,
              lr = mr ? __ffsll((long long)mr) - 1 : 0;
    unsigned bg = 0, bd = 0, br = 0;
    if (mg && lane == lg) bg = atomicAdd(&sc.n_gen, (unsigned)__popcll(mg));
    if (md && lane == ld) bd = atomicAdd(&sc.n_del, (unsigned)__popcll(md));
    if (mr && lane == lr) br = atomicAdd(&sc.n_rel, (unsigned)__popcll(mr));
    bg = __shfl(bg, lg);
    bd = __shfl(bd, ld);
    br = __shfl(br, lr);
    if (pg) {
        const unsigned s = bg + mbcnt(mg);
        if (s < e.cap_ev) {
            const size_t ev = (size_t)seg * e.cap_ev + s;
            e.gen_idx[ev] = (uint32_t)i;
            const float r[3] = {x, y, z};
            float *d = e.dup + ev * (size_t)(3 + p.nc);
            for (int c = 0; c < p.dim; ++c) {
                d[c] = r[c];
                e.gen_new[4 * ev + c] = (float)((double)r[c] - b.shift[c]);
            }
            float rho = 0.0f;
            if constexpr (kPrefetched) {
#pragma unroll
                for (int f = 0; f < SPH_MAX_CARRIED; ++f) {
                    if (f >= p.nc) continue;
                    d[3 + f] = carv[f];
                    if (f == e.rho_field) rho = carv[f];
                }
            } else {
                for (int f = 0; f < p.nc; ++f) {
                    const float v = p.car[f][i];
                    d[3 + f] = v;
                    if (f == e.rho_field) rho = v;
                }
            }
            // density of the recycled particle: the boundary value at a pressure
            // boundary (Eq. postulate-density), otherwise unchanged
            if (e.rho_field >= 0) e.gen_new[4 * ev + 3] = b.bc_kind == SPH_BC_PRESSURE ? b.rho_rec : rho;
        }
    }
    if (pd) {
        const unsigned s = bd + mbcnt(md);
        if (s < e.cap_ev) e.del_idx[(size_t)seg * e.cap_ev + s] = (uint32_t)i;
    }
    if (pr) {
        const unsigned s = br + mbcnt(mr);
        if (s < e.cap_rel) e.rel[(size_t)seg * e.cap_rel + s] = ((unsigned long long)i << 32) | (unsigned)o.newlab;
    }
}

// --------------------------------------------------------------- K0 build --
//
// Counting sort of the particle indices by cell in three launches:
//   count  : cell key of every particle and its rank among the particles of its
//            cell (one returning atomic per run of equal keys in consecutive
//            lanes), stored packed in 32 bits: key << rbits | rank, where rbits
//            is what the largest key leaves free.  A rank that does not fit
//            (rank >= 2^rbits - 1, a very crowded cell) stores the all-ones
//            marker and spills the full (key, rank) to a 64-bit buffer;
//   scan   : exclusive prefix of the counts -> cell_start, counts zeroed;
//   scatter: cell_idx[cell_start[key] + rank] = i.
// The order inside a cell is whatever the atomics make it; nothing downstream
// depends on it.

// Cell keys of J particles (none = the key of an invalid one).  On a brick grid
// the J brick-slot loads are issued together before any key is formed: one
// round trip per group, not one per particle.  Coordinates are clamped (NaN lands
// in cell 0), so every brick index is in range, invalid lanes included.
template <int J>
__device__ __forceinline__ void keys_of(const Grid &g, const float (&px)[J], const float (&py)[J],
                                        const float (&pz)[J], const bool (&valid)[J], uint32_t none,
                                        uint32_t (&key)[J], bool &bad) {
    uint32_t ix[J], iy[J], iz[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (valid[j]) bad |= !(isfinite(px[j]) && isfinite(py[j]) && isfinite(pz[j]));
        cell_coords(g, px[j], py[j], pz[j], ix[j], iy[j], iz[j]);
    }
    if (g.blog2 == 0) {
#pragma unroll
        for (int j = 0; j < J; ++j) key[j] = ix[j] + (uint32_t)g.dims[0] * (iy[j] + (uint32_t)g.dims[1] * iz[j]);
    } else {
        const uint32_t b = (uint32_t)g.blog2, m = (1u << b) - 1u;
        int32_t slot[J];
#pragma unroll
        for (int j = 0; j < J; ++j)
            slot[j] = g.brick_slot[(ix[j] >> b) +
                                   (uint32_t)g.bdims[0] * ((iy[j] >> b) + (uint32_t)g.bdims[1] * (iz[j] >> b))];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t local = (ix[j] & m) + ((iy[j] & m) << b) + (g.dim == 3 ? ((iz[j] & m) << (2 * b)) : 0u);
            key[j] = slot[j] < 0 ? g.overflow_key : ((uint32_t)slot[j] << (g.dim * b)) + local;
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
        if (!valid[j]) key[j] = none;
}

template <int J>
__device__ __forceinline__ void group_keys(const Grid &g, const float (&px)[J], const float (&py)[J],
                                           const float (&pz)[J], const bool (&valid)[J], uint32_t (&key)[J],
                                           bool &bad) {
    keys_of<J>(g, px, py, pz, valid, 0xffffffffu, key, bad);
}

// Runs of equal keys in consecutive lanes: the run's first lane (head) issues one
// returning atomic for the run's length; old[j] is then in flight.
template <int J>
__device__ __forceinline__ void group_runs_issue(int32_t *count, const uint32_t (&key)[J], const bool (&valid)[J],
                                                 int lane, int (&my_head)[J], int (&old)[J]) {
    int len[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t prev = __shfl_up(key[j], 1);
        const bool head = !valid[j] || lane == 0 || key[j] != prev;
        const unsigned long long heads = __ballot(head);
        const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        my_head[j] = 63 - __clzll((long long)(heads & le));
        const unsigned long long gt = heads & ~le;
        len[j] = (gt ? __ffsll((long long)gt) - 1 : 64) - my_head[j];
        if (!valid[j]) len[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        old[j] = len[j];  // any value already in the register: no copy that would wait on the atomic before
        if (len[j] > 0 && lane == my_head[j]) old[j] = atomicAdd(&count[key[j]], len[j]);
    }
}

// Rank of each lane in its cell: the run's base from its head plus the offset in the run.
template <int J>
__device__ __forceinline__ void group_ranks(const int (&my_head)[J], const int (&old)[J], int lane,
                                            int32_t (&rank)[J]) {
#pragma unroll
    for (int j = 0; j < J; ++j) rank[j] = __shfl(old[j], my_head[j]) + (lane - my_head[j]);
}

// Element o of an array whose base is uniform, addressed by a 32-bit byte offset
// (o * sizeof(T) < 2^32): the address is base + offset in one memory instruction,
// no 64-bit address arithmetic per lane.
template <class T>
__device__ __forceinline__ const T &at32(const T *base, uint32_t o) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (size_t)(uint32_t)(o * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T &at32(T *base, uint32_t o) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (size_t)(uint32_t)(o * (uint32_t)sizeof(T)));
}

constexpr int kCountBatch = 2;
constexpr int64_t kCountPer = 2048;  // particles per count workgroup (single domain)

// FP32 check-region test widened by the guard band: true for every member of C_k.
// (The caller first tests the axis-aligned box bmin..bmax, rounded outward: it
// never drops a member, and a NaN coordinate fails it.)
__device__ __forceinline__ bool near_region(const BufDev &b, int dim, float x, float y, float z) {
    const float d0 = (x - b.ohi[0]) - b.olo[0];
    const float d1 = (y - b.ohi[1]) - b.olo[1];
    const float d2 = dim == 3 ? (z - b.ohi[2]) - b.olo[2] : 0.0f;
    const float l0 = b.qf[0] * d0 + b.qf[1] * d1 + b.qf[2] * d2;
    const float l1 = b.qf[3] * d0 + b.qf[4] * d1 + b.qf[5] * d2;
    const float l2 = b.qf[6] * d0 + b.qf[7] * d1 + b.qf[8] * d2;
    const float g = b.guard;
    return fabsf(l0) < b.thrf[3] + g && fabsf(l1) < b.thrf[4] + g && (dim == 2 || fabsf(l2) < b.thrf[5] + g);
}

// ------------------------------------------------- merged step: candidates --
//
// The count pass of a merged step lists its candidates: the particles of the
// buffers' cover cells (bit k of the cell's cover mask) that lie near check region
// k.  A workgroup gathers them in LDS (particle offset in the workgroup << 4 |
// buffer; one LDS atomic per wave) and appends them to the candidate list with one
// global atomic; a workgroup with more than Cap of them appends the rest one by
// one.  E holds the offset: 16 bits for workgroups of at most 4096 particles.

template <typename E, int Cap>
struct CandLds {
    E e[Cap];
    unsigned n;
    unsigned long long base;
};

// What the candidate test reads of a buffer, kept in LDS (the full record is 15
// times larger): the FP32 frame, the widened half-extents, the axis-aligned box.
struct BufNear {
    float qf[9], ohi[3], olo[3];
    float lim[3];        // thrf[3..5] + guard, summed in FP32 as the full scan's filter does
    float bmin[3], bmax[3];
};

__device__ __forceinline__ void near_load(BufNear *sb, const BufDev *bufs, int nb) {
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        const BufDev &b = bufs[k];
        BufNear n;
        for (int q = 0; q < 9; ++q) n.qf[q] = b.qf[q];
        for (int q = 0; q < 3; ++q) {
            n.ohi[q] = b.ohi[q];
            n.olo[q] = b.olo[q];
            n.lim[q] = b.thrf[3 + q] + b.guard;
            n.bmin[q] = b.bmin[q];
            n.bmax[q] = b.bmax[q];
        }
        sb[k] = n;
    }
}

// near_region's test (and the box in front of it) on the LDS record.
__device__ __forceinline__ bool near_test(const BufNear &b, int dim, float x, float y, float z) {
    if (!(x > b.bmin[0] && x < b.bmax[0] && y > b.bmin[1] && y < b.bmax[1] && z > b.bmin[2] && z < b.bmax[2]))
        return false;
    const float d0 = (x - b.ohi[0]) - b.olo[0];
    const float d1 = (y - b.ohi[1]) - b.olo[1];
    const float d2 = dim == 3 ? (z - b.ohi[2]) - b.olo[2] : 0.0f;
    const float l0 = b.qf[0] * d0 + b.qf[1] * d1 + b.qf[2] * d2;
    const float l1 = b.qf[3] * d0 + b.qf[4] * d1 + b.qf[5] * d2;
    const float l2 = b.qf[6] * d0 + b.qf[7] * d1 + b.qf[8] * d2;
    return fabsf(l0) < b.lim[0] && fabsf(l1) < b.lim[1] && (dim == 2 || fabsf(l2) < b.lim[2]);
}

struct CandArgs {
    const uint16_t *cover;   // per cell: cover bits of the buffers
    const BufDev *bufs;
    int nb;
    unsigned long long *cand;  // (index << 4) | buffer
    int64_t cap_cand;
};

// Q particles per lane at once (cm = 0 where there is nothing to test; z = 0 in
// 2-D); called by whole waves.  One branch, one prefix sum and one LDS atomic per
// wave for all Q, and none of them when no lane has a cover bit or nothing passes
// the test.
template <int Q, typename E, int Cap>
__device__ __forceinline__ void cand_append(const CandArgs &c, const BufNear *sb, int dim, const uint32_t (&cm)[Q],
                                            const float (&x)[Q], const float (&y)[Q], const float (&z)[Q],
                                            const uint32_t (&local)[Q], const int64_t (&idx)[Q], int lane,
                                            CandLds<E, Cap> &L, Ctl *ctl) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) any |= cm[q] != 0u;
    if (__ballot(any) == 0ull) return;  // wave-uniform
    uint32_t cb[Q];
    unsigned mine = 0u;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        cb[q] = 0u;
        uint32_t m = cm[q];
        while (m) {
            const int k = __ffs(m) - 1;
            m &= m - 1u;
            if (near_test(sb[k], dim, x[q], y[q], z[q])) cb[q] |= 1u << k;
        }
        mine += (unsigned)__popc(cb[q]);
    }
    if (__ballot(mine != 0u) == 0ull) return;  // cover cells, but nothing near a region
    unsigned incl = mine;
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    const unsigned tot = __shfl(incl, kWave - 1);
    unsigned at = 0u;
    if (lane == 0) at = atomicAdd(&L.n, tot);
    at = __shfl(at, 0) + (incl - mine);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        uint32_t m = cb[q];
        while (m) {
            const int k = __ffs(m) - 1;
            m &= m - 1u;
            if (at < (unsigned)Cap) {
                L.e[at] = (E)((local[q] << 4) | (uint32_t)k);
            } else {  // a workgroup full of candidates: the rest one by one
                const unsigned long long g = atomicAdd(&ctl->cand_count, 1ull);
                if (g < (unsigned long long)c.cap_cand)
                    c.cand[g] = ((unsigned long long)idx[q] << 4) | (unsigned long long)k;
                else
                    ctl->cand_overflow = 1u;
            }
            ++at;
        }
    }
}

// The workgroup's gathered candidates into the list (after a barrier; has barriers).
template <typename E, int Cap>
__device__ __forceinline__ void cand_flush(const CandArgs &c, CandLds<E, Cap> &L, int64_t s0, Ctl *ctl) {
    const unsigned nc = min(L.n, (unsigned)Cap);
    if (threadIdx.x == 0) L.base = nc ? atomicAdd(&ctl->cand_count, (unsigned long long)nc) : 0ull;
    __syncthreads();
    for (unsigned e = threadIdx.x; e < nc; e += blockDim.x) {
        const unsigned long long g = L.base + e;
        const uint32_t v = (uint32_t)L.e[e];
        if (g < (unsigned long long)c.cap_cand)
            c.cand[g] = ((unsigned long long)(s0 + (v >> 4)) << 4) | (unsigned long long)(v & 15u);
        else
            ctl->cand_overflow = 1u;
    }
}

struct CountArgs {
    const float *x, *y, *z;
    const int64_t *n_dev;
    int64_t capacity;
    Grid g;
    int32_t *count;
    uint32_t *packed;               // key << rbits | rank, or all ones
    unsigned long long *spill;      // (key << 32 | rank) of the particles marked all ones
    int32_t rbits;
    unsigned long long *tile_state;
    int64_t n_tiles;
    Ctl *ctl;
    unsigned int *nonfinite;        // flag to raise on a non-finite position
    CandArgs c;                     // merged step: the candidate list
};

template <bool kCand>
__device__ __forceinline__ void count_body(const CountArgs &a, const int lb, const int G) {
    const int64_t N = live_count(a.n_dev, a.capacity);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nthreads = (int64_t)G * blockDim.x;
    // reset the scan's tile state for this build
    for (int64_t t = (int64_t)lb * blockDim.x + threadIdx.x; t < a.n_tiles; t += nthreads) a.tile_state[t] = 0ull;
    if (lb == 0 && threadIdx.x == 0) {
        a.ctl->tile_counter = 0u;
        a.ctl->scan_fault = 0u;
        a.ctl->n_built = N;
    }
    // Each logical block walks kCountBatch * W slices of L particles, one per wave and
    // row (kCountBatch rows per wave): at every step the block's waves take the next
    // 64 particles of each of their slices, so the particles whose atomics are in
    // flight together lie a slice apart -- beyond the few lattice rows that share a
    // cell -- and rarely meet on one counter (same-address atomics queue at the
    // memory side).  One contiguous segment of the block is cut into its slices.
    const int W = (int)(blockDim.x / kWave);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // uniform: scalar row bases
    const int64_t slices = (int64_t)W * kCountBatch;
    const int64_t per = ((N + G - 1) / G + slices * kWave - 1) / (slices * kWave) * (slices * kWave);
    const int64_t L = per / slices;
    const int64_t s0 = (int64_t)lb * per;
    bool bad = false;
    const uint32_t rmask = (1u << a.rbits) - 1u;
    if (s0 >= N) return;  // block-uniform: no particle here
    __shared__ BufNear sb[kCand ? SPH_MAX_BUFFERS : 1];
    __shared__ std::conditional_t<kCand, CandLds<uint32_t, 2048>, char> s_cand;
    if constexpr (kCand) {
        near_load(sb, a.c.bufs, a.c.nb);
        if (threadIdx.x == 0) s_cand.n = 0u;
        __syncthreads();
    }
    constexpr int J = kCountBatch;
    const uint32_t L32 = (uint32_t)L;
    // per row: first particle, particles in it (slice-relative 32-bit offsets from
    // uniform base pointers)
    int64_t rb[J];
    uint32_t nr[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int64_t q = (int64_t)j * W + w;
        rb[j] = s0 + q * L;
        const int64_t left = N - rb[j];
        nr[j] = left <= 0 ? 0u : (left >= L ? L32 : (uint32_t)left);
    }
    const bool d3 = a.g.dim == 3;
    const float *xr[J], *yr[J], *zr[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        xr[j] = a.x + rb[j];
        yr[j] = a.y + rb[j];
        zr[j] = d3 ? a.z + rb[j] : a.x + rb[j];
    }
    // Software pipelined: once a step has its keys it issues the next step's position
    // loads, then its run detection and atomics, so the two round trips overlap.
    float px[J], py[J], pz[J];
    // The positions are loaded without a branch (lanes past a row's end re-read its
    // first particle, rows with none the array's first; a 2-D z is a copy of x,
    // unused): behind a branch the compiler waits for every outstanding access, the
    // previous step's stores included, before the next loads.
    const float *xl[J], *yl[J], *zl[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        xl[j] = nr[j] ? xr[j] : a.x;
        yl[j] = nr[j] ? yr[j] : a.y;
        zl[j] = nr[j] ? zr[j] : (d3 ? a.z : a.x);
    }
    auto load = [&](uint32_t it) {
        const uint32_t o = it + (uint32_t)lane;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t oc = o < nr[j] ? o : 0u;
            px[j] = at32(xl[j], oc);
            py[j] = at32(yl[j], oc);
            pz[j] = at32(zl[j], oc);
        }
    };
    load(0);
    for (uint32_t it = 0; it < L32; it += kWave) {
        const uint32_t o = it + (uint32_t)lane;
        uint32_t key[J];
        int32_t rank[J];
        bool valid[J];
#pragma unroll
        for (int j = 0; j < J; ++j) valid[j] = o < nr[j];
        group_keys<J>(a.g, px, py, pz, valid, key, bad);
        // merged step: the cover bits of the keys' cells, loaded before the next
        // positions and the atomics (their positions kept for the tests)
        uint32_t cm[J];
        float cx[J], cy[J], cz[J];
        if constexpr (kCand) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                cm[j] = valid[j] ? a.c.cover[key[j]] : 0u;
                cx[j] = px[j];
                cy[j] = py[j];
                cz[j] = d3 ? pz[j] : 0.0f;
            }
        }
        const uint32_t nx = it + kWave;
        if (nx < L32) load(nx);  // block-uniform; the positions are consumed
        int my_head[J], old[J];
        group_runs_issue<J>(a.count, key, valid, lane, my_head, old);
        group_ranks<J>(my_head, old, lane, rank);
#pragma unroll
        for (int j = 0; j < kCountBatch; ++j) {
            if (!valid[j]) continue;
            if ((uint32_t)rank[j] < rmask) {
                at32(a.packed + rb[j], o) = (key[j] << a.rbits) | (uint32_t)rank[j];
            } else {
                at32(a.packed + rb[j], o) = 0xffffffffu;
                at32(a.spill + rb[j], o) = ((unsigned long long)key[j] << 32) | (unsigned)rank[j];
            }
        }
        if constexpr (kCand) {
            uint32_t loc[J];
            int64_t idx[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                idx[j] = rb[j] + (int64_t)o;
                loc[j] = (uint32_t)(idx[j] - s0);
            }
            cand_append<J>(a.c, sb, a.g.dim, cm, cx, cy, cz, loc, idx, lane, s_cand, a.ctl);
        }
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(a.nonfinite, 1u);
    if constexpr (kCand) {  // the workgroup's candidates into the list
        __syncthreads();
        cand_flush(a.c, s_cand, s0, a.ctl);
    }
}

template <bool kCand>
__global__ __launch_bounds__(kBuildBlock) void k_count(CountArgs a) {
    count_body<kCand>(a, logical_block(), gridDim.x);
}

// Decoupled look-back scan state: bits 62..63 = flag (1 aggregate, 2 prefix),
// low 32 bits = value.
constexpr unsigned long long kAgg = 1ull << 62, kPre = 2ull << 62;

__device__ __forceinline__ unsigned long long load_state(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_state(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct ScanArgs {
    int32_t *count;        // C + 1 entries (last is always 0); zeroed on the way
    int32_t *cell_start;   // C + 1 entries
    int64_t m;             // C + 1
    unsigned long long *tile_state;
    Ctl *ctl;
};

// One tile of kScanTile counts per block: coalesced loads through LDS into
// per-thread runs of kScanItems, wave and block scans, a decoupled look-back
// over the preceding tiles (tile order from an atomic ticket, so a tile only
// ever waits on tiles that started before it), and coalesced stores.
struct ScanLds {
    unsigned tile;
    int wave[kScanBlock / kWave];
    int excl;
    int buf[kScanTile + kScanTile / 32];  // padded: index j at j + j / 32
};

__device__ __forceinline__ void scan_body(const ScanArgs &a, ScanLds &L) {
    unsigned &s_tile = L.tile;
    auto &s_wave = L.wave;
    int &s_excl = L.excl;
    auto &s_buf = L.buf;
    if (threadIdx.x == 0) {
        s_tile = atomicAdd(&a.ctl->tile_counter, 1u);
        if (s_tile == 0u) {  // the count phase is complete: keep its verdict for the next update
            a.ctl->nonfinite_seen = a.ctl->nonfinite_build;
            a.ctl->nonfinite_build = 0u;
        }
    }
    __syncthreads();
    const unsigned tile = s_tile;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t t0 = (int64_t)tile * kScanTile;
    // every count of the tile is loaded before any is cleared: a wave waiting for a
    // load also waits for the stores it issued before it
    int vq[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t gj = t0 + q * kScanBlock + (int)threadIdx.x;
        vq[q] = gj < a.m ? a.count[gj] : 0;
    }
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int j = q * kScanBlock + (int)threadIdx.x;
        const int64_t gj = t0 + j;
        if (gj < a.m && vq[q] != 0) a.count[gj] = 0;  // empty cells are left alone (no write)
        s_buf[j + j / 32] = vq[q];
    }
    __syncthreads();
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int j = (int)threadIdx.x * kScanItems + q;
        v[q] = s_buf[j + j / 32];
        sum += v[q];
    }
    // inclusive wave scan of per-thread sums
    int incl = sum;
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    int wave_off = 0, total = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        if (w < wave) wave_off += s_wave[w];
        total += s_wave[w];
    }
    // publish the tile aggregate, then look back (wave 0)
    if (wave == 0) {
        if (lane == 0) store_state(&a.tile_state[tile], (tile == 0 ? kPre : kAgg) | (unsigned)total);
        int excl = 0;
        if (tile > 0) {
            int64_t t = (int64_t)tile - 1;
            while (true) {
                const int64_t tt = t - lane;
                unsigned long long s = tt >= 0 ? load_state(&a.tile_state[tt]) : kPre;
                unsigned spins = 0;
                while (__ballot((s >> 62) == 0ull) != 0ull) {
                    if ((s >> 62) == 0ull) s = load_state(&a.tile_state[tt]);
                    if (++spins > (1u << 22)) {  // predecessors never published: give up loudly
                        if (lane == 0) atomicOr(&a.ctl->scan_fault, 1u);
                        s = kPre;
                    }
                }
                const unsigned long long pre = __ballot((s >> 62) == 2ull);
                const int stop = pre ? __ffsll((long long)pre) - 1 : kWave;  // nearest tile with a prefix
                int contrib = (lane <= stop && tt >= 0) ? (int)(unsigned)(s & 0xffffffffull) : 0;
                for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
                excl += contrib;
                if (pre) break;
                t -= kWave;
            }
            if (lane == 0) store_state(&a.tile_state[tile], kPre | (unsigned)(excl + total));
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    int run = s_excl + wave_off + incl - sum;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int j = (int)threadIdx.x * kScanItems + q;
        s_buf[j + j / 32] = run;
        run += v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int j = q * kScanBlock + (int)threadIdx.x;
        const int64_t gj = t0 + j;
        if (gj < a.m) a.cell_start[gj] = s_buf[j + j / 32];
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan(ScanArgs a) {
    __shared__ ScanLds L;
    scan_body(a, L);
}

struct ScatterArgs {
    const int64_t *n_dev;
    int64_t capacity;
    const Ctl *ctl;
    const uint32_t *packed;
    const unsigned long long *spill;
    int32_t rbits;
    const int32_t *cell_start;
    int32_t *cell_idx;
};

constexpr int kScatterBatch = 4;

__device__ __forceinline__ void scatter_body(const ScatterArgs &a, const int lb, const int G) {
    if (a.ctl->scan_fault) return;
    const int64_t N = live_count(a.n_dev, a.capacity);
    const int64_t per = ((N + G - 1) / G + blockDim.x - 1) / blockDim.x * blockDim.x;
    const int64_t s0 = (int64_t)lb * per;
    const int64_t s1 = min(N, s0 + per);
    const uint32_t rmask = (1u << a.rbits) - 1u;
    const int64_t B = blockDim.x;
    for (int64_t base = s0 + threadIdx.x; base < s1; base += B * kScatterBatch) {
        uint32_t v[kScatterBatch];  // every load of the batch first
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j) {
            const int64_t i = base + j * B;
            v[j] = i < s1 ? a.packed[i] : 0u;
        }
        uint32_t key[kScatterBatch], rank[kScatterBatch];
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j) {
            key[j] = v[j] >> a.rbits;
            rank[j] = v[j] & rmask;
            if (v[j] == 0xffffffffu) {
                const unsigned long long kr = a.spill[base + j * B];
                key[j] = (uint32_t)(kr >> 32);
                rank[j] = (uint32_t)(kr & 0xffffffffull);
            }
        }
        int32_t start[kScatterBatch];
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j) start[j] = base + j * B < s1 ? a.cell_start[key[j]] : 0;
#pragma unroll
        for (int j = 0; j < kScatterBatch; ++j)
            if (base + j * B < s1) a.cell_idx[start[j] + (int32_t)rank[j]] = (int32_t)(base + j * B);
    }
}

__global__ __launch_bounds__(kBuildBlock) void k_scatter(ScatterArgs a) { scatter_body(a, logical_block(), gridDim.x); }

// Occupied bricks of the sparse grid (setup: sph_grid_fit).
__global__ __launch_bounds__(kBuildBlock) void k_mark_bricks(const float *x, const float *y, const float *z,
                                                             const int64_t *n_dev, int64_t capacity, Grid g,
                                                             uint8_t *mask) {
    const int64_t N = live_count(n_dev, capacity);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t ix, iy, iz;
        cell_coords(g, x[i], y[i], g.dim == 3 ? z[i] : 0.0f, ix, iy, iz);
        const uint32_t b = (uint32_t)g.blog2;
        mask[(ix >> b) + (uint32_t)g.bdims[0] * ((iy >> b) + (uint32_t)g.bdims[1] * (iz >> b))] = 1;
    }
}

// ------------------------------------------------------------- K1 classify --

struct LocalArgs {
    Parts p;
    const BufDev *bufs;
    int nb;
    const int32_t *run_first;  // compact run list; its length is Ctl::n_runs
    const int32_t *run_len;
    const uint8_t *run_buf;
    const int32_t *cell_start;
    const int32_t *cell_idx;
    EventArgs e;
    int rpb;  // runs per workgroup and round, 1..kMaxRunsPerBlock
};

// A workgroup takes kRunsPerBlock runs of cover cells at a time: wave 0 loads
// their records and the particle ranges of their cells, the block lays the runs'
// particles out flat (a prefix over the runs in LDS), and every thread takes one
// particle per round -- its cell_idx entry, then its position, label and (where
// a duplicate may be made) carried fields, the test, the decision and the
// emission.  The buffer varies from lane to lane.
constexpr int kMaxRunsPerBlock = 8;
constexpr int kRunsPerBlock = 3;  // default

__device__ __forceinline__ void classify_body(const LocalArgs &a, const int vb, const int vg) {
    __shared__ BufDev sb[SPH_MAX_BUFFERS];
    __shared__ unsigned s_cnt[2 * SPH_MAX_BUFFERS];
    __shared__ int s_j0[kMaxRunsPerBlock], s_pre[kMaxRunsPerBlock + 1], s_k[kMaxRunsPerBlock];
    __shared__ int s_nruns, s_fault;
    for (int t = threadIdx.x; t < a.nb * (int)(sizeof(BufDev) / 4); t += blockDim.x)
        reinterpret_cast<uint32_t *>(sb)[t] = reinterpret_cast<const uint32_t *>(a.bufs)[t];
    if (threadIdx.x == 0) {  // with the records: one round trip
        s_nruns = a.e.ctl->n_runs;
        s_fault = (int)a.e.ctl->scan_fault;
    }
    block_counts_init(s_cnt);
    __syncthreads();
    if (s_fault) {
        block_counts_store(a.e, s_cnt, a.nb);
        return;
    }
    const int n_runs = s_nruns;
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const int dim = a.p.dim;
    const int seg = (vb * wpb + wave) % kSeg;
    const int R = a.rpb < 1 ? 1 : (a.rpb > kMaxRunsPerBlock ? kMaxRunsPerBlock : a.rpb);
    for (int r0 = vb * R; r0 < n_runs; r0 += vg * R) {  // block-uniform
        if (threadIdx.x < kWave) {  // wave 0: the runs' records and candidate ranges
            const int q = threadIdx.x, r = r0 + q;
            int len = 0, j0 = 0, k = 0;
            if (q < R && r < n_runs) {
                k = a.run_buf[r];
                const int c0 = a.run_first[r], c1 = c0 + a.run_len[r];
                j0 = a.cell_start[c0];
                len = a.cell_start[c1] - j0;
            }
            int incl = len;
            for (int off = 1; off < kMaxRunsPerBlock; off <<= 1) {
                const int t = __shfl_up(incl, off);
                if (q >= off) incl += t;
            }
            if (q < R) {
                s_j0[q] = j0;
                s_pre[q] = incl - len;
                s_k[q] = k;
                if (q == R - 1) s_pre[R] = incl;
            }
        }
        __syncthreads();
        const int total = s_pre[R];
        for (int base = 0; base < total; base += blockDim.x) {  // block-uniform
            const int t = base + (int)threadIdx.x;
            int q = 0;
#pragma unroll
            for (int qq = 1; qq < kMaxRunsPerBlock; ++qq)
                if (qq < R && s_pre[qq] <= t) q = qq;
            const int k = s_k[q];
            const BufDev &b = sb[k];
            int64_t i = t < total ? a.cell_idx[s_j0[q] + (t - s_pre[q])] : 0;
            const bool valid = t < total && i < N;  // a list older than the live count cannot index past it
            int lab = 0;
            float x = 0.0f, y = 0.0f, z = 0.0f;
            float carv[SPH_MAX_CARRIED];
            Outcome o{kEvNone, -1, false};
            if (valid) {
                x = a.p.pos[0][i];
                y = a.p.pos[1][i];
                z = dim == 3 ? a.p.pos[2][i] : 0.0f;
                lab = a.p.label[i];  // loaded with the position: one dependent round trip less
                // carried fields too, where a duplicate may be made: its payload is then
                // in registers when the event slot comes back
                if (b.kind != SPH_OUTLET) {
#pragma unroll
                    for (int f = 0; f < SPH_MAX_CARRIED; ++f)
                        if (f < a.p.nc) carv[f] = a.p.car[f][i];
                }
                const unsigned bits = classify(b, dim, x, y, z);
                if (bits & kIn) o = decide(b, k, dim, bits, lab, x, y, z);
            }
            unsigned long long found = 0, post = 0;
            emit<true>(a.e, a.p, b, k, seg, valid, i, lab, o, x, y, z, carv, found, post);
            if (found) atomicAdd(&s_cnt[2 * k], 1u);  // the buffer differs from lane to lane
            if (post) atomicAdd(&s_cnt[2 * k + 1], 1u);
        }
        __syncthreads();  // the run tables are reused by the next round
    }
    __syncthreads();
    block_counts_store(a.e, s_cnt, a.nb);
}

__global__ __launch_bounds__(kClassifyBlock) void k_classify_local(LocalArgs a) {
    classify_body(a, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------- K1f full scan (baseline) --
//
// Two launches.  The filter tests every particle against every buffer's check
// region in FP32, widened by the guard band so that no member can be missed, and
// appends the candidates (index, buffer) to one list (one atomic per block).
// The candidate pass then takes each through the same exact test, decision and
// emission as the local classify.

constexpr int kFullVec = 4;  // particles per thread per step of the filter (a multiple of 4)
constexpr int64_t kCandSlack = 4096;  // candidate list: capacity + this many entries
constexpr int kCandBlocks = 2048;     // grid of the candidate pass (grid-stride over the list)
constexpr int kCandBlocksMerged = 1024;  // ... beside the bucket scatter (fewer candidates: cover cells only)

struct FullArgs {
    Parts p;
    const BufDev *bufs;
    int nb;
    EventArgs e;
    unsigned long long *cand;  // (index << 4) | buffer
    int64_t cap_cand;
    int vec;                   // positions 16-byte aligned: vector loads allowed
};


__global__ __launch_bounds__(kClassifyBlock) void k_filter_full(FullArgs a) {
    __shared__ BufDev sb[SPH_MAX_BUFFERS];
    __shared__ unsigned s_wtot[kClassifyBlock / kWave];
    __shared__ unsigned long long s_base;
    for (int t = threadIdx.x; t < a.nb * (int)(sizeof(BufDev) / 4); t += blockDim.x)
        reinterpret_cast<uint32_t *>(sb)[t] = reinterpret_cast<const uint32_t *>(a.bufs)[t];
    __syncthreads();
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int dim = a.p.dim;
    const int lb = logical_block();
    constexpr int kVec = kFullVec;
    const int64_t quant = (int64_t)blockDim.x * kVec;
    const int64_t per = ((N + gridDim.x - 1) / gridDim.x + quant - 1) / quant * quant;
    const int64_t s0 = (int64_t)lb * per;
    const int64_t s1 = min(N, s0 + per);
    bool bad = false;
    for (int64_t base = s0; base < s1; base += quant) {  // block-uniform trip count
        const int64_t i0 = base + (int64_t)kVec * threadIdx.x;
        float px[kVec], py[kVec], pz[kVec];
        if (a.vec && i0 + kVec <= s1) {
#pragma unroll
            for (int h = 0; h < kVec; h += 4) {
                const float4 vx = *reinterpret_cast<const float4 *>(a.p.pos[0] + i0 + h);
                const float4 vy = *reinterpret_cast<const float4 *>(a.p.pos[1] + i0 + h);
                px[h] = vx.x; px[h + 1] = vx.y; px[h + 2] = vx.z; px[h + 3] = vx.w;
                py[h] = vy.x; py[h + 1] = vy.y; py[h + 2] = vy.z; py[h + 3] = vy.w;
                if (dim == 3) {
                    const float4 vz = *reinterpret_cast<const float4 *>(a.p.pos[2] + i0 + h);
                    pz[h] = vz.x; pz[h + 1] = vz.y; pz[h + 2] = vz.z; pz[h + 3] = vz.w;
                } else {
                    pz[h] = pz[h + 1] = pz[h + 2] = pz[h + 3] = 0.0f;
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < kVec; ++c) {
                const bool ok = i0 + c < s1;
                px[c] = ok ? a.p.pos[0][i0 + c] : 0.0f;
                py[c] = ok ? a.p.pos[1][i0 + c] : 0.0f;
                pz[c] = ok && dim == 3 ? a.p.pos[2][i0 + c] : 0.0f;
            }
        }
        // candidate bits: bit c * 16 + k for particle c of this lane and buffer k
        unsigned long long bits = 0ull;
        unsigned mine = 0;
#pragma unroll
        for (int c = 0; c < kVec; ++c)
            if (i0 + c < s1) bad |= !(isfinite(px[c]) && isfinite(py[c]) && isfinite(pz[c]));
        for (int k = 0; k < a.nb; ++k) {  // buffer outer: its box is read once for all kVec particles
            const BufDev &b = sb[k];
            const float x0 = b.bmin[0], x1 = b.bmax[0], y0 = b.bmin[1], y1 = b.bmax[1], z0 = b.bmin[2],
                        z1 = b.bmax[2];
#pragma unroll
            for (int c = 0; c < kVec; ++c) {
                const bool in_box = i0 + c < s1 && px[c] > x0 && px[c] < x1 && py[c] > y0 && py[c] < y1 &&
                                    pz[c] > z0 && pz[c] < z1;
                if (in_box && near_region(b, dim, px[c], py[c], pz[c])) {
                    bits |= 1ull << (16 * c + k);
                    ++mine;
                }
            }
        }
        unsigned incl = mine;  // lane prefix of the candidate counts
        for (int off = 1; off < kWave; off <<= 1) {
            const unsigned t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        if (lane == kWave - 1) s_wtot[wave] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned tot = 0;
            for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += s_wtot[w];
            s_base = tot ? atomicAdd(&a.e.ctl->cand_count, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        unsigned long long at = s_base + (incl - mine);
        for (int w = 0; w < wave; ++w) at += s_wtot[w];
        while (bits) {
            const int bit = __ffsll((long long)bits) - 1;
            bits &= bits - 1ull;
            if (at < (unsigned long long)a.cap_cand)
                a.cand[at] = ((unsigned long long)(i0 + bit / 16) << 4) | (unsigned long long)(bit % 16);
            else
                a.e.ctl->cand_overflow = 1u;
            ++at;
        }
        __syncthreads();  // s_wtot and s_base are reused by the next step
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&a.e.ctl->nonfinite_full, 1u);
}

// Clears the events and label counts a classifying count pass emitted for an update
// that will not finalize them (the state changed since, or a new build or a full
// scan replaces them).  clear_nf: also its non-finite flag.
__global__ void k_reset_events(Ctl *ctl, unsigned *part, int clear_nf) {
    if (threadIdx.x < kSeg) {
        ctl->seg[threadIdx.x].n_gen = 0u;
        ctl->seg[threadIdx.x].n_del = 0u;
        ctl->seg[threadIdx.x].n_rel = 0u;
    }
    if (threadIdx.x == 0) {
        if (clear_nf) ctl->nonfinite_full = 0u;
        ctl->cand_count = 0ull;  // the merged step's candidates
        ctl->cand_overflow = 0u;
    }
    for (int w = threadIdx.x; w < kCountReplicas * 2 * SPH_MAX_BUFFERS; w += blockDim.x) part[w] = 0u;
}

__device__ __forceinline__ void classify_cand_body(const FullArgs &a, const int lb, const int G) {
    __shared__ BufDev sb[SPH_MAX_BUFFERS];
    __shared__ unsigned s_cnt[2 * SPH_MAX_BUFFERS];
    for (int t = threadIdx.x; t < a.nb * (int)(sizeof(BufDev) / 4); t += blockDim.x)
        reinterpret_cast<uint32_t *>(sb)[t] = reinterpret_cast<const uint32_t *>(a.bufs)[t];
    block_counts_init(s_cnt);
    __syncthreads();
    const unsigned long long cc = a.e.ctl->cand_count;
    const int64_t n_cand = cc < (unsigned long long)a.cap_cand ? (int64_t)cc : a.cap_cand;
    const int dim = a.p.dim;
    const int seg = (int)((lb * (blockDim.x / kWave) + threadIdx.x / kWave) % kSeg);
    for (int64_t t0 = (int64_t)lb * blockDim.x; t0 < n_cand; t0 += (int64_t)G * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        const bool valid = t < n_cand;
        const unsigned long long ent = valid ? a.cand[t] : 0ull;
        const int64_t i = (int64_t)(ent >> 4);
        const int k = valid ? (int)(ent & 15ull) : 0;
        const BufDev &b = sb[k];
        int lab = 0;
        float x = 0.0f, y = 0.0f, z = 0.0f;
        float carv[SPH_MAX_CARRIED];
        Outcome o{kEvNone, -1, false};
        if (valid) {
            x = a.p.pos[0][i];
            y = a.p.pos[1][i];
            z = dim == 3 ? a.p.pos[2][i] : 0.0f;
            lab = a.p.label[i];
            if (b.kind != SPH_OUTLET) {
#pragma unroll
                for (int f = 0; f < SPH_MAX_CARRIED; ++f)
                    if (f < a.p.nc) carv[f] = a.p.car[f][i];
            }
            const unsigned bits = classify(b, dim, x, y, z);
            if (bits & kIn) o = decide(b, k, dim, bits, lab, x, y, z);
        }
        unsigned long long found = 0, post = 0;
        emit<true>(a.e, a.p, b, k, seg, valid, i, lab, o, x, y, z, carv, found, post);
        if (found) atomicAdd(&s_cnt[2 * k], 1u);  // the buffer differs from lane to lane
        if (post) atomicAdd(&s_cnt[2 * k + 1], 1u);
    }
    __syncthreads();
    block_counts_store(a.e, s_cnt, a.nb);
}

__global__ __launch_bounds__(kClassifyBlock) void k_classify_cand(FullArgs a) {
    classify_cand_body(a, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------- bucketed cell list --
//
// The cell list of a context is built by a two-level counting sort whose memory
// traffic does not depend on the order of the particle arrays (particles drift out
// of any spatial order as the flow shears them; with one global atomic per cell
// run, the counting-sort build above then pays for line-sized atomics spread over
// the whole counter array and shared by all XCDs):
//   k_bk_count : workgroups of kBkPer particles in array order (coalesced loads):
//                cell keys, an LDS histogram over buckets of 2^bshift consecutive
//                cells, one global atomic per (workgroup, bucket) for the
//                workgroup's base in the bucket, then each particle's (key, rank
//                in its bucket); the workgroup with the last ticket turns the
//                bucket counts into bucket starts.  On the merged path the
//                particles of the buffers' cover cells that lie near a check
//                region are also appended to the candidate list.
//   k_bk_scatter : (key, particle) into bucket order; a workgroup's run of a
//                bucket lands contiguously.
//   k_bk_sort  : one workgroup per bucket: an LDS counting sort of its entries
//                over its cells, writing the bucket's cell starts and its
//                contiguous range of cell_idx.
// The order inside a cell is whatever the LDS atomics make it.

constexpr int kBkBlock = 256;
constexpr int kBkPer = 4096;          // particles per k_bk_count workgroup
constexpr int kBkIt = kBkPer / kBkBlock;
constexpr int kBkBatch = 4;           // particles per thread with loads in flight together
constexpr int kMaxBuckets = 4096;
constexpr int kMaxBucketCells = 4096;
static_assert(kBkIt % kBkBatch == 0, "whole batches");

struct BkArgs {
    const float *x, *y, *z;
    const int64_t *n_dev;
    int64_t capacity;
    Grid g;
    int32_t bshift;           // cells per bucket: 1 << bshift
    int32_t nbk;              // buckets
    int64_t n_cells;          // C: cell_start holds C + 1 entries
    uint32_t *bk_count;       // [nbk] zero between builds
    uint32_t *bk_start;       // [nbk + 1]
    uint2 *ent;               // [capacity] (key, rank in its bucket) per particle
    uint2 *tmp;               // [capacity] (key, particle) in bucket order
    int32_t *cell_start;
    int32_t *cell_idx;
    Ctl *ctl;
    unsigned int *nonfinite;  // flag to raise on a non-finite position
    // merged step: candidate list of the cover cells
    const uint16_t *cover;
    const BufDev *bufs;
    int nb;
    unsigned long long *cand;  // (index << 4) | buffer
    int64_t cap_cand;
};

// Runs of equal values in consecutive lanes: the head lane of this lane's run and
// the run's length (an invalid lane is a run of its own, of length 0).
__device__ __forceinline__ void lane_runs(uint32_t v, bool valid, int lane, int &head, int &len) {
    const uint32_t prev = __shfl_up(v, 1);
    const bool h = !valid || lane == 0 || v != prev;
    const unsigned long long heads = __ballot(h);
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    head = 63 - __clzll((long long)(heads & le));
    const unsigned long long gt = heads & ~le;
    len = valid ? (gt ? __ffsll((long long)gt) - 1 : 64) - head : 0;
}

// Exclusive prefix over v[0..n) in LDS, in place, by one workgroup of NT threads
// (each takes kMaxBuckets / NT consecutive entries); returns the total.
template <int NT>
__device__ __forceinline__ uint32_t lds_exclusive_scan(uint32_t *v, int n, uint32_t *s_w) {
    constexpr int kPer = kMaxBuckets / NT;
    static_assert(kMaxBuckets == kMaxBucketCells, "one scan for both");
    const int t0 = (int)threadIdx.x * kPer;
    uint32_t loc[kPer];
    uint32_t sum = 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        loc[q] = t0 + q < n ? v[t0 + q] : 0u;
        sum += loc[q];
    }
    const int lane = (int)threadIdx.x & (kWave - 1), wave = (int)threadIdx.x / kWave;
    uint32_t incl = sum;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t base = 0u, total = 0u;
    for (int w = 0; w < NT / kWave; ++w) {
        if (w < wave) base += s_w[w];
        total += s_w[w];
    }
    uint32_t run = base + incl - sum;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (t0 + q < n) v[t0 + q] = run;
        run += loc[q];
    }
    __syncthreads();
    return total;
}

template <bool kCand>
__global__ __launch_bounds__(kBkBlock) void k_bk_count(BkArgs a) {
    static_assert(kBkPer <= 4096, "candidate offsets are 12 bits");
    __shared__ uint32_t s_h[kMaxBuckets];  // counts, then bases, then cursors per bucket
    __shared__ BufNear sb[kCand ? SPH_MAX_BUFFERS : 1];
    // (1024 slots: every workgroup of 4096 particles but those crowded with candidates)
    __shared__ std::conditional_t<kCand, CandLds<uint16_t, 1024>, char> s_cand;
    __shared__ uint32_t s_w[kBkBlock / kWave];
    __shared__ unsigned s_last;
    const int64_t N = live_count(a.n_dev, a.capacity);
    const int lb = logical_block(), G = (int)gridDim.x;
    const int lane = (int)threadIdx.x & (kWave - 1);
    if (lb == 0 && threadIdx.x == 0) {
        a.ctl->n_built = N;
        a.ctl->scan_fault = 0u;  // (raised only by the look-back scan of the three-kernel build)
    }
    for (int t = threadIdx.x; t < a.nbk; t += kBkBlock) s_h[t] = 0u;
    if constexpr (kCand) {
        near_load(sb, a.bufs, a.nb);
        if (threadIdx.x == 0) s_cand.n = 0u;
    }
    __syncthreads();
    const CandArgs ca{a.cover, a.bufs, a.nb, a.cand, a.cap_cand};
    const int64_t s0 = (int64_t)lb * kBkPer;
    const bool d3 = a.g.dim == 3;
    const float *zb = d3 ? a.z : a.x;  // a 2-D z is a copy of x, unused
    bool bad = false;
    const int dim = a.g.dim;
    // keys of this thread's particles s0 + it * kBkBlock + threadIdx.x (kept for the ranks)
    uint32_t key[kBkIt];
    const bool live = s0 < N;  // block-uniform
    if (live) {
        // ---- counts per bucket (and the merged step's candidates) ----
#pragma unroll
        for (int it = 0; it < kBkIt; it += kBkBatch) {
            float px[kBkBatch], py[kBkBatch], pz[kBkBatch];
            bool ok[kBkBatch];
#pragma unroll
            for (int q = 0; q < kBkBatch; ++q) {  // every load of the batch first (no branch)
                const int64_t i = s0 + (int64_t)(it + q) * kBkBlock + threadIdx.x;
                ok[q] = i < N;
                const int64_t ic = ok[q] ? i : 0;
                px[q] = a.x[ic];
                py[q] = a.y[ic];
                pz[q] = zb[ic];
            }
            {
                uint32_t kq[kBkBatch];
                keys_of<kBkBatch>(a.g, px, py, pz, ok, 0u, kq, bad);
#pragma unroll
                for (int q = 0; q < kBkBatch; ++q) key[it + q] = kq[q];
            }
            uint32_t cm[kBkBatch];
            if constexpr (kCand) {  // the cover bits of the batch, all loads issued together
#pragma unroll
                for (int q = 0; q < kBkBatch; ++q) cm[q] = ok[q] ? a.cover[key[it + q]] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kBkBatch; ++q) {
                int head, len;
                lane_runs(key[it + q] >> a.bshift, ok[q], lane, head, len);
                if (len > 0 && lane == head) atomicAdd(&s_h[key[it + q] >> a.bshift], (uint32_t)len);
            }
            if constexpr (kCand) {
                // each cover bit kept only if the particle is near that check region
                // (the full scan's FP32 test widened by the guard band, which keeps
                // every member)
                uint32_t loc[kBkBatch];
                int64_t idx[kBkBatch];
                float zq[kBkBatch];
#pragma unroll
                for (int q = 0; q < kBkBatch; ++q) {
                    loc[q] = (uint32_t)((it + q) * kBkBlock) + threadIdx.x;
                    idx[q] = s0 + (int64_t)loc[q];
                    zq[q] = d3 ? pz[q] : 0.0f;
                }
                cand_append<kBkBatch>(ca, sb, dim, cm, px, py, zq, loc, idx, lane, s_cand, a.ctl);
            }
        }
    }
    __syncthreads();
    if constexpr (kCand) cand_flush(ca, s_cand, s0, a.ctl);  // the workgroup's candidates into the list
    // ---- the workgroup's base in each bucket it meets: one global atomic each ----
    // A thread issues all its atomics before it uses the first result (a loop that
    // stores each result before the next atomic waits a device atomic's full round
    // trip per bucket).
    constexpr int kPerT = kMaxBuckets / kBkBlock;
    {
        uint32_t r[kPerT];
#pragma unroll
        for (int q = 0; q < kPerT; ++q) {
            const int t = q * kBkBlock + (int)threadIdx.x;
            const uint32_t c = t < a.nbk ? s_h[t] : 0u;
            r[q] = c ? atomicAdd(&a.bk_count[t], c) : 0u;
        }
#pragma unroll
        for (int q = 0; q < kPerT; ++q) {
            const int t = q * kBkBlock + (int)threadIdx.x;
            if (t < a.nbk) s_h[t] = r[q];
        }
    }
    __syncthreads();
    if (live) {
        // ---- each particle's rank in its bucket ----
#pragma unroll
        for (int it = 0; it < kBkIt; ++it) {
            const int64_t i = s0 + (int64_t)it * kBkBlock + threadIdx.x;
            const bool ok = i < N;
            int head, len;
            lane_runs(key[it] >> a.bshift, ok, lane, head, len);
            uint32_t old = 0u;
            if (len > 0 && lane == head) old = atomicAdd(&s_h[key[it] >> a.bshift], (uint32_t)len);
            const uint32_t rank = __shfl(old, head) + (uint32_t)(lane - head);
            if (ok) a.ent[i] = make_uint2(key[it], rank);
        }
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(a.nonfinite, 1u);
    // ---- the last workgroup: bucket starts from the counts (then cleared) ----
    // Every bucket atomic of a workgroup has returned (its base was stored in LDS)
    // before the barrier that precedes its ticket, so the workgroup that draws the
    // last ticket finds all of them done; it takes the counts by atomic exchanges.
    // (No fence: a device-scope release would write back the whole L2.)
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(&a.ctl->bk_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 (unsigned)G - 1u;
    __syncthreads();
    if (!s_last) return;
    {  // read and cleared where the atomics were done, all of a thread's in flight together
        uint32_t r[kPerT];
#pragma unroll
        for (int q = 0; q < kPerT; ++q) {
            const int t = q * kBkBlock + (int)threadIdx.x;
            r[q] = t < a.nbk ? atomicExch(&a.bk_count[t], 0u) : 0u;
        }
#pragma unroll
        for (int q = 0; q < kPerT; ++q) {
            const int t = q * kBkBlock + (int)threadIdx.x;
            if (t < a.nbk) s_h[t] = r[q];
        }
    }
    __syncthreads();
    const uint32_t total = lds_exclusive_scan<kBkBlock>(s_h, a.nbk, s_w);
    for (int t = threadIdx.x; t < a.nbk; t += kBkBlock) a.bk_start[t] = s_h[t];
    if (threadIdx.x == 0) {
        a.bk_start[a.nbk] = total;
        a.ctl->bk_ticket = 0u;
    }
}

// (key, particle) of every particle the count pass saw into bucket order.
__device__ __forceinline__ void bk_scatter_body(const BkArgs &a, const int lb, const int G) {
    if (lb == 0 && threadIdx.x == 0) {  // the count pass is complete: keep its verdict for the update
        a.ctl->nonfinite_seen = a.ctl->nonfinite_build;
        a.ctl->nonfinite_build = 0u;
    }
    const int64_t nb_ = a.ctl->n_built;
    const int64_t N = nb_ < 0 ? 0 : (nb_ > a.capacity ? a.capacity : nb_);
    constexpr int kB = 4;
    const int64_t quant = (int64_t)kBkBlock * kB;
    const int64_t per = ((N + G - 1) / G + quant - 1) / quant * quant;
    const int64_t s0 = (int64_t)lb * per, s1 = min(N, s0 + per);
    for (int64_t base = s0 + threadIdx.x; base < s1; base += quant) {
        uint2 e[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const int64_t i = base + (int64_t)q * kBkBlock;
            e[q] = i < s1 ? a.ent[i] : make_uint2(0u, 0u);
        }
        uint32_t st[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) st[q] = base + (int64_t)q * kBkBlock < s1 ? a.bk_start[e[q].x >> a.bshift] : 0u;
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const int64_t i = base + (int64_t)q * kBkBlock;
            if (i < s1) a.tmp[st[q] + e[q].y] = make_uint2(e[q].x, (uint32_t)i);
        }
    }
}

__global__ __launch_bounds__(kBkBlock) void k_bk_scatter(BkArgs a) { bk_scatter_body(a, logical_block(), gridDim.x); }

// Block b of the g blocks that follow the first ncls of a launch, renumbered so
// that each XCD takes a contiguous range, as logical_block does for a whole launch
// (the counting scatter's blocks then meet the particle ranges the count pass's
// blocks of the same XCD wrote: 65 -> 56 us on the network's late states; the bucket
// scatter got slower with it, 46 -> 53 us, and keeps the plain order).
__device__ __forceinline__ int xcd_block(int b, int g, int ncls) {
    if ((g & 7) || (ncls & 7)) return b;
    return (b & 7) * (g >> 3) + (b >> 3);
}

// The merged step's update, first launch: the candidates' classification (the
// first ncls workgroups) beside the bucket scatter (the others).
__global__ __launch_bounds__(kBkBlock) void k_bk_scatter_cls(BkArgs a, FullArgs f, int ncls) {
    static_assert(kBkBlock == kClassifyBlock, "one launch");
    if ((int)blockIdx.x < ncls)
        classify_cand_body(f, (int)blockIdx.x, ncls);
    else
        bk_scatter_body(a, (int)blockIdx.x - ncls, (int)gridDim.x - ncls);
}

// The same for the counting build: classification beside its scatter.
__global__ __launch_bounds__(kBuildBlock) void k_scatter_cls(ScatterArgs a, FullArgs f, int ncls) {
    static_assert(kBuildBlock == kClassifyBlock, "one launch");
    if ((int)blockIdx.x < ncls)
        classify_cand_body(f, (int)blockIdx.x, ncls);
    else
        scatter_body(a, xcd_block((int)blockIdx.x - ncls, (int)gridDim.x - ncls, ncls), (int)gridDim.x - ncls);
}

constexpr int kSortBlock = 512;

__global__ __launch_bounds__(kSortBlock) void k_bk_sort(BkArgs a) {
    __shared__ uint32_t s_c[kMaxBucketCells];
    __shared__ uint32_t s_w[kSortBlock / kWave];
    const int b = (int)blockIdx.x;
    if (b >= a.nbk) return;
    const uint32_t n0 = a.bk_start[b], n1 = a.bk_start[b + 1];
    const int64_t c0 = (int64_t)b << a.bshift;
    const int nc = (int)min<int64_t>((int64_t)1 << a.bshift, a.n_cells - c0);
    // The bucket's first kHeld entries are read once and kept in registers (kR per
    // thread, all loads in flight together) for both passes; only the entries of a
    // bucket past that are read again (streamed, the next round's loads issued before
    // the current round is counted or placed).  One LDS atomic per entry: in bucket
    // order the lanes of a wave rarely share a cell.  A bucket of at most kHeld
    // entries is placed in LDS and stored in order (scattered 4-byte stores into
    // the bucket's range cost more than the LDS round).
    constexpr int kR = 8;
    constexpr uint32_t kHeld = (uint32_t)kSortBlock * kR;
    __shared__ int32_t s_out[kHeld];
    uint2 h[kR];
#pragma unroll
    for (int q = 0; q < kR; ++q) {
        const uint32_t e = n0 + (uint32_t)q * kSortBlock + threadIdx.x;
        h[q] = e < n1 ? a.tmp[e] : make_uint2((uint32_t)c0, 0u);
    }
    for (int t = threadIdx.x; t < nc; t += kSortBlock) s_c[t] = 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kR; ++q)
        if (n0 + (uint32_t)q * kSortBlock + threadIdx.x < n1) atomicAdd(&s_c[h[q].x - (uint32_t)c0], 1u);
    constexpr int kB = 4;  // entries per thread and round of the streamed rest
    constexpr uint32_t kStep = (uint32_t)kSortBlock * kB;
    const uint32_t r0 = n0 + kHeld;  // first streamed entry
    auto load = [&](uint32_t e0, uint2 (&u)[kB]) {
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const uint32_t e = e0 + (uint32_t)q * kSortBlock + threadIdx.x;
            u[q] = e < n1 ? a.tmp[e] : make_uint2((uint32_t)c0, 0u);
        }
    };
    uint2 u[kB], un[kB];
    if (r0 < n1) load(r0, u);
    for (uint32_t e0 = r0; e0 < n1; e0 += kStep) {  // block-uniform trip count
        if (e0 + kStep < n1) load(e0 + kStep, un);
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (e0 + (uint32_t)q * kSortBlock + threadIdx.x < n1) atomicAdd(&s_c[u[q].x - (uint32_t)c0], 1u);
#pragma unroll
        for (int q = 0; q < kB; ++q) u[q] = un[q];
    }
    __syncthreads();
    lds_exclusive_scan<kSortBlock>(s_c, nc, s_w);
    for (int t = threadIdx.x; t < nc; t += kSortBlock) a.cell_start[c0 + t] = (int32_t)(n0 + s_c[t]);
    if (b == a.nbk - 1 && threadIdx.x == 0) a.cell_start[a.n_cells] = (int32_t)n1;
    __syncthreads();  // every offset read before the cursors move
    if (n1 - n0 <= kHeld) {  // block-uniform: every entry is held
#pragma unroll
        for (int q = 0; q < kR; ++q)
            if (n0 + (uint32_t)q * kSortBlock + threadIdx.x < n1)
                s_out[atomicAdd(&s_c[h[q].x - (uint32_t)c0], 1u)] = (int32_t)h[q].y;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < n1 - n0; t += kSortBlock) a.cell_idx[n0 + t] = s_out[t];
        return;
    }
#pragma unroll
    for (int q = 0; q < kR; ++q)
        if (n0 + (uint32_t)q * kSortBlock + threadIdx.x < n1)
            a.cell_idx[n0 + atomicAdd(&s_c[h[q].x - (uint32_t)c0], 1u)] = (int32_t)h[q].y;
    if (r0 < n1) load(r0, u);
    for (uint32_t e0 = r0; e0 < n1; e0 += kStep) {
        if (e0 + kStep < n1) load(e0 + kStep, un);
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (e0 + (uint32_t)q * kSortBlock + threadIdx.x < n1)
                a.cell_idx[n0 + atomicAdd(&s_c[u[q].x - (uint32_t)c0], 1u)] = (int32_t)u[q].y;
#pragma unroll
        for (int q = 0; q < kB; ++q) u[q] = un[q];
    }
}


// ------------------------------------------------------------- K2 finalize --
//
// nfb workgroups per domain, each through the same four phases; every block
// takes the status decision itself (all checks come before any write) and sorts
// both event lists in LDS, and no block writes a location that another block
// reads:
//   A. one round of loads: the counters, the label counts and the first kSpec
//      slots of every event segment (the entries of a segment past kSpec, rare,
//      take a second round once the counters are known);
//   B. the entries into flat lists; recycle and relabel of particles below the
//      new count N' = N - |D| are issued in place by the entry's owner block
//      (those particles neither move nor are deleted); an LDS map of the tail
//      [N', N) holds each tail particle's recycle entry and new label;
//   C. both lists sorted: 256-key chunks in registers (one wave each), then the
//      rank of every key is its place in its chunk plus the keys below it in the
//      list's other chunks (binary searches in LDS);
//   D. the positions p of the tail [N', N' + max(|G|, |D|)) are split among the
//      blocks: the thread of p loads the survivor at p (with its map entry) and
//      the payload of the duplicate appended at p, then moves the survivor into
//      its hole (the k-th surviving tail particle fills the k-th smallest
//      deleted index) and writes the duplicate at p.
// The block that takes the last ticket (every block has read the counters by
// then) writes the result and clears the counters for the next update.

constexpr int kFinBlocksMax = 32;
constexpr int kSpec = 128;  // slots per event segment loaded with the counters
static_assert(kSeg * kSpec == 2 * 1024, "two speculative entries per finalize thread");

struct FinArgs {
    Parts p;
    int nb;
    int local;
    int nf_full;  // the non-finite flag is the one a full scan or a classifying count pass raises
    EventArgs e;
    uint32_t *gen_sorted;  // [cap_ev] sources in ascending order (for sph_last_events)
    uint32_t *del_sorted;  // [cap_ev] deleted indices in ascending order
    sph_result *result;
};

// Value held by lane (lane ^ J).  J = 1, 2: one DPP quad permutation; J = 4, 8:
// two DPP moves (mirror within 8 or 16 lanes, then xor 3 or xor 7); J = 16:
// ds_swizzle in xor mode (within 32 lanes); J = 32: ds_bpermute.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x) {
    const int v = (int)x;
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
    } else if constexpr (J == 4) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true), 0x1B, 0xF, 0xF,
                                                  true);
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true), 0x141, 0xF,
                                                  0xF, true);
    } else if constexpr (J == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x401F);
    } else {
        static_assert(J == 32, "lane distance");
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, v);
    }
}

// Bitonic sort of 256 keys with payloads held by one wave, four per lane
// (element r * 64 + lane in register r).  Partners at distance >= 64 sit in
// another register of the same lane; closer ones in another lane.
constexpr int kChunk = 4 * kWave;

template <int K, int J>
__device__ __forceinline__ void bitonic_step(uint32_t (&k)[4], uint32_t (&v)[4], int lane) {
    if constexpr (J >= kWave) {
        constexpr int RJ = J / kWave;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r & RJ) continue;
            const int rp = r | RJ;
            const bool asc = ((r * kWave) & K) == 0;
            const bool sw = asc ? k[rp] < k[r] : k[rp] > k[r];
            const uint32_t k0 = k[r], v0 = v[r];
            k[r] = sw ? k[rp] : k0;
            v[r] = sw ? v[rp] : v0;
            k[rp] = sw ? k0 : k[rp];
            v[rp] = sw ? v0 : v[rp];
        }
    } else {
        const bool lower = (lane & J) == 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool asc = ((r * kWave + lane) & K) == 0;
            const uint32_t kp = xor_lane<J>(k[r]), vp = xor_lane<J>(v[r]);
            const bool take = lower == asc ? kp < k[r] : kp > k[r];
            k[r] = take ? kp : k[r];
            v[r] = take ? vp : v[r];
        }
    }
}

template <int K, int J>
__device__ __forceinline__ void bitonic_merge(uint32_t (&k)[4], uint32_t (&v)[4], int lane) {
    bitonic_step<K, J>(k, v, lane);
    if constexpr (J > 1) bitonic_merge<K, J / 2>(k, v, lane);
}

template <int K>
__device__ __forceinline__ void bitonic_sort256(uint32_t (&k)[4], uint32_t (&v)[4], int lane) {
    bitonic_merge<K, K / 2>(k, v, lane);
    if constexpr (K < kChunk) bitonic_sort256<K * 2>(k, v, lane);
}

// Keys of a sorted 256-key chunk below x (keys are distinct; padding is all ones).
__device__ __forceinline__ unsigned below_in_chunk(const uint32_t *c, uint32_t x) {
    unsigned lo = 0;
#pragma unroll
    for (unsigned step = kChunk / 2; step > 0; step >>= 1)
        if (c[lo + step - 1] < x) lo += step;
    return lo + (c[lo] < x ? 1u : 0u);
}

// Even split of [0, n) among nparts: part q gets [lo, hi).
__device__ __forceinline__ void share_of(unsigned n, int q, int nparts, unsigned &lo, unsigned &hi) {
    const unsigned chunk = (n + (unsigned)nparts - 1u) / (unsigned)nparts;
    lo = min(n, (unsigned)q * chunk);
    hi = min(n, lo + chunk);
}

constexpr uint32_t kMapRelShift = 20;  // tail map: bits 0..19 recycle slot + 1, bits 20.. new label + 1
static_assert(kSeg * kMaxEv < (1u << kMapRelShift), "recycle slot fits the tail map");

// LDS of one finalize workgroup.
struct FinLds {
    uint32_t k[2][2][kMaxEv];          // [list: 0 sources, 1 deleted][0: flat, 1: sorted] keys
    uint32_t v[2][kMaxEv];             // event slot of each source, [0: flat, 1: sorted]
    uint32_t map[kMaxEv];              // tail position t = p - N': recycle slot and new label
    unsigned bits[kMaxEv / 32], wpre[kMaxEv / 32];  // deleted tail positions, prefix per word
    unsigned cnt[3][kSeg];             // per list (gen, del, rel): segment counts
    unsigned off[3][kSeg + 1];         // exclusive offsets; [kSeg] = total
    unsigned ovf[3][kSeg + 1];         // exclusive offsets of the entries past kSpec; [kSeg] = total
    int status;
    unsigned last;
    long long N, next;
    unsigned found[SPH_MAX_BUFFERS], post[SPH_MAX_BUFFERS];
    long long nl[SPH_MAX_BUFFERS];
    unsigned flags[3];
};

__device__ __forceinline__ void finalize_body(const FinArgs &a, const int fb, const int nfb, FinLds &L) {
    Ctl *c = a.e.ctl;
    const int tid = threadIdx.x;
    const unsigned bd = blockDim.x;
    const unsigned cap = a.e.cap_ev, cap_rel = a.e.cap_rel;
    const int words = kCountReplicas * 2 * SPH_MAX_BUFFERS;
    // ---- A: counters, label counts and the first kSpec slots of every segment,
    //      all in one round of loads ----
    unsigned sc[3] = {0u, 0u, 0u};
    long long nlk = 0, nx = 0, nN = 0;
    unsigned fl[3] = {0u, 0u, 0u};
    if (tid < kSeg) {
        sc[0] = c->seg[tid].n_gen;
        sc[1] = c->seg[tid].n_del;
        sc[2] = c->seg[tid].n_rel;
    } else if (tid >= kWave && tid < kWave + SPH_MAX_BUFFERS) {
        nlk = c->n_labelled[tid - kWave];
    } else if (tid == 2 * kWave) {
        nx = c->next_id;
        nN = *a.p.n_dev;
        fl[0] = c->scan_fault;
        fl[1] = a.nf_full ? c->nonfinite_full : c->nonfinite_seen;
        fl[2] = c->cand_overflow;
    }
    unsigned pv[(kCountReplicas * 2 * SPH_MAX_BUFFERS + 1023) / 1024];
#pragma unroll
    for (int q = 0; q < (int)(sizeof(pv) / sizeof(pv[0])); ++q) {
        const int w = q * (int)bd + tid;
        pv[q] = w < words ? a.e.part[w] : 0u;
    }
    uint32_t gi[2], di[2];
    unsigned long long rv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {  // speculative entry q * 1024 + tid: segment e / kSpec, slot e % kSpec
        const unsigned e = (unsigned)q * 1024u + (unsigned)tid, g = e / kSpec, sl = e % kSpec;
        gi[q] = sl < cap ? a.e.gen_idx[(size_t)g * cap + sl] : 0u;
        di[q] = sl < cap ? a.e.del_idx[(size_t)g * cap + sl] : 0u;
        rv[q] = sl < cap_rel ? a.e.rel[(size_t)g * cap_rel + sl] : 0ull;
    }
    if (tid < SPH_MAX_BUFFERS) {
        L.found[tid] = 0u;
        L.post[tid] = 0u;
    }
    __syncthreads();
    if (tid < kSeg) {
        L.cnt[0][tid] = sc[0];
        L.cnt[1][tid] = sc[1];
        L.cnt[2][tid] = sc[2];
    } else if (tid >= kWave && tid < kWave + SPH_MAX_BUFFERS) {
        L.nl[tid - kWave] = nlk;
    } else if (tid == 2 * kWave) {
        L.next = nx;
        L.N = nN;
        L.flags[0] = fl[0];
        L.flags[1] = fl[1];
        L.flags[2] = fl[2];
    }
    for (unsigned w = tid; w < kMaxEv / 32; w += bd) L.bits[w] = 0u;
    for (unsigned t = tid; t < kMaxEv; t += bd) L.map[t] = 0u;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(pv) / sizeof(pv[0])); ++q) {
        const int w = q * (int)bd + tid;
        const int slot = w % (2 * SPH_MAX_BUFFERS);
        if (pv[q]) atomicAdd(slot & 1 ? &L.post[slot >> 1] : &L.found[slot >> 1], pv[q]);
    }
    __syncthreads();
    // Every counter this block reads has been read: its ticket can be taken now
    // (the result is needed only at the end).
    unsigned ticket = 0u;
    if (tid == 0) ticket = __hip_atomic_fetch_add(&c->fin_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid < kWave) {  // segment offsets (lane l * kSeg + g: segment g of list l), overflow offsets, status
        const int l = tid / kSeg, g = tid % kSeg;
        const unsigned v = tid < 3 * kSeg ? L.cnt[l][g] : 0u;
        const unsigned o = v > (unsigned)kSpec ? v - (unsigned)kSpec : 0u;
        unsigned incl = v, oincl = o;
        for (int off = 1; off < kSeg; off <<= 1) {
            const unsigned t = __shfl_up(incl, off, kSeg), to = __shfl_up(oincl, off, kSeg);
            if (g >= off) {
                incl += t;
                oincl += to;
            }
        }
        if (tid < 3 * kSeg) {
            L.off[l][g] = incl - v;
            L.ovf[l][g] = oincl - o;
            if (g == kSeg - 1) {
                L.off[l][kSeg] = incl;
                L.ovf[l][kSeg] = oincl;
            }
        }
        const unsigned tot0 = __shfl(incl, kSeg - 1), tot1 = __shfl(incl, 2 * kSeg - 1),
                       tot2 = __shfl(incl, 3 * kSeg - 1);
        if (tid == 0) {
            const long long N_raw = L.N;
            const long long N = N_raw < 0 ? 0 : (N_raw > a.p.capacity ? a.p.capacity : N_raw);
            int st = SPH_OK;
            if (N_raw != N) st = SPH_ERR_ARG;
            else if (a.local && L.flags[0]) st = SPH_ERR_HIP;
            else if (L.flags[1]) st = SPH_ERR_NONFINITE;
            for (int k = 0; k < a.nb && st == SPH_OK; ++k)
                if ((long long)L.found[k] < L.nl[k]) st = SPH_ERR_CFL;
            if (st == SPH_OK && (tot0 > cap || tot1 > cap || tot2 > cap_rel)) st = SPH_ERR_EVENTS;
            if (st == SPH_OK && !a.local && L.flags[2]) st = SPH_ERR_EVENTS;  // the full scan's candidate list overflowed
            if (st == SPH_OK && N - (long long)tot1 + (long long)tot0 > a.p.capacity) st = SPH_ERR_CAPACITY;
            L.status = st;
            L.N = N;
        }
    }
    __syncthreads();
    const int st = L.status;
    const unsigned G = L.off[0][kSeg], D = L.off[1][kSeg];
    const long long N = L.N;
    if (st == SPH_OK) {
        const Parts &p = a.p;
        const long long Np = N - (long long)D;
        const int dim = p.dim, nc = p.nc, ds = 3 + nc;
        // ---- B: entries into the flat lists, the tail map and the deleted bits;
        //      in-place recycle and relabel below N' by the entry's owner block ----
        // (an entry is owned by block (its speculative or overflow number) % nfb)
        unsigned own_slot[2] = {0u, 0u}, own_i[2] = {0u, 0u};
        bool own_rec[2] = {false, false};
        auto place = [&](int l, unsigned g, unsigned sl, uint32_t idx, unsigned long long r, bool mine, int q) {
            const unsigned e = L.off[l][g] + sl;
            if (l == 0) {
                L.k[0][0][e] = idx;
                L.v[0][e] = g * cap + sl;
                if ((long long)idx >= Np) atomicOr(&L.map[idx - Np], g * cap + sl + 1u);
                else if (mine) {  // recycle in place (its recycled position is loaded in D)
                    own_rec[q] = true;
                    own_slot[q] = g * cap + sl;
                    own_i[q] = idx;
                }
            } else if (l == 1) {
                L.k[1][0][e] = idx;
                if ((long long)idx >= Np) atomicOr(&L.bits[(idx - Np) >> 5], 1u << ((idx - Np) & 31));
            } else {
                const long long i = (long long)(r >> 32);
                const uint32_t lab = (uint32_t)(r & 0xffffffffull);
                if (i >= Np) atomicOr(&L.map[i - Np], (lab + 1u) << kMapRelShift);
                else if (mine) p.label[i] = (int32_t)lab;
            }
        };
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned e = (unsigned)q * 1024u + (unsigned)tid, g = e / kSpec, sl = e % kSpec;
            const bool mine = (int)(e % (unsigned)nfb) == fb;
            if (sl < L.cnt[0][g]) place(0, g, sl, gi[q], 0ull, mine, q);
            if (sl < L.cnt[1][g]) place(1, g, sl, di[q], 0ull, mine, q);
            if (sl < L.cnt[2][g]) place(2, g, sl, 0u, rv[q], mine, q);
        }
        // entries past the first kSpec slots of their segment (block-uniform test)
        if (L.ovf[0][kSeg] + L.ovf[1][kSeg] + L.ovf[2][kSeg] > 0u) {
            for (int l = 0; l < 3; ++l) {
                const unsigned tot = L.ovf[l][kSeg];
                for (unsigned f = tid; f < tot; f += bd) {
                    int g = 0;
                    while (g + 1 < kSeg && L.ovf[l][g + 1] <= f) ++g;
                    const unsigned sl = (unsigned)kSpec + (f - L.ovf[l][g]);
                    const bool mine = (int)(f % (unsigned)nfb) == fb;
                    if (l == 0) {
                        const uint32_t idx = a.e.gen_idx[(size_t)g * cap + sl];
                        const unsigned e = L.off[0][g] + sl;
                        L.k[0][0][e] = idx;
                        L.v[0][e] = g * cap + sl;
                        if ((long long)idx >= Np) atomicOr(&L.map[idx - Np], g * cap + sl + 1u);
                        else if (mine) {  // recycled in place below, right away (rare path)
                            for (int q2 = 0; q2 < dim; ++q2)
                                p.pos[q2][idx] = a.e.gen_new[4 * ((size_t)g * cap + sl) + q2];
                            if (a.e.rho_field >= 0)
                                p.car[a.e.rho_field][idx] = a.e.gen_new[4 * ((size_t)g * cap + sl) + 3];
                        }
                    } else if (l == 1) {
                        const uint32_t idx = a.e.del_idx[(size_t)g * cap + sl];
                        L.k[1][0][L.off[1][g] + sl] = idx;
                        if ((long long)idx >= Np) atomicOr(&L.bits[(idx - Np) >> 5], 1u << ((idx - Np) & 31));
                    } else {
                        const unsigned long long r = a.e.rel[(size_t)g * cap_rel + sl];
                        const long long i = (long long)(r >> 32);
                        const uint32_t lab = (uint32_t)(r & 0xffffffffull);
                        if (i >= Np) atomicOr(&L.map[i - Np], (lab + 1u) << kMapRelShift);
                        else if (mine) p.label[i] = (int32_t)lab;
                    }
                }
            }
        }
        __syncthreads();
        // ---- C: sort both lists (256-key chunks in registers, then ranks by search) ----
        if (tid >= kFinBlock - kWave) {  // exclusive prefix of the deleted bits per 32-position word (<= 128 words)
            const unsigned lane = (unsigned)tid & (kWave - 1), nw = (D + 31) / 32;
            const unsigned w0 = 2u * lane, w1 = w0 + 1u;
            const unsigned c0 = w0 < nw ? (unsigned)__popc(L.bits[w0]) : 0u;
            const unsigned c1 = w1 < nw ? (unsigned)__popc(L.bits[w1]) : 0u;
            unsigned incl = c0 + c1;
            for (unsigned off = 1; off < kWave; off <<= 1) {
                const unsigned t = __shfl_up(incl, off);
                if (lane >= off) incl += t;
            }
            const unsigned excl = incl - c0 - c1;
            if (w0 < nw) L.wpre[w0] = excl;
            if (w1 < nw) L.wpre[w1] = excl + c0;
        }
        const unsigned ncg = (G + kChunk - 1) / kChunk, ncd = (D + kChunk - 1) / kChunk;
        {
            const unsigned wave = (unsigned)tid / kWave, lane = (unsigned)tid & (kWave - 1), nwave = bd / kWave;
            for (unsigned ch = wave; ch < ncg + ncd; ch += nwave) {  // wave-uniform
                const bool is_g = ch < ncg;
                const unsigned base = (is_g ? ch : ch - ncg) * kChunk, n = is_g ? G : D;
                uint32_t *kk = L.k[is_g ? 0 : 1][0];
                uint32_t key[4], val[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned e = base + (unsigned)r * kWave + lane;
                    key[r] = e < n ? kk[e] : 0xffffffffu;
                    val[r] = is_g && e < n ? L.v[0][e] : 0u;
                }
                bitonic_sort256<2>(key, val, (int)lane);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned e = base + (unsigned)r * kWave + lane;
                    kk[e] = key[r];  // padding included: a chunk is always whole
                    if (is_g) L.v[0][e] = val[r];
                }
            }
        }
        __syncthreads();
        for (unsigned t = tid; t < G + D; t += bd) {  // rank = place in the chunk + keys below in the other chunks
            const bool is_g = t < G;
            const unsigned e = is_g ? t : t - G, nch = is_g ? ncg : ncd, own = e / kChunk;
            const uint32_t *kk = L.k[is_g ? 0 : 1][0];
            const uint32_t x = kk[e];
            unsigned rank = e - own * kChunk;
            for (unsigned chn = 0; chn < nch; ++chn)
                if (chn != own) rank += below_in_chunk(kk + chn * kChunk, x);
            L.k[is_g ? 0 : 1][1][rank] = x;
            if (is_g) L.v[1][rank] = L.v[0][e];
        }
        __syncthreads();
        const uint32_t *gslot = L.v[1], *del = L.k[1][1];
        // ---- D: one round of loads (the recycled positions of this block's
        //      in-place recycles, the tail survivors, the appended payloads), then
        //      the stores ----
        float rec[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int f = 0; f < 4; ++f)
                rec[q][f] = own_rec[q] && (f < dim || (f == 3 && a.e.rho_field >= 0))
                                ? a.e.gen_new[4 * (size_t)own_slot[q] + f] : 0.0f;
        unsigned t0, t1;
        share_of(G > D ? G : D, fb, nfb, t0, t1);
        for (unsigned t = t0 + tid; t < t1; t += bd) {
            const long long pi = Np + t;
            const bool survivor = t < D && !((L.bits[t >> 5] >> (t & 31)) & 1u);
            const bool append = t < G;
            float v[3 + SPH_MAX_CARRIED], d[3 + SPH_MAX_CARRIED];
            int32_t lab = 0;
            int64_t id = 0;
            long long hole = 0;
            if (survivor) {  // issue every load before any store
                const unsigned below = L.wpre[t >> 5] + (unsigned)__popc(L.bits[t >> 5] & ((1u << (t & 31)) - 1u));
                hole = del[t - below];  // the k-th survivor of the tail fills the k-th smallest hole
                const uint32_t m = L.map[t];
                const uint32_t ge = m & ((1u << kMapRelShift) - 1u), rl = m >> kMapRelShift;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (q < dim) v[q] = ge ? a.e.gen_new[4 * (size_t)(ge - 1u) + q] : p.pos[q][pi];
#pragma unroll
                for (int f = 0; f < SPH_MAX_CARRIED; ++f)
                    if (f < nc) v[3 + f] = ge && f == a.e.rho_field ? a.e.gen_new[4 * (size_t)(ge - 1u) + 3] : p.car[f][pi];
                lab = rl ? (int32_t)(rl - 1u) : p.label[pi];
                id = p.id[pi];
            }
            if (append) {
                const float *src = a.e.dup + (size_t)gslot[t] * (size_t)ds;
#pragma unroll
                for (int q = 0; q < 3 + SPH_MAX_CARRIED; ++q)
                    if (q < dim || (q >= 3 && q < 3 + nc)) d[q] = src[q];
            }
            if (survivor) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (q < dim) p.pos[q][hole] = v[q];
#pragma unroll
                for (int f = 0; f < SPH_MAX_CARRIED; ++f)
                    if (f < nc) p.car[f][hole] = v[3 + f];
                p.label[hole] = lab;
                p.id[hole] = id;
            }
            if (append) {  // duplicate of the t-th smallest source: label 0, fresh id
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (q < dim) p.pos[q][pi] = d[q];
#pragma unroll
                for (int f = 0; f < SPH_MAX_CARRIED; ++f)
                    if (f < nc) p.car[f][pi] = d[3 + f];
                p.label[pi] = 0;
                p.id[pi] = L.next + (long long)t;
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (own_rec[q]) {
                for (int f = 0; f < dim; ++f) p.pos[f][own_i[q]] = rec[q][f];
                if (a.e.rho_field >= 0) p.car[a.e.rho_field][own_i[q]] = rec[q][3];
            }
        // the sorted lists for sph_last_events
        if (fb == 0) {
            for (unsigned j = tid; j < G; j += bd) a.gen_sorted[j] = L.k[0][1][j];
            for (unsigned j = tid; j < D; j += bd) a.del_sorted[j] = del[j];
        }
    }
    // ---- the last block to take a ticket publishes the result and clears the counters ----
    if (tid == 0) L.last = ticket == (unsigned)nfb - 1u ? 1u : 0u;
    __syncthreads();
    if (L.last) {
        sph_result *r = a.result;
        if (tid < SPH_MAX_BUFFERS) {
            const long long nl = st == SPH_OK && tid < a.nb ? (long long)L.post[tid] : L.nl[tid];
            r->n_labelled[tid] = nl;
            c->n_labelled[tid] = nl;
        }
        if (tid >= kWave && tid < kWave + kSeg) {
            SegCtr &sc2 = c->seg[tid - kWave];
            sc2.n_gen = 0u;
            sc2.n_del = 0u;
            sc2.n_rel = 0u;
        }
        if (tid == 2 * kWave) {
            r->status = st;
            r->n_buffers = a.nb;
            r->n_generated = st == SPH_OK ? G : 0;
            r->n_deleted = st == SPH_OK ? D : 0;
            r->n_before = N;
            r->n_after = st == SPH_OK ? N - (long long)D + (long long)G : N;
            r->next_id = st == SPH_OK ? L.next + G : L.next;
            if (a.nf_full) c->nonfinite_full = 0u;
            c->cand_count = 0ull;
            c->cand_overflow = 0u;
            c->fin_ticket = 0u;
            if (st == SPH_OK) {
                c->next_id = L.next + G;
                *a.p.n_dev = N - (long long)D + (long long)G;
            }
        }
        for (int w = tid; w < words; w += (int)bd) a.e.part[w] = 0u;
    }
}

__global__ __launch_bounds__(kFinBlock) void k_finalize(FinArgs a) {
    __shared__ FinLds L;
    finalize_body(a, blockIdx.x, gridDim.x, L);
}

// ------------------------------------------------------------- identify --

struct IdentArgs {
    Parts p;
    const BufDev *bufs;
    int nb;
    int which;  // 0-based buffer or -1
    Ctl *ctl;
};

__global__ __launch_bounds__(kBuildBlock) void k_ident_check(IdentArgs a) {
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = a.p.pos[0][i], y = a.p.pos[1][i], z = a.p.dim == 3 ? a.p.pos[2][i] : 0.0f;
        bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
    }
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&a.ctl->ident_bad, 1u);
}

__global__ __launch_bounds__(kBuildBlock) void k_ident_apply(IdentArgs a) {
    __shared__ unsigned long long s_cnt[SPH_MAX_BUFFERS];
    if (threadIdx.x < SPH_MAX_BUFFERS) s_cnt[threadIdx.x] = 0ull;
    __syncthreads();
    if (a.ctl->ident_bad) return;
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    const int dim = a.p.dim;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t iters = (N + stride - 1) / stride;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t i = it * stride + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = i < N;
        int lab = -1;
        if (valid) {
            lab = a.p.label[i];
            const float x = a.p.pos[0][i], y = a.p.pos[1][i], z = dim == 3 ? a.p.pos[2][i] : 0.0f;
            for (int k = 0; k < a.nb; ++k) {
                if (a.which >= 0 && a.which != k) continue;
                const unsigned bits = classify(a.bufs[k], dim, x, y, z);
                if (bits & kBox) lab = k + 1;
            }
            a.p.label[i] = lab;
        }
        for (int k = 0; k < a.nb; ++k) {
            const unsigned long long n = (unsigned long long)__popcll(__ballot(valid && lab == k + 1));
            if ((threadIdx.x & 63) == 0 && n) atomicAdd(&s_cnt[k], n);
        }
    }
    __syncthreads();
    if (threadIdx.x < a.nb && s_cnt[threadIdx.x]) atomicAdd(&a.ctl->ident_count[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void k_ident_commit(IdentArgs a) {
    if (threadIdx.x == 0 && !a.ctl->ident_bad)
        for (int k = 0; k < a.nb; ++k) a.ctl->n_labelled[k] = (long long)a.ctl->ident_count[k];
}

// ------------------------------------- boundary conditions, rotating buffers --
//
// One wave per run of cover cells (as the classify step); a candidate is handled
// if it carries the buffer's label and lies in the check region (the exact
// decision, guard band included).  Every value is computed in FP64 with the
// expression order of the definition and rounded to FP32 once.

struct BcArgs {
    Parts p;
    const BufDev *bufs;
    int nb;
    const Ctl *ctl;            // Ctl::n_runs: length of the compact run list
    const int32_t *run_first;
    const int32_t *run_len;
    const uint8_t *run_buf;
    const int32_t *cell_start;
    const int32_t *cell_idx;
    int32_t vel[3];
    int which;         // rotation of this buffer (0-based); -1: boundary conditions of every buffer
    double center[3];  // rotation centre
    double m[9];       // rotation matrix, row-major
    unsigned *found;   // kCountReplicas copies of the per-buffer count of handled particles
};

// y = m x, rows summed left to right (two terms in 2-D).
__device__ __forceinline__ void mat_vec64(int dim, const double *m, const double x[3], double y[3]) {
#pragma clang fp contract(off)
    for (int r = 0; r < 3; ++r) {
        double acc = __dadd_rn(__dmul_rn(m[3 * r], x[0]), __dmul_rn(m[3 * r + 1], x[1]));
        if (dim == 3) acc = __dadd_rn(acc, __dmul_rn(m[3 * r + 2], x[2]));
        y[r] = acc;
    }
}

__device__ void apply_bc_one(const BcArgs &a, const BufDev &b, int64_t i, float x, float y, float z) {
#pragma clang fp contract(off)
    const Parts &p = a.p;
    const int dim = p.dim;
    if (b.bc_kind == SPH_BC_VELOCITY) {
        // local frame: r' = Q (r - O'), rows summed left to right
        const double d0 = __dadd_rn((double)x, -b.o[0]), d1 = __dadd_rn((double)y, -b.o[1]);
        const double d2 = dim == 3 ? __dadd_rn((double)z, -b.o[2]) : 0.0;
        double l1 = __dadd_rn(__dmul_rn(b.q[3], d0), __dmul_rn(b.q[4], d1));
        double l2 = 0.0;
        if (dim == 3) {
            l1 = __dadd_rn(l1, __dmul_rn(b.q[5], d2));
            l2 = __dadd_rn(__dadd_rn(__dmul_rn(b.q[6], d0), __dmul_rn(b.q[7], d1)), __dmul_rn(b.q[8], d2));
        }
        double f = 1.0;
        if (b.profile == SPH_PROFILE_PARABOLIC_Y) {
            const double q = __ddiv_rn(l1, b.bc_radius);
            f = __dadd_rn(1.0, -__dmul_rn(q, q));
        } else if (b.profile == SPH_PROFILE_PARABOLIC_R) {
            const double r2 = __dadd_rn(__dmul_rn(l1, l1), __dmul_rn(l2, l2));
            f = __dadd_rn(1.0, -__ddiv_rn(r2, __dmul_rn(b.bc_radius, b.bc_radius)));
        }
        const double w = __dmul_rn(b.bc_u, f);  // v' = (u f, 0, 0); v = Q^T v'
        for (int c = 0; c < dim; ++c) p.car[a.vel[c]][i] = (float)__dmul_rn(b.q[c], w);
    } else {
        // v <- (v . u_hat) u_hat with u_hat = Q^T e_x, the first row of Q
        double v[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < dim; ++c) v[c] = (double)p.car[a.vel[c]][i];
        double dot = __dadd_rn(__dmul_rn(b.q[0], v[0]), __dmul_rn(b.q[1], v[1]));
        if (dim == 3) dot = __dadd_rn(dot, __dmul_rn(b.q[2], v[2]));
        for (int c = 0; c < dim; ++c) p.car[a.vel[c]][i] = (float)__dmul_rn(dot, b.q[c]);
    }
}

__device__ void rotate_one(const BcArgs &a, int64_t i, float x, float y, float z) {
#pragma clang fp contract(off)
    const Parts &p = a.p;
    const int dim = p.dim;
    const double d[3] = {__dadd_rn((double)x, -a.center[0]), __dadd_rn((double)y, -a.center[1]),
                         dim == 3 ? __dadd_rn((double)z, -a.center[2]) : 0.0};
    double e[3];
    mat_vec64(dim, a.m, d, e);
    for (int c = 0; c < dim; ++c) p.pos[c][i] = (float)__dadd_rn(a.center[c], e[c]);
    if (a.vel[0] >= 0) {
        double v[3] = {0.0, 0.0, 0.0}, w[3];
        for (int c = 0; c < dim; ++c) v[c] = a.vel[c] >= 0 ? (double)p.car[a.vel[c]][i] : 0.0;
        mat_vec64(dim, a.m, v, w);
        for (int c = 0; c < dim; ++c)
            if (a.vel[c] >= 0) p.car[a.vel[c]][i] = (float)w[c];
    }
}

__global__ __launch_bounds__(kClassifyBlock) void k_buffer_bc(BcArgs a) {
    __shared__ BufDev sb[SPH_MAX_BUFFERS];
    __shared__ unsigned s_cnt[SPH_MAX_BUFFERS];
    __shared__ int s_nruns;
    for (int t = threadIdx.x; t < a.nb * (int)(sizeof(BufDev) / 4); t += blockDim.x)
        reinterpret_cast<uint32_t *>(sb)[t] = reinterpret_cast<const uint32_t *>(a.bufs)[t];
    if (threadIdx.x < SPH_MAX_BUFFERS) s_cnt[threadIdx.x] = 0u;
    if (threadIdx.x == 0) s_nruns = a.ctl->n_runs;
    __syncthreads();
    const int n_runs = s_nruns;
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const int dim = a.p.dim;
    for (int r = blockIdx.x * wpb + wave; r < n_runs; r += gridDim.x * wpb) {
        const int k = a.run_buf[r];
        const BufDev &b = sb[k];
        if (a.which < 0 ? b.bc_kind == SPH_BC_NONE : k != a.which) continue;  // wave-uniform
        const int c0 = a.run_first[r];
        const int j0 = a.cell_start[c0];
        const int j1 = a.cell_start[c0 + a.run_len[r]];
        unsigned long long handled = 0;
        for (int jb = j0; jb < j1; jb += kWave) {
            const int j = jb + lane;
            const int64_t i = j < j1 ? a.cell_idx[j] : 0;
            if (!(j < j1 && i < N)) continue;
            const float x = a.p.pos[0][i], y = a.p.pos[1][i], z = dim == 3 ? a.p.pos[2][i] : 0.0f;
            if (a.p.label[i] != k + 1) continue;
            if (!(classify(b, dim, x, y, z) & kIn)) continue;  // outside the check region: reported
            ++handled;
            if (a.which < 0) apply_bc_one(a, b, i, x, y, z);
            else rotate_one(a, i, x, y, z);
        }
        handled = wave_sum(handled);
        if (lane == 0 && handled) atomicAdd(&s_cnt[k], (unsigned)handled);
    }
    __syncthreads();
    if (threadIdx.x < a.nb && s_cnt[threadIdx.x])
        atomicAdd(&a.found[(size_t)(blockIdx.x % kCountReplicas) * SPH_MAX_BUFFERS + threadIdx.x], s_cnt[threadIdx.x]);
}

// Sum the per-buffer counts (one thread per copy and buffer), clear them, and
// compare with the labelled counts of the buffers the pass was meant to handle.
constexpr int kBcFinishBlock = kCountReplicas * 16;

__global__ __launch_bounds__(kBcFinishBlock) void k_bc_finish(unsigned *found, const BufDev *bufs, int nb, int which,
                                                              Ctl *ctl) {
    __shared__ unsigned s_tot[SPH_MAX_BUFFERS];
    if (threadIdx.x < SPH_MAX_BUFFERS) s_tot[threadIdx.x] = 0u;
    __syncthreads();
    const int r = threadIdx.x / 16, k = threadIdx.x % 16;
    if (k < nb) {
        unsigned *w = &found[(size_t)r * SPH_MAX_BUFFERS + k];
        const unsigned v = *w;
        if (v) {
            *w = 0u;
            atomicAdd(&s_tot[k], v);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned bad = 0;
        for (int j = 0; j < nb; ++j) {
            const bool involved = which < 0 ? bufs[j].bc_kind != SPH_BC_NONE : j == which;
            if (involved && (long long)s_tot[j] != ctl->n_labelled[j]) bad = 1;
        }
        ctl->bc_status = bad ? (unsigned)SPH_ERR_CFL : (unsigned)SPH_OK;
    }
}

// ------------------------------------------- cover cells of a turned buffer --
//
// The cells of a dense grid whose boxes, dilated by eps and with the edge cells
// extended to infinity, meet a buffer's check region (an oriented box), as the
// host computes them at definition, here on the device for a buffer that has
// just been turned.  Along a row of cells (fixed y and z) the cells that meet a
// convex region form an interval; its ends are found by two binary searches on
// unions of consecutive cells (the union of cells lo..x is one box, and whether
// it meets the region is monotone in x).  One thread per row finds the interval
// (k_cover_rows), then one workgroup lays the rows' runs out (k_cover_write),
// maps them to cell keys, keeps the per-cell cover mask, and rebuilds the
// compact run list that the classify and boundary kernels walk.

struct CoverObb {
    double c[3];
    double ax[3][3];  // rows: local axes
    double h[3];      // half-extents of the check region
};

// Separating-axis test of the oriented box against the axis-aligned box lo..hi
// (true when they may intersect; a relative 1e-12 slack keeps it conservative
// near touching), as in the host geometry.
__device__ bool obb_meets_box(int m, const CoverObb &b, const double lo[3], const double hi[3]) {
    double ac[3], ah[3], t[3];
    for (int j = 0; j < 3; ++j) {
        ac[j] = 0.5 * (lo[j] + hi[j]);
        ah[j] = 0.5 * (hi[j] - lo[j]);
        t[j] = ac[j] - b.c[j];
    }
    auto separated = [&](const double L[3]) {
        double proj_t = 0.0, ra = 0.0, rb = 0.0;
        for (int j = 0; j < m; ++j) {
            proj_t += L[j] * t[j];
            ra += ah[j] * fabs(L[j]);
        }
        for (int i = 0; i < m; ++i) {
            double d = 0.0;
            for (int j = 0; j < m; ++j) d += L[j] * b.ax[i][j];
            rb += b.h[i] * fabs(d);
        }
        const double slack = 1e-12 * (fabs(proj_t) + ra + rb);
        return fabs(proj_t) > ra + rb + slack;
    };
    for (int j = 0; j < m; ++j) {
        double L[3] = {0.0, 0.0, 0.0};
        L[j] = 1.0;
        if (separated(L)) return false;
    }
    for (int i = 0; i < m; ++i)
        if (separated(b.ax[i])) return false;
    if (m == 3) {
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                double E[3] = {0.0, 0.0, 0.0};
                E[j] = 1.0;
                const double *a = b.ax[i];
                const double L[3] = {E[1] * a[2] - E[2] * a[1], E[2] * a[0] - E[0] * a[2], E[0] * a[1] - E[1] * a[0]};
                if (L[0] * L[0] + L[1] * L[1] + L[2] * L[2] < 1e-20) continue;
                if (separated(L)) return false;
            }
    }
    return true;
}

struct CoverArgs {
    Ctl *ctl;
    int k, dim;
    CoverObb obb;
    double blo[3], bhi[3];       // axis-aligned box of the check region
    double glo[3], cs, eps;      // grid origin, cell size, dilation of the cell boxes
    int32_t dims[3];
    int32_t lo_i[3], hi_i[3];    // cells to consider (inclusive)
    int32_t *row_lo, *row_hi;    // per row (y fastest, then z): covered x interval (lo > hi: none)
    int64_t max_rows;
    // k_cover_write
    BufDev rec;                  // the turned buffer's record
    BufDev *bufs;
    int nb;
    int cap;                     // cells per run at most
    int32_t rbase[SPH_MAX_BUFFERS], rmax[SPH_MAX_BUFFERS];
    int32_t *src_first, *src_len;
    int32_t *run_first, *run_len;
    uint8_t *run_buf;
    unsigned *cover;             // per-cell mask (two 16-bit cells per word), or null
    Grid g;                      // key mapping (dense or brick-sparse)
};

// Box of the cells ix0..ix1 of row (iy, iz), dilated and edge-extended.
__device__ void cells_box(const CoverArgs &a, int ix0, int ix1, int iy, int iz, double lo[3], double hi[3]) {
    const int idx0[3] = {ix0, iy, iz}, idx1[3] = {ix1, iy, iz};
    for (int j = 0; j < 3; ++j) {
        lo[j] = hi[j] = 0.0;
        if (j >= a.dim) continue;
        lo[j] = a.glo[j] + idx0[j] * a.cs - a.eps;
        hi[j] = a.glo[j] + (idx1[j] + 1) * a.cs + a.eps;
        if (idx0[j] == 0) lo[j] = fmin(lo[j], a.blo[j] - a.cs);
        if (idx1[j] == a.dims[j] - 1) hi[j] = fmax(hi[j], a.bhi[j] + a.cs);
    }
}

__global__ __launch_bounds__(256) void k_cover_rows(CoverArgs a) {
    const int ny = a.hi_i[1] - a.lo_i[1] + 1;
    const int nz = a.dim == 3 ? a.hi_i[2] - a.lo_i[2] + 1 : 1;
    const int64_t rows = (int64_t)ny * nz;
    // the buffer's old cover leaves the mask (its new one is set by k_cover_write)
    if (a.cover) {
        const int n_old = a.ctl->run_cnt[a.k];
        const unsigned clear = ~(1u << a.k);
        for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_old; r += gridDim.x * blockDim.x) {
            const int32_t f = a.src_first[a.rbase[a.k] + r], l = a.src_len[a.rbase[a.k] + r];
            for (int32_t q = 0; q < l; ++q) {
                const uint32_t key = (uint32_t)(f + q);
                atomicAnd(&a.cover[key >> 1], (key & 1u) ? ((clear << 16) | 0xffffu) : (clear | 0xffff0000u));
            }
        }
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows && r < a.max_rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int iy = a.lo_i[1] + (int)(r % ny), iz = a.dim == 3 ? a.lo_i[2] + (int)(r / ny) : 0;
        const int x0 = a.lo_i[0], x1 = a.hi_i[0];
        double lo[3], hi[3];
        int xa = x1 + 1, xb = x0 - 1;
        cells_box(a, x0, x1, iy, iz, lo, hi);
        if (obb_meets_box(a.dim, a.obb, lo, hi)) {
            // leftmost x whose union x0..x meets the region, rightmost whose union x..x1 does
            int l = x0 - 1, h = x1;  // P(l) false (empty union), P(h) true
            while (h - l > 1) {
                const int mid = l + (h - l) / 2;
                cells_box(a, x0, mid, iy, iz, lo, hi);
                if (obb_meets_box(a.dim, a.obb, lo, hi)) h = mid;
                else l = mid;
            }
            xa = h;
            l = x0;
            h = x1 + 1;  // Q(l) true, Q(h) false (empty union)
            while (h - l > 1) {
                const int mid = l + (h - l) / 2;
                cells_box(a, mid, x1, iy, iz, lo, hi);
                if (obb_meets_box(a.dim, a.obb, lo, hi)) l = mid;
                else h = mid;
            }
            xb = l;
        }
        a.row_lo[r] = xa;
        a.row_hi[r] = xb;
    }
}

// Runs of row r (covered cells xa..xb) as keys: consecutive keys, at most cap
// cells; on the brick-sparse grid a run also ends at a brick face, and cells of
// inactive bricks are left to the overflow cell (reported through *ovf).
template <bool kWrite>
__device__ int row_runs(const CoverArgs &a, int xa, int xb, int iy, int iz, int32_t *first, int32_t *len, bool &ovf) {
    int n = 0;
    uint32_t start = 0, prev = 0;
    int cur = 0;
    for (int ix = xa; ix <= xb; ++ix) {
        const uint32_t key = key_of_cell(a.g, (uint32_t)ix, (uint32_t)iy, (uint32_t)iz);
        if (a.g.blog2 > 0 && key == a.g.overflow_key) {
            ovf = true;
            if (cur > 0) {
                if (kWrite) {
                    first[n] = (int32_t)start;
                    len[n] = cur;
                }
                ++n;
                cur = 0;
            }
            continue;
        }
        if (cur > 0 && key == prev + 1u && cur < a.cap) {
            ++cur;
        } else {
            if (cur > 0) {
                if (kWrite) {
                    first[n] = (int32_t)start;
                    len[n] = cur;
                }
                ++n;
            }
            start = key;
            cur = 1;
        }
        prev = key;
    }
    if (cur > 0) {
        if (kWrite) {
            first[n] = (int32_t)start;
            len[n] = cur;
        }
        ++n;
    }
    return n;
}

constexpr int kCoverBlock = 1024;

// One workgroup: the turned buffer's record, its runs from the row intervals, its
// mask bits and run count, then the compact run list of every buffer.
__global__ __launch_bounds__(kCoverBlock) void k_cover_write(CoverArgs a) {
    __shared__ int s_wave[kCoverBlock / kWave];
    __shared__ int s_base, s_ovf;
    __shared__ int s_pre[SPH_MAX_BUFFERS + 1];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0) {
        s_base = 0;
        s_ovf = 0;
    }
    for (int w = tid; w < (int)(sizeof(BufDev) / 4); w += blockDim.x)
        reinterpret_cast<uint32_t *>(a.bufs + a.k)[w] = reinterpret_cast<const uint32_t *>(&a.rec)[w];
    __syncthreads();
    const int ny = a.hi_i[1] - a.lo_i[1] + 1;
    const int nz = a.dim == 3 ? a.hi_i[2] - a.lo_i[2] + 1 : 1;
    const int64_t rows = min((int64_t)ny * nz, a.max_rows);
    int32_t *df = a.src_first + a.rbase[a.k], *dl = a.src_len + a.rbase[a.k];
    for (int64_t r0 = 0; r0 < rows; r0 += blockDim.x) {  // block-uniform
        const int64_t r = r0 + tid;
        int xa = 0, xb = -1, iy = 0, iz = 0;
        if (r < rows) {
            xa = a.row_lo[r];
            xb = a.row_hi[r];
            iy = a.lo_i[1] + (int)(r % ny);
            iz = a.dim == 3 ? a.lo_i[2] + (int)(r / ny) : 0;
        }
        bool ovf = false;
        const int n = xa <= xb ? row_runs<false>(a, xa, xb, iy, iz, nullptr, nullptr, ovf) : 0;
        if (ovf) s_ovf = 1;
        int incl = n;
        for (int off = 1; off < kWave; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        if (lane == kWave - 1) s_wave[wave] = incl;
        __syncthreads();
        int before = s_base;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        int total = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) total += s_wave[w];
        const int at = before + incl - n;
        if (n > 0 && at + n <= a.rmax[a.k]) row_runs<true>(a, xa, xb, iy, iz, df + at, dl + at, ovf);
        __syncthreads();
        if (tid == 0) s_base += total;
        __syncthreads();
    }
    int cnt = s_base;
    if (s_ovf && a.g.blog2 > 0) {  // every inactive brick is one overflow cell: one run for it
        if (tid == 0 && cnt < a.rmax[a.k]) {
            df[cnt] = (int32_t)a.g.overflow_key;
            dl[cnt] = 1;
        }
        ++cnt;
    }
    if (cnt > a.rmax[a.k]) {  // cannot happen with the range sized from the sphere bound; keep what fits
        if (tid == 0) {
            a.ctl->cover_fault = 1;
            a.ctl->bc_status = (unsigned)SPH_ERR_HIP;
        }
        cnt = a.rmax[a.k];
    }
    __syncthreads();
    if (a.cover) {  // the new cover's mask bits
        for (int r = tid; r < cnt; r += blockDim.x)
            for (int32_t q = 0; q < dl[r]; ++q) {
                const uint32_t key = (uint32_t)(df[r] + q);
                atomicOr(&a.cover[key >> 1], (1u << a.k) << ((key & 1u) * 16u));
            }
    }
    // the compact list of every buffer's runs
    if (tid == 0) {
        int acc = 0;
        for (int k = 0; k < a.nb; ++k) {
            const int c = k == a.k ? cnt : a.ctl->run_cnt[k];
            s_pre[k] = acc;
            acc += c;
        }
        s_pre[a.nb] = acc;
        a.ctl->run_cnt[a.k] = cnt;
        a.ctl->n_runs = acc;
    }
    __syncthreads();
    for (int k = 0; k < a.nb; ++k) {
        const int c = s_pre[k + 1] - s_pre[k];
        for (int q = tid; q < c; q += blockDim.x) {
            a.run_first[s_pre[k] + q] = a.src_first[a.rbase[k] + q];
            a.run_len[s_pre[k] + q] = a.src_len[a.rbase[k] + q];
            a.run_buf[s_pre[k] + q] = (uint8_t)k;
        }
    }
}

// Compact run list from the per-buffer ranges (after a definition or a grid fit).
__global__ __launch_bounds__(kCoverBlock) void k_runs_assemble(CoverArgs a) {
    __shared__ int s_pre[SPH_MAX_BUFFERS + 1];
    const int tid = threadIdx.x;
    if (tid == 0) {
        int acc = 0;
        for (int k = 0; k < a.nb; ++k) {
            s_pre[k] = acc;
            acc += a.ctl->run_cnt[k];
        }
        s_pre[a.nb] = acc;
        a.ctl->n_runs = acc;
    }
    __syncthreads();
    for (int k = 0; k < a.nb; ++k) {
        const int c = s_pre[k + 1] - s_pre[k];
        for (int q = tid; q < c; q += blockDim.x) {
            a.run_first[s_pre[k] + q] = a.src_first[a.rbase[k] + q];
            a.run_len[s_pre[k] + q] = a.src_len[a.rbase[k] + q];
            a.run_buf[s_pre[k] + q] = (uint8_t)k;
        }
    }
}

// Per-cell cover mask from the compact run list (the mask is cleared before).
__global__ __launch_bounds__(256) void k_mask_set(CoverArgs a) {
    const int n = a.ctl->n_runs;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int32_t f = a.run_first[r], l = a.run_len[r];
        const unsigned bit = 1u << a.run_buf[r];
        for (int32_t q = 0; q < l; ++q) {
            const uint32_t key = (uint32_t)(f + q);
            atomicOr(&a.cover[key >> 1], bit << ((key & 1u) * 16u));
        }
    }
}

// ------------------------------------------------------ neighbour search --
//
// The cell list also serves the solver's neighbour search: with the cell size at
// least the search radius (the kernel support 2h of Section 3 is the cell size,
// 2.6 dp), every particle closer than the radius lies in the 3^d cells around the
// particle's own.  Binning is FP32, so two particles less than one cell apart can
// land two cells apart when one of them lies within `band` (cell units, from the
// binning error bound) of its cell's face; on such a side the block is widened by
// one cell.  Distances: FP32 first; within a relative 2^-16 of the squared radius
// the decision is taken in FP64 as ((dx*dx + dy*dy) + dz*dz), dx = (double)x_i -
// (double)x_j, each operation rounded separately.
//
// The positions are first copied into cell order (slot k of cell_idx), so one
// thread per slot reads its own position coalesced, the threads of one cell walk
// identical loops over the same contiguous slots, and on the dense grid the three
// cells of a stencil row are one contiguous slot range.

struct NbrArgs {
    Parts p;
    Grid g;
    const int32_t *cell_start;
    const int32_t *cell_idx;
    float *xs, *ys, *zs;  // positions in cell order (build scratch)
    double r2;            // radius^2
    float r2_in, r2_out;  // FP32 squared distances surely inside / outside
    float band;           // cell units
    int32_t *counts;
};

constexpr int kNbrBlock = 256;

__global__ __launch_bounds__(kNbrBlock) void k_nbr_order(NbrArgs a) {
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = a.cell_idx[k];
        a.xs[k] = a.p.pos[0][j];
        a.ys[k] = a.p.pos[1][j];
        if (a.g.dim == 3) a.zs[k] = a.p.pos[2][j];
    }
}

// Pairs of slot k with the slots [m0, m1): FP32 test, FP64 in the band.  The main
// loop counts the pairs surely inside without a branch (four candidates' loads
// issued together) and only notes whether any pair fell in the band; the rare
// range that has one is walked again for the exact decisions of those pairs.
template <bool d3>
__device__ __forceinline__ int nbr_range(const NbrArgs &a, int64_t k, const float (&pi)[3], int32_t m0, int32_t m1) {
    constexpr int U = 4;
    int cnt = 0;
    bool band = false;
    auto test = [&](int32_t m, float xj, float yj, float zj) {
        const float dx = pi[0] - xj, dy = pi[1] - yj, dz = pi[2] - zj;
        const float d2 = (dx * dx + dy * dy) + dz * dz;
        const bool other = m != k;
        cnt += (other && d2 < a.r2_in) ? 1 : 0;
        band = band || (other && !(d2 < a.r2_in) && !(d2 > a.r2_out));
    };
    int32_t m = m0;
    for (; m + U <= m1; m += U) {
        float xj[U], yj[U], zj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xj[u] = a.xs[m + u];
            yj[u] = a.ys[m + u];
            zj[u] = d3 ? a.zs[m + u] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) test(m + u, xj[u], yj[u], zj[u]);
    }
    for (; m < m1; ++m) test(m, a.xs[m], a.ys[m], d3 ? a.zs[m] : 0.0f);
    if (band) {
        for (m = m0; m < m1; ++m) {
            if (m == k) continue;
            const float xj = a.xs[m], yj = a.ys[m], zj = d3 ? a.zs[m] : 0.0f;
            const float dx = pi[0] - xj, dy = pi[1] - yj, dz = pi[2] - zj;
            const float d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 < a.r2_in || d2 > a.r2_out) continue;  // decided above
            const double ex = __dadd_rn((double)pi[0], -(double)xj);
            const double ey = __dadd_rn((double)pi[1], -(double)yj);
            const double ez = __dadd_rn((double)pi[2], -(double)zj);
            const double e2 = __dadd_rn(__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)), __dmul_rn(ez, ez));
            if (e2 < a.r2) ++cnt;
        }
    }
    return cnt;
}

template <int dim>
__global__ __launch_bounds__(kNbrBlock) void k_neighbor_count(NbrArgs a) {
    constexpr bool d3 = dim == 3;
    const int64_t N = live_count(a.p.n_dev, a.p.capacity);
    const Grid &g = a.g;
    // XCD-contiguous tiles: the stencil rows an XCD reads stay within a narrower slot
    // window, so more of them hit its L2 (2.12 -> 2.01 ms on the pipe)
    for (int64_t k = (int64_t)logical_block() * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        const float pi[3] = {a.xs[k], a.ys[k], d3 ? a.zs[k] : 0.0f};
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
        for (int ax = 0; ax < dim; ++ax) {
            const float t = (pi[ax] - g.lo[ax]) * g.inv_cs;  // as in cell_coords
            const float f = floorf(t);
            const float cl = fminf(fmaxf(f, 0.0f), (float)(g.dims[ax] - 1));
            const int c = (int)cl;
            const bool inside = f == cl;  // not clamped to an edge cell (and not NaN)
            const float fr = t - f;       // exact
            lo[ax] = max(0, c - 1 - ((inside && fr < a.band) ? 1 : 0));
            hi[ax] = min(g.dims[ax] - 1, c + 1 + ((inside && fr > 1.0f - a.band) ? 1 : 0));
        }
        int cnt = 0;
        if (g.blog2 == 0) {
            // dense: the cells lo[0]..hi[0] of a row are consecutive keys, one slot range
            for (int iz = lo[2]; iz <= hi[2]; ++iz)
                for (int iy = lo[1]; iy <= hi[1]; ++iy) {
                    const uint32_t k0 = key_of_cell(g, (uint32_t)lo[0], (uint32_t)iy, (uint32_t)iz);
                    const uint32_t k1 = k0 + (uint32_t)(hi[0] - lo[0]);
                    cnt += nbr_range<d3>(a, k, pi, a.cell_start[k0], a.cell_start[k1 + 1]);
                }
        } else {
            bool overflow_seen = false;
            for (int iz = lo[2]; iz <= hi[2]; ++iz)
                for (int iy = lo[1]; iy <= hi[1]; ++iy)
                    for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                        const uint32_t key = key_of_cell(g, (uint32_t)ix, (uint32_t)iy, (uint32_t)iz);
                        if (key == g.overflow_key) {  // one cell for all inactive bricks
                            if (overflow_seen) continue;
                            overflow_seen = true;
                        }
                        cnt += nbr_range<d3>(a, k, pi, a.cell_start[key], a.cell_start[key + 1]);
                    }
        }
        a.counts[a.cell_idx[k]] = cnt;
    }
}

// ----------------------------------------------------------------- batches --
//
// Every phase of every domain of a batch in one launch: a static table maps each
// block to (domain, block index within that domain's share of the launch).

struct BlockMap {
    int32_t d;   // domain
    int32_t vb;  // block within the domain
};

// The tables are padded to a multiple of 8 entries (padding: d = -1) and read in
// the XCD-renumbered order, so each XCD takes a contiguous range of the table (and
// so of each domain's particles, as in the single-domain launches).
__global__ __launch_bounds__(kBuildBlock) void kb_count(const CountArgs *args, const BlockMap *map,
                                                        const int32_t *vg) {
    const BlockMap m = map[logical_block()];
    if (m.d < 0) return;
    count_body<false>(args[m.d], m.vb, vg[m.d]);
}

__global__ __launch_bounds__(kScanBlock) void kb_scan(const ScanArgs *args, const BlockMap *map) {
    const BlockMap m = map[logical_block()];
    if (m.d < 0) return;
    __shared__ ScanLds L;
    scan_body(args[m.d], L);
}

__global__ __launch_bounds__(kBuildBlock) void kb_scatter(const ScatterArgs *args, const BlockMap *map,
                                                          const int32_t *vg) {
    const BlockMap m = map[logical_block()];
    if (m.d < 0) return;
    scatter_body(args[m.d], m.vb, vg[m.d]);
}

__global__ __launch_bounds__(kClassifyBlock) void kb_classify(const LocalArgs *args, const BlockMap *map,
                                                              const int32_t *vg) {
    const BlockMap m = map[logical_block()];
    if (m.d < 0) return;
    classify_body(args[m.d], m.vb, vg[m.d]);
}

__global__ __launch_bounds__(kFinBlock) void kb_finalize(const FinArgs *args, int nfb) {
    __shared__ FinLds L;
    finalize_body(args[blockIdx.x / nfb], blockIdx.x % nfb, nfb, L);
}

}  // namespace

// ====================================================================== host ==

// ------------------------------------------------------------ build method --
//
// Two builds give the same cell list (up to the order inside a cell): the
// three-kernel counting sort (one atomic per run of equal keys in a wave on the
// cell counters, look-back scan, scatter) and the bucketed one (workgroup
// histograms of cell buckets, bucket scatter, LDS counting sort per bucket).  Which
// is faster depends on the particle order: the counting sort wins while the array
// keeps long runs of one cell (a lattice just built), the bucketed one once the
// flow has scattered it.  SPH_BUILD_AUTO times both on the stream with events and
// runs the faster: each is timed on kExploreSamples builds after one untimed
// warm-up build, then the choice is re-checked every kReprobe builds by timing one
// build of each (a 3 % margin before switching).  A method's time is the median of
// its last three timings (with two, the smaller): a build slowed by something else
// on the GPU only ever adds time.  Events are read only once they have completed
// (hipEventQuery), so the host never waits on them.

constexpr int kMethCounting = 0, kMethBucketed = 1;
constexpr int kTimerSets = 8;
constexpr int kExploreSamples = 3;
constexpr int kReprobe = 64;

struct BuildTimer {
    bool init = false, ok = false;   // events created (ok: all of them)
    hipEvent_t ev[kTimerSets][4] = {};  // count pass start/end, cells pass start/end
    bool busy[kTimerSets] = {};
    bool cells_done[kTimerSets] = {};
    int meth[kTimerSets] = {};
    double last[2][3] = {};          // latest timings per method (us), a ring
    double est[2] = {0.0, 0.0};      // build time per method (us) from the ring
    int64_t samples[2] = {0, 0};
    int64_t builds = 0;
    int cur = kMethCounting;
};

struct sph_ctx {
    int dim = 2;
    double lo[3] = {0, 0, 0};
    double cs = 0, dp = 0;
    int32_t dims[3] = {1, 1, 1};
    int64_t n_cells = 0;
    // brick-sparse grid (blog2 > 0)
    int blog2 = 0, bmargin = 1;
    int32_t bdims[3] = {1, 1, 1};
    int64_t n_bricks = 0;
    std::vector<int32_t> h_brick_slot;
    int32_t *d_brick_slot = nullptr;
    int64_t capacity = 0;
    unsigned max_events = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int build_blocks = 0;
    int full_blocks = 0;
    bool built = false;          // a build is pending for the next local update
    int64_t built_capacity = 0;
    // bumped whenever what a batch bakes into its launch tables changes (cover runs,
    // grid arrays, field roles): a batch made before refuses to step
    uint64_t layout_gen = 0;

    int nb = 0;
    BufDev hb[SPH_MAX_BUFFERS];
    double b_origin[SPH_MAX_BUFFERS][3], b_rot[SPH_MAX_BUFFERS][9], b_half[SPH_MAX_BUFFERS][3],
        b_margin[SPH_MAX_BUFFERS];
    // Cover runs: buffer k's runs live in its own range [rbase[k], rbase[k] + rmax[k])
    // of d_src_* (sized for any orientation, so a turn recomputes them in place on
    // the device); the compact list d_run_* (all buffers' runs back to back, count
    // in Ctl::n_runs) is what the classify and boundary kernels walk.
    int32_t rbase[SPH_MAX_BUFFERS] = {}, rmax[SPH_MAX_BUFFERS] = {}, hcnt[SPH_MAX_BUFFERS] = {};
    int64_t src_cap = 0, max_rows = 0;
    int32_t *d_src_first = nullptr, *d_src_len = nullptr;
    int32_t *d_row_lo = nullptr, *d_row_hi = nullptr;  // per-row intervals of a turned buffer's cover

    BufDev *d_bufs = nullptr;
    int32_t *d_run_first = nullptr, *d_run_len = nullptr;
    uint8_t *d_run_buf = nullptr;
    int n_runs = 0;  // runs at the last host computation (launch sizes; the kernels read Ctl::n_runs)

    int32_t *d_count = nullptr, *d_cell_start = nullptr, *d_cell_idx = nullptr;
    unsigned long long *d_cand = nullptr;        // candidate list of the full scan
    // merged step (the default update path): the count pass of the build also lists
    // the cover cells' particles near a check region as candidates; the update
    // classifies them beside the build's scatter, then finalizes.  Off: the update
    // walks the cover cells of the finished cell list.
    bool merged = true;
    bool scan_pending = false;   // a merged build's cells pass is not enqueued yet
    bool ev_pending = false;     // a merged build's candidates are not classified and finalized yet
    bool nf_full_next = false;   // the next cover-walk finalize reads the count pass's non-finite flag
    uint16_t *d_cover = nullptr; // per cell: bit k set if the cell is in buffer k's cover
    // bucketed build (grids of at most kMaxBuckets * kMaxBucketCells cells; the
    // three-kernel counting sort otherwise)
    bool bk = false;
    int bshift = 0, nbk = 0;
    uint32_t *d_bk_count = nullptr, *d_bk_start = nullptr;
    uint2 *d_ent = nullptr, *d_tmp = nullptr;
    // build method: sph_config::build_method; meth is the latest build's (its cells
    // pass follows it), timed on timer set tset (-1: untimed)
    int build_pref = SPH_BUILD_AUTO;
    int last_method = SPH_BUILD_AUTO;  // sph_build_method of the latest build (AUTO: none yet)
    int meth = 0;
    int tset = -1;
    BuildTimer bt;
    int64_t cover_cells = 0;
    uint32_t *d_keys = nullptr;                  // packed (key, rank) of each particle (three-kernel build)
    unsigned long long *d_keyrank = nullptr;     // full (key, rank) of the particles that do not fit
    int32_t rbits = 1;                           // rank bits of the packed form
    unsigned long long *d_tile_state = nullptr;
    int64_t n_tiles = 0;

    uint32_t *d_gen_idx = nullptr, *d_del_idx = nullptr, *d_gen_sorted = nullptr, *d_del_sorted = nullptr;
    float *d_gen_new = nullptr, *d_dup = nullptr;
    unsigned long long *d_rel = nullptr;
    Ctl *d_ctl = nullptr;
    unsigned *d_part = nullptr;
    unsigned *d_bcfound = nullptr;    // per-buffer counts of a boundary-condition / rotation pass
    unsigned *h_bc_status = nullptr;  // pinned
    sph_fields fields = {{-1, -1, -1}, -1};
    sph_result *d_result = nullptr;
    sph_result *h_result = nullptr;  // pinned
    bool any_update = false;

    // optional per-launch timing
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;  // 2 per slot
    std::vector<int> prof_phase;      // phase of each used slot
    size_t prof_used = 0;
    double prof_ms[SPH_NPHASE] = {};
    int64_t prof_n[SPH_NPHASE] = {};
};

namespace {

#define HIP_TRY(expr)                               \
    do {                                            \
        if ((expr) != hipSuccess) return SPH_ERR_HIP; \
    } while (0)

#define HIP_CHECKED(expr)                           \
    do {                                            \
        const sph_status st_ = (expr);              \
        if (st_ != SPH_OK) return st_;              \
    } while (0)

constexpr size_t kProfSlots = 8192;
constexpr int kBatchPhases = 5;  // count, scan, scatter, classify, finalize

// Bracket one launch with events when profiling is on (a no-op otherwise).
struct ProfScope {
    sph_ctx *c;
    hipStream_t s;
    size_t slot = 0;
    bool on = false;
    ProfScope(sph_ctx *ctx, int phase, hipStream_t stream = nullptr) : c(ctx), s(stream ? stream : ctx->stream) {
        if (!c->prof_on || c->prof_used >= kProfSlots) return;
        slot = c->prof_used++;
        c->prof_phase[slot] = phase;
        on = hipEventRecord(c->prof_ev[2 * slot], s) == hipSuccess;
    }
    ~ProfScope() {
        if (on) (void)hipEventRecord(c->prof_ev[2 * slot + 1], s);
    }
};

void prof_drain(sph_ctx *c) {
    for (size_t s = 0; s < c->prof_used; ++s) {
        float ms = 0.0f;
        if (hipEventSynchronize(c->prof_ev[2 * s + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms, c->prof_ev[2 * s], c->prof_ev[2 * s + 1]) == hipSuccess) {
            c->prof_ms[c->prof_phase[s]] += ms;
            c->prof_n[c->prof_phase[s]] += 1;
        }
    }
    c->prof_used = 0;
}

// Rank bits of the packed (key, rank) form: what the largest cell key leaves of 32.
int32_t rank_bits(int64_t n_cells) {
    int kb = 1;
    while (kb < 31 && ((int64_t)1 << kb) < n_cells) ++kb;
    return 32 - kb;
}

bool aligned16(const void *q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

sph_status parts_of(const sph_ctx *ctx, const sph_particles *p, Parts &out) {
    if (!p || !p->pos[0] || !p->pos[1] || (ctx->dim == 3 && !p->pos[2]) || !p->label || !p->id || !p->n_dev)
        return SPH_ERR_ARG;
    if (p->n_carried < 0 || p->n_carried > SPH_MAX_CARRIED) return SPH_ERR_ARG;
    if (p->capacity <= 0 || p->capacity > ctx->capacity) return SPH_ERR_ARG;
    for (int f = 0; f < p->n_carried; ++f)
        if (!p->carried[f]) return SPH_ERR_ARG;
    std::memset(&out, 0, sizeof(out));
    for (int c = 0; c < 3; ++c) out.pos[c] = p->pos[c];
    if (ctx->dim == 2) out.pos[2] = nullptr;
    for (int f = 0; f < p->n_carried; ++f) out.car[f] = p->carried[f];
    out.nc = p->n_carried;
    out.dim = ctx->dim;
    out.label = p->label;
    out.id = p->id;
    out.n_dev = p->n_dev;
    out.capacity = p->capacity;
    return SPH_OK;
}

Grid grid_of(const sph_ctx *ctx) {
    Grid g{};
    for (int c = 0; c < 3; ++c) {
        g.lo[c] = (float)ctx->lo[c];
        g.dims[c] = ctx->dims[c];
        g.bdims[c] = ctx->bdims[c];
    }
    g.inv_cs = (float)(1.0 / ctx->cs);
    g.dim = ctx->dim;
    g.blog2 = ctx->blog2;
    g.brick_slot = ctx->d_brick_slot;
    g.overflow_key = (uint32_t)(ctx->n_cells - 1);
    return g;
}

EventArgs events_of(const sph_ctx *ctx) {
    EventArgs e{};
    e.ctl = ctx->d_ctl;
    e.gen_idx = ctx->d_gen_idx;
    e.gen_new = ctx->d_gen_new;
    e.dup = ctx->d_dup;
    e.del_idx = ctx->d_del_idx;
    e.rel = ctx->d_rel;
    e.cap_ev = ctx->max_events;
    e.cap_rel = ctx->max_events * kRelPerEvent;
    e.part = ctx->d_part;
    e.rho_field = ctx->fields.rho;
    return e;
}

// Buckets of the bucketed build: the fewest cells per bucket (a power of two) that
// keep the buckets within kMaxBuckets; grids beyond kMaxBuckets * kMaxBucketCells
// cells take the three-kernel counting sort.
void bk_layout(sph_ctx *c) {
    c->bk = c->n_cells >= 1 && c->n_cells <= (int64_t)kMaxBuckets * kMaxBucketCells;
    c->bshift = 0;
    while (((c->n_cells + (int64_t(1) << c->bshift) - 1) >> c->bshift) > kMaxBuckets) ++c->bshift;
    c->nbk = (int)((c->n_cells + (int64_t(1) << c->bshift) - 1) >> c->bshift);
    // a new grid: the build times start over (the events in flight are still read)
    c->bt.samples[0] = c->bt.samples[1] = 0;
    c->bt.est[0] = c->bt.est[1] = 0.0;
}

// Workgroups of k_bk_count for a particle array of this capacity (a multiple of 8).
int bk_blocks(int64_t capacity) {
    const int64_t want = (capacity + kBkPer - 1) / kBkPer;
    return (int)std::max<int64_t>(8, (want + 7) / 8 * 8);
}

// Count workgroups for a particle array of this capacity (a multiple of 8, so the
// XCD renumbering applies).
int count_blocks(int64_t capacity) {
    const int64_t want = (capacity + kCountPer - 1) / kCountPer;
    return (int)std::max<int64_t>(8, std::min<int64_t>(16384, (want + 7) / 8 * 8));
}

// Arguments of the counting build's count pass (cand: with the merged step's
// candidate list).
CountArgs count_args(const sph_ctx *ctx, const Parts &pp, bool cand = false) {
    CountArgs ca{};
    ca.x = pp.pos[0];
    ca.y = pp.pos[1];
    ca.z = pp.pos[2];
    ca.n_dev = pp.n_dev;
    ca.capacity = pp.capacity;
    ca.g = grid_of(ctx);
    ca.count = ctx->d_count;
    ca.packed = ctx->d_keys;
    ca.spill = ctx->d_keyrank;
    ca.rbits = ctx->rbits;
    ca.tile_state = ctx->d_tile_state;
    ca.n_tiles = ctx->n_tiles;
    ca.ctl = ctx->d_ctl;
    ca.nonfinite = cand ? &ctx->d_ctl->nonfinite_full : &ctx->d_ctl->nonfinite_build;
    if (cand) {
        ca.c.cover = ctx->d_cover;
        ca.c.bufs = ctx->d_bufs;
        ca.c.nb = ctx->nb;
        ca.c.cand = ctx->d_cand;
        ca.c.cap_cand = ctx->capacity + kCandSlack;
    }
    return ca;
}

ScanArgs scan_args(const sph_ctx *ctx) {
    ScanArgs sa{};
    sa.count = ctx->d_count;
    sa.cell_start = ctx->d_cell_start;
    sa.m = ctx->n_cells + 1;
    sa.tile_state = ctx->d_tile_state;
    sa.ctl = ctx->d_ctl;
    return sa;
}

ScatterArgs scatter_args(const sph_ctx *ctx, int64_t capacity) {
    ScatterArgs xa{};
    xa.n_dev = &ctx->d_ctl->n_built;  // the particles the count pass saw, whatever an update did since
    xa.capacity = capacity;
    xa.ctl = ctx->d_ctl;
    xa.packed = ctx->d_keys;
    xa.spill = ctx->d_keyrank;
    xa.rbits = ctx->rbits;
    xa.cell_start = ctx->d_cell_start;
    xa.cell_idx = ctx->d_cell_idx;
    return xa;
}

LocalArgs local_args(const sph_ctx *ctx, const Parts &pp) {
    LocalArgs la{};
    la.p = pp;
    la.bufs = ctx->d_bufs;
    la.nb = ctx->nb;
    la.run_first = ctx->d_run_first;
    la.run_len = ctx->d_run_len;
    la.run_buf = ctx->d_run_buf;
    la.cell_start = ctx->d_cell_start;
    la.cell_idx = ctx->d_cell_idx;
    la.e = events_of(ctx);
    la.rpb = kRunsPerBlock;
    return la;
}

FinArgs fin_args(const sph_ctx *ctx, const Parts &pp, bool local) {
    FinArgs f{};
    f.p = pp;
    f.local = local ? 1 : 0;
    f.nf_full = local ? 0 : 1;
    f.nb = ctx->nb;
    f.e = events_of(ctx);
    f.gen_sorted = ctx->d_gen_sorted;
    f.del_sorted = ctx->d_del_sorted;
    f.result = ctx->d_result;
    return f;
}

sph_status launch_finalize(sph_ctx *ctx, const Parts &pp, bool local, int n_part) {
    (void)n_part;
    FinArgs f = fin_args(ctx, pp, local);
    if (local && ctx->nf_full_next) f.nf_full = 1;  // a merged build raised its flag there
    ctx->nf_full_next = false;
    {
        ProfScope ps(ctx, SPH_PHASE_FINALIZE);
        hipLaunchKernelGGL(k_finalize, dim3(kFinBlocksMax), dim3(kFinBlock), 0, ctx->stream, f);
    }
    HIP_TRY(hipGetLastError());
    ctx->any_update = true;
    return SPH_OK;
}

// Arguments of the bucketed build; the count pass reads the particles of pp
// (cand: with the merged step's candidate list), the scatter and the sort only
// the context's arrays.
BkArgs bk_args(const sph_ctx *ctx, const Parts *pp, bool cand) {
    BkArgs a{};
    if (pp) {
        a.x = pp->pos[0];
        a.y = pp->pos[1];
        a.z = pp->pos[2];
        a.n_dev = pp->n_dev;
    }
    a.capacity = ctx->built_capacity;
    a.g = grid_of(ctx);
    a.bshift = ctx->bshift;
    a.nbk = ctx->nbk;
    a.n_cells = ctx->n_cells;
    a.bk_count = ctx->d_bk_count;
    a.bk_start = ctx->d_bk_start;
    a.ent = ctx->d_ent;
    a.tmp = ctx->d_tmp;
    a.cell_start = ctx->d_cell_start;
    a.cell_idx = ctx->d_cell_idx;
    a.ctl = ctx->d_ctl;
    a.nonfinite = cand ? &ctx->d_ctl->nonfinite_full : &ctx->d_ctl->nonfinite_build;
    if (cand) {
        a.cover = ctx->d_cover;
        a.bufs = ctx->d_bufs;
        a.nb = ctx->nb;
        a.cand = ctx->d_cand;
        a.cap_cand = ctx->capacity + kCandSlack;
    }
    return a;
}

// The candidate list's exact tests (full scan, merged step).
FullArgs cand_args(const sph_ctx *ctx, const Parts &pp) {
    FullArgs fa{};
    fa.p = pp;
    fa.bufs = ctx->d_bufs;
    fa.nb = ctx->nb;
    fa.e = events_of(ctx);
    fa.vec = aligned16(pp.pos[0]) && aligned16(pp.pos[1]) && aligned16(pp.pos[2]) ? 1 : 0;
    fa.cand = ctx->d_cand;
    fa.cap_cand = ctx->capacity + kCandSlack;
    return fa;
}

// Bucketed build after its count pass: the bucket scatter, then the bucket sort
// (fa: the merged step's candidates are classified beside the scatter).
sph_status bk_cells(sph_ctx *c, const FullArgs *fa) {
    const BkArgs ba = bk_args(c, nullptr, false);
    {
        ProfScope ps(c, SPH_PHASE_SCATTER);
        if (fa)
            hipLaunchKernelGGL(k_bk_scatter_cls, dim3(kCandBlocksMerged + c->build_blocks), dim3(kBkBlock), 0,
                               c->stream, ba, *fa, kCandBlocksMerged);
        else
            hipLaunchKernelGGL(k_bk_scatter, dim3(c->build_blocks), dim3(kBkBlock), 0, c->stream, ba);
    }
    HIP_TRY(hipGetLastError());
    {
        ProfScope ps(c, SPH_PHASE_SORT);
        hipLaunchKernelGGL(k_bk_sort, dim3(c->nbk), dim3(kSortBlock), 0, c->stream, ba);
    }
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

// Counting build after its count pass: the look-back scan, then the scatter (fa:
// the merged step's candidates are classified beside it).
sph_status count_cells(sph_ctx *c, const FullArgs *fa) {
    const ScanArgs sa = scan_args(c);
    {
        ProfScope ps(c, SPH_PHASE_SCAN);
        hipLaunchKernelGGL(k_scan, dim3((unsigned)c->n_tiles), dim3(kScanBlock), 0, c->stream, sa);
    }
    HIP_TRY(hipGetLastError());
    const ScatterArgs xa = scatter_args(c, c->built_capacity);
    {
        ProfScope ps(c, SPH_PHASE_SCATTER);
        if (fa)
            hipLaunchKernelGGL(k_scatter_cls, dim3(kCandBlocksMerged + c->build_blocks), dim3(kBuildBlock), 0,
                               c->stream, xa, *fa, kCandBlocksMerged);
        else
            hipLaunchKernelGGL(k_scatter, dim3(c->build_blocks), dim3(kBuildBlock), 0, c->stream, xa);
    }
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

// Timer events of the build method choice (created with an automatic context, so
// that builds allocate nothing).
bool timers_ready(sph_ctx *c) {
    BuildTimer &t = c->bt;
    if (!t.init) {
        t.init = true;
        t.ok = true;
        for (auto &set : t.ev)
            for (hipEvent_t &e : set)
                if (hipEventCreate(&e) != hipSuccess) {
                    e = nullptr;
                    t.ok = false;
                }
        (void)hipGetLastError();
    }
    return t.ok;
}

void timers_free(sph_ctx *c) {
    for (auto &set : c->bt.ev)
        for (hipEvent_t e : set)
            if (e) (void)hipEventDestroy(e);
}

// Timings whose events have completed into the estimates (never waits).
void timers_harvest(sph_ctx *c) {
    BuildTimer &t = c->bt;
    for (int s = 0; s < kTimerSets; ++s) {
        if (!t.busy[s]) continue;
        if (!t.cells_done[s]) {  // its build ended early (an error): nothing to read
            if (s != c->tset) t.busy[s] = false;
            continue;
        }
        const hipError_t q = hipEventQuery(t.ev[s][3]);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();  // not an error of any call
            continue;
        }
        t.busy[s] = false;
        float a = 0.0f, b = 0.0f;
        if (q != hipSuccess || hipEventElapsedTime(&a, t.ev[s][0], t.ev[s][1]) != hipSuccess ||
            hipEventElapsedTime(&b, t.ev[s][2], t.ev[s][3]) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        const double us = 1e3 * ((double)a + (double)b);
        const int m = t.meth[s];
        t.last[m][t.samples[m] % 3] = us;
        ++t.samples[m];
        const double *v = t.last[m];
        if (t.samples[m] == 1)
            t.est[m] = v[0];
        else if (t.samples[m] == 2)
            t.est[m] = std::min(v[0], v[1]);
        else
            t.est[m] = std::max(std::min(v[0], v[1]), std::min(std::max(v[0], v[1]), v[2]));
    }
    if (t.samples[0] >= kExploreSamples && t.samples[1] >= kExploreSamples) {
        const int o = 1 - t.cur;
        if (t.est[o] < 0.97 * t.est[t.cur]) t.cur = o;
    }
}

// The next build's method; sets c->tset when it is to be timed.
int pick_method(sph_ctx *c) {
    c->tset = -1;
    if (!c->bk || c->build_pref == SPH_BUILD_COUNTING) return kMethCounting;
    if (c->build_pref == SPH_BUILD_BUCKETED) return kMethBucketed;
    BuildTimer &t = c->bt;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return t.cur;  // no events inside a captured graph
    }
    if (!timers_ready(c)) return kMethBucketed;
    timers_harvest(c);
    const int64_t b = t.builds++;
    int m = t.cur;
    bool timed = false;
    if (b < 2) {
        m = (int)b;  // warm-up: one untimed build of each
    } else if (t.samples[0] < kExploreSamples || t.samples[1] < kExploreSamples) {
        m = (int)(b & 1);
        timed = true;
    } else {
        const int64_t k = b % kReprobe;
        m = k == kReprobe - 1 ? 1 - t.cur : t.cur;
        timed = k >= kReprobe - 2;
    }
    for (int s = 0; timed && s < kTimerSets; ++s) {
        if (t.busy[s]) continue;
        t.busy[s] = true;
        t.cells_done[s] = false;
        t.meth[s] = m;
        c->tset = s;
        break;
    }
    return m;
}

// Timer event k (0, 1: around the count pass; 2, 3: around the cells pass) of a
// timed build.
void tmark(sph_ctx *c, int k) {
    if (c->tset < 0) return;
    BuildTimer &t = c->bt;
    if (hipEventRecord(t.ev[c->tset][k], c->stream) != hipSuccess) {
        (void)hipGetLastError();
        t.busy[c->tset] = false;
        c->tset = -1;
        return;
    }
    if (k == 3) {
        t.cells_done[c->tset] = true;
        c->tset = -1;
    }
}

// The cells pass of the latest build (after its count pass), by its method.
sph_status build_cells(sph_ctx *c, const FullArgs *fa) {
    tmark(c, 2);
    HIP_CHECKED(c->meth == kMethBucketed ? bk_cells(c, fa) : count_cells(c, fa));
    tmark(c, 3);
    return SPH_OK;
}

// Merged step: enqueue the cells pass a merged build left for its update (every
// call that reads the cell list needs it first).
sph_status merged_cells(sph_ctx *c) {
    if (!c->scan_pending) return SPH_OK;
    c->scan_pending = false;
    return build_cells(c, nullptr);
}

// Merged step: drop the events of a merged build once a call changes what they were
// decided on (the update then walks the cover cells instead), or before a new build
// or a full scan fills the event lists again (rebuild: its non-finite flag too).
sph_status merged_drop(sph_ctx *c, bool rebuild) {
    HIP_CHECKED(merged_cells(c));
    // a merged build's non-finite flag no finalize consumed (its events may have
    // been dropped earlier) must not reach the next build's or full scan's finalize
    const bool clear_nf = rebuild && c->nf_full_next;
    if (rebuild) c->nf_full_next = false;
    if (!c->ev_pending && !clear_nf) return SPH_OK;
    hipLaunchKernelGGL(k_reset_events, dim3(1), dim3(256), 0, c->stream, c->d_ctl, c->d_part, clear_nf ? 1 : 0);
    HIP_TRY(hipGetLastError());
    c->ev_pending = false;
    return SPH_OK;
}

sph_status wait_result(sph_ctx *ctx) {
    HIP_TRY(hipMemcpyAsync(ctx->h_result, ctx->d_result, sizeof(sph_result), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SPH_OK;
}

void free_ctx(sph_ctx *c) {
    if (!c) return;
    (void)hipFree(c->d_bufs);
    (void)hipFree(c->d_run_first);
    (void)hipFree(c->d_run_len);
    (void)hipFree(c->d_run_buf);
    (void)hipFree(c->d_src_first);
    (void)hipFree(c->d_src_len);
    (void)hipFree(c->d_row_lo);
    (void)hipFree(c->d_row_hi);
    (void)hipFree(c->d_count);
    (void)hipFree(c->d_brick_slot);
    (void)hipFree(c->d_cell_start);
    (void)hipFree(c->d_cell_idx);
    (void)hipFree(c->d_keyrank);
    (void)hipFree(c->d_keys);
    (void)hipFree(c->d_cand);
    (void)hipFree(c->d_cover);
    (void)hipFree(c->d_bk_count);
    (void)hipFree(c->d_bk_start);
    (void)hipFree(c->d_ent);
    (void)hipFree(c->d_tmp);
    (void)hipFree(c->d_tile_state);
    (void)hipFree(c->d_gen_idx);
    (void)hipFree(c->d_del_idx);
    (void)hipFree(c->d_gen_sorted);
    (void)hipFree(c->d_del_sorted);
    (void)hipFree(c->d_gen_new);
    (void)hipFree(c->d_rel);
    (void)hipFree(c->d_dup);
    (void)hipFree(c->d_ctl);
    (void)hipFree(c->d_part);
    (void)hipFree(c->d_bcfound);
    if (c->h_bc_status) (void)hipHostFree(c->h_bc_status);
    (void)hipFree(c->d_result);
    if (c->h_result) (void)hipHostFree(c->h_result);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    timers_free(c);
    delete c;
}

}  // namespace

// Device record of one buffer's frame: FP64 and FP32 forms of the rotation,
// hi/lo split of the origin, thresholds, guard band, bounding sphere, recycle
// shift.  Boundary-condition members are zero (none).
static BufDev frame_record(const sph_ctx *ctx, int kind, const double o[3], const double q[9], const double h[3],
                           double margin) {
    const int dim = ctx->dim;
    BufDev b{};
    for (int i = 0; i < 9; ++i) {
        b.q[i] = q[i];
        b.qf[i] = (float)q[i];
    }
    for (int c = 0; c < 3; ++c) {
        b.o[c] = o[c];
        b.ohi[c] = (float)o[c];
        b.olo[c] = (float)(o[c] - (double)b.ohi[c]);
        b.thr[c] = h[c];
        b.thr[3 + c] = h[c] + margin;
        b.thrf[c] = (float)b.thr[c];
        b.thrf[3 + c] = (float)b.thr[3 + c];
    }
    const double a = 2.0 * h[0];
    for (int c = 0; c < 3; ++c) b.shift[c] = c < dim ? a * q[c] : 0.0;
    b.guard = (float)sphbuf::guard_band(dim, o, h, margin, ctx->cs, ctx->dp);
    const double R = sphbuf::sphere_radius(dim, h, margin);
    b.rsq = (float)(R * R);
    // x - O' = Q^T r': a member's global offset along axis g is below
    // sum_i |Q_ig| (h_i + margin); the guard band and a relative 1e-6 on top
    for (int g = 0; g < 3; ++g) {
        if (g >= dim) {
            b.bmin[g] = -INFINITY;
            b.bmax[g] = INFINITY;
            continue;
        }
        double ext = 0.0;
        for (int i = 0; i < dim; ++i) ext += std::fabs(q[3 * i + g]) * (h[i] + margin);
        ext = (ext + dim * (double)b.guard) * (1.0 + 1e-6);
        b.bmin[g] = std::nextafter((float)(o[g] - ext), -INFINITY);
        b.bmax[g] = std::nextafter((float)(o[g] + ext), INFINITY);
    }
    b.kind = (int32_t)kind;
    return b;
}

// Copy the boundary-condition members of one record into another.
static void copy_bc(BufDev &dst, const BufDev &src) {
    dst.bc_kind = src.bc_kind;
    dst.profile = src.profile;
    dst.rho_rec = src.rho_rec;
    dst.bc_u = src.bc_u;
    dst.bc_radius = src.bc_radius;
}

// Candidate cells of one check region as runs of consecutive cell keys, at most
// a wave's worth of candidates per run (one wave takes one run).  For the
// brick-sparse grid the dense cover is mapped to keys and the overflow cell is
// added whenever part of the region lies in inactive bricks.
static sph_status cover_runs(const sph_ctx *ctx, const double o[3], const double q[9], const double h[3],
                             double margin, std::vector<int32_t> &first, std::vector<int32_t> &len) {
    first.clear();
    len.clear();
    std::vector<int32_t> f0, l0;
    const sph_status cs = sphbuf::grid_cover(ctx->dim, ctx->lo, ctx->cs, ctx->dims, o, q, h, margin, f0, l0);
    if (cs != SPH_OK) return cs;
    const int cap = ctx->dim == 3 ? 4 : 12;
    if (ctx->blog2 == 0) {
        for (size_t r = 0; r < f0.size(); ++r)
            for (int s = 0; s < l0[r]; s += cap) {
                first.push_back(f0[r] + s);
                len.push_back(std::min(cap, l0[r] - s));
            }
        return SPH_OK;
    }
    const int b = ctx->blog2, m = (1 << b) - 1;
    std::vector<int64_t> keys;
    bool overflow = false;
    for (size_t r = 0; r < f0.size(); ++r)
        for (int s = 0; s < l0[r]; ++s) {
            const int64_t lin = (int64_t)f0[r] + s;
            const int64_t ix = lin % ctx->dims[0], iy = (lin / ctx->dims[0]) % ctx->dims[1],
                          iz = lin / ((int64_t)ctx->dims[0] * ctx->dims[1]);
            const int64_t brick = (ix >> b) + (int64_t)ctx->bdims[0] * ((iy >> b) + (int64_t)ctx->bdims[1] * (iz >> b));
            const int32_t slot = ctx->h_brick_slot[(size_t)brick];
            if (slot < 0) {
                overflow = true;
                continue;
            }
            const int64_t local = (ix & m) + ((iy & m) << b) + (ctx->dim == 3 ? ((iz & m) << (2 * b)) : 0);
            keys.push_back(((int64_t)slot << (ctx->dim * b)) + local);
        }
    if (overflow) keys.push_back(ctx->n_cells - 1);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (size_t i = 0; i < keys.size();) {
        size_t j = i + 1;
        while (j < keys.size() && keys[j] == keys[j - 1] + 1 && (int)(j - i) < cap) ++j;
        first.push_back((int32_t)keys[i]);
        len.push_back((int32_t)(j - i));
        i = j;
    }
    return SPH_OK;
}

// Cells of a run at most (a wave of the classify takes a few runs).
static int run_cap(const sph_ctx *ctx) { return ctx->dim == 3 ? 4 : 12; }

// Size of a buffer's run range: its cover in any orientation.  The check box lies
// in the sphere of radius R around its origin, so in at most n = 2 (R + eps) / cs
// + 4 cells per axis, n^(d-1) rows of at most n + 1 runs each, plus the overflow
// cell of a brick-sparse grid.
static void run_range(const sph_ctx *ctx, const double h[3], double margin, int32_t &rmax, int64_t &rows) {
    const double R = sphbuf::sphere_radius(ctx->dim, h, margin);
    const double err = sphbuf::binning_error_cells(ctx->dim, ctx->lo, ctx->cs, ctx->dims);
    const double eps = std::max(1e-2, 1.5 * err) * ctx->cs;
    const int64_t n = (int64_t)std::ceil(2.0 * (R + eps) / ctx->cs) + 4;
    rows = ctx->dim == 3 ? n * n : n;
    rmax = (int32_t)std::min<int64_t>(rows * (n + 1) + 1, (int64_t)1 << 30);
}

static CoverArgs cover_args(const sph_ctx *ctx) {
    CoverArgs a{};
    a.ctl = ctx->d_ctl;
    a.dim = ctx->dim;
    a.nb = ctx->nb;
    a.cap = run_cap(ctx);
    for (int k = 0; k < SPH_MAX_BUFFERS; ++k) {
        a.rbase[k] = ctx->rbase[k];
        a.rmax[k] = ctx->rmax[k];
    }
    a.src_first = ctx->d_src_first;
    a.src_len = ctx->d_src_len;
    a.run_first = ctx->d_run_first;
    a.run_len = ctx->d_run_len;
    a.run_buf = ctx->d_run_buf;
    a.cover = ctx->merged ? reinterpret_cast<unsigned *>(ctx->d_cover) : nullptr;
    a.g = grid_of(ctx);
    for (int c = 0; c < 3; ++c) {
        a.glo[c] = ctx->lo[c];
        a.dims[c] = ctx->dims[c];
    }
    a.cs = ctx->cs;
    a.row_lo = ctx->d_row_lo;
    a.row_hi = ctx->d_row_hi;
    a.max_rows = ctx->max_rows;
    return a;
}

// Grow the per-buffer run ranges and the compact list to hold buffer k's range
// (setup: allocates, copies the other buffers' runs over).
static sph_status grow_ranges(sph_ctx *ctx, int k, int32_t rmax, int64_t rows) {
    const int64_t cap = ctx->src_cap + rmax;
    int32_t *sf = nullptr, *sl = nullptr, *rf = nullptr, *rl = nullptr, *lo = nullptr, *hi = nullptr;
    uint8_t *rb = nullptr;
    const int64_t mr = std::max(ctx->max_rows, rows);
    bool ok = hipMalloc(&sf, sizeof(int32_t) * cap) == hipSuccess && hipMalloc(&sl, sizeof(int32_t) * cap) == hipSuccess &&
              hipMalloc(&rf, sizeof(int32_t) * cap) == hipSuccess && hipMalloc(&rl, sizeof(int32_t) * cap) == hipSuccess &&
              hipMalloc(&rb, (size_t)cap) == hipSuccess && hipMalloc(&lo, sizeof(int32_t) * mr) == hipSuccess &&
              hipMalloc(&hi, sizeof(int32_t) * mr) == hipSuccess;
    if (ok && ctx->src_cap > 0)
        ok = hipMemcpyAsync(sf, ctx->d_src_first, sizeof(int32_t) * ctx->src_cap, hipMemcpyDeviceToDevice,
                            ctx->stream) == hipSuccess &&
             hipMemcpyAsync(sl, ctx->d_src_len, sizeof(int32_t) * ctx->src_cap, hipMemcpyDeviceToDevice,
                            ctx->stream) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(ctx->stream) == hipSuccess;
    if (!ok) {
        for (void *q : {(void *)sf, (void *)sl, (void *)rf, (void *)rl, (void *)rb, (void *)lo, (void *)hi})
            (void)hipFree(q);
        return SPH_ERR_HIP;
    }
    for (void *q : {(void *)ctx->d_src_first, (void *)ctx->d_src_len, (void *)ctx->d_run_first,
                    (void *)ctx->d_run_len, (void *)ctx->d_run_buf, (void *)ctx->d_row_lo, (void *)ctx->d_row_hi})
        (void)hipFree(q);
    ctx->d_src_first = sf;
    ctx->d_src_len = sl;
    ctx->d_run_first = rf;
    ctx->d_run_len = rl;
    ctx->d_run_buf = rb;
    ctx->d_row_lo = lo;
    ctx->d_row_hi = hi;
    ctx->rbase[k] = (int32_t)ctx->src_cap;
    ctx->rmax[k] = rmax;
    ctx->src_cap = cap;
    ctx->max_rows = mr;
    ctx->layout_gen++;
    return SPH_OK;
}

// Install host-computed runs of the given buffers into their ranges, rebuild the
// compact list and the per-cell cover mask (setup: waits for the stream).
static sph_status install_runs(sph_ctx *ctx, const std::vector<int> &which,
                               const std::vector<std::vector<int32_t>> &first,
                               const std::vector<std::vector<int32_t>> &len) {
    for (size_t w = 0; w < which.size(); ++w) {
        const int k = which[w];
        const size_t nr = first[w].size();
        if ((int64_t)nr > ctx->rmax[k]) return SPH_ERR_ARG;  // cannot happen: the range holds any orientation
        if (nr > 0) {
            HIP_TRY(hipMemcpyAsync(ctx->d_src_first + ctx->rbase[k], first[w].data(), sizeof(int32_t) * nr,
                                   hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(ctx->d_src_len + ctx->rbase[k], len[w].data(), sizeof(int32_t) * nr,
                                   hipMemcpyHostToDevice, ctx->stream));
        }
        ctx->hcnt[k] = (int32_t)nr;
    }
    HIP_TRY(hipMemcpyAsync(ctx->d_ctl->run_cnt, ctx->hcnt, sizeof(int32_t) * SPH_MAX_BUFFERS, hipMemcpyHostToDevice,
                           ctx->stream));
    // the cover mask of the merged step (two 16-bit cells per word)
    if (ctx->merged) {
        const int64_t words = (ctx->n_cells + 1) / 2;
        if (ctx->cover_cells != ctx->n_cells) {
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            (void)hipFree(ctx->d_cover);
            ctx->d_cover = nullptr;
            ctx->cover_cells = 0;
            HIP_TRY(hipMalloc(&ctx->d_cover, sizeof(uint32_t) * (size_t)words));
            ctx->cover_cells = ctx->n_cells;
        }
        HIP_TRY(hipMemsetAsync(ctx->d_cover, 0, sizeof(uint32_t) * (size_t)words, ctx->stream));
    }
    CoverArgs a = cover_args(ctx);
    hipLaunchKernelGGL(k_runs_assemble, dim3(1), dim3(kCoverBlock), 0, ctx->stream, a);
    HIP_TRY(hipGetLastError());
    int64_t total = 0;
    for (int k = 0; k < ctx->nb; ++k) total += ctx->hcnt[k];
    if (ctx->merged && total > 0) {
        const int blocks = (int)std::min<int64_t>(1024, (total + 255) / 256);
        hipLaunchKernelGGL(k_mask_set, dim3(blocks), dim3(256), 0, ctx->stream, a);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->n_runs = (int)total;
    ctx->built = false;  // covers changed: the next update needs a build with them
    return SPH_OK;
}

extern "C" sph_status sph_create(const sph_config *cfg, sph_ctx **out) {
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    if (!cfg || (cfg->dim != 2 && cfg->dim != 3)) return SPH_ERR_ARG;
    if (!(cfg->cell_size > 0.0) || !std::isfinite(cfg->cell_size) || !(cfg->dp > 0.0)) return SPH_ERR_ARG;
    if (cfg->capacity <= 0 || cfg->capacity >= (int64_t(1) << 31)) return SPH_ERR_ARG;
    if (cfg->max_events < 1 || cfg->max_events > SPH_MAX_EVENTS_LIMIT) return SPH_ERR_ARG;
    int32_t dims[3] = {1, 1, 1};
    double cells = 1.0;
    for (int c = 0; c < cfg->dim; ++c) {
        if (!std::isfinite(cfg->lo[c]) || !std::isfinite(cfg->hi[c]) || !(cfg->hi[c] > cfg->lo[c])) return SPH_ERR_ARG;
        const double n = std::ceil((cfg->hi[c] - cfg->lo[c]) / cfg->cell_size);
        if (n > (double)(1 << 24)) return SPH_ERR_ARG;
        dims[c] = (int32_t)std::max(1.0, n);
        cells *= dims[c];
    }
    if (cfg->brick_log2 < 0 || cfg->brick_log2 > 5 || cfg->brick_margin < 0 || cfg->brick_margin > 64)
        return SPH_ERR_ARG;
    const int blog2 = cfg->brick_log2;
    int32_t bdims[3] = {1, 1, 1};
    double bricks = 1.0;
    if (blog2 > 0) {
        for (int c = 0; c < cfg->dim; ++c) {
            bdims[c] = (dims[c] + (1 << blog2) - 1) >> blog2;
            bricks *= bdims[c];
        }
        if (bricks >= 2147483000.0) return SPH_ERR_ARG;
        cells = 1.0;  // only the overflow cell until sph_grid_fit activates bricks
    } else if (cells >= 2147483000.0) {
        return SPH_ERR_ARG;
    }
    if (cfg->update_path != SPH_UPDATE_MERGED && cfg->update_path != SPH_UPDATE_CELLS) return SPH_ERR_ARG;
    if (cfg->build_method < SPH_BUILD_AUTO || cfg->build_method > SPH_BUILD_BUCKETED) return SPH_ERR_ARG;
    {   // FP32 binning must place every particle within a quarter cell of its cell
        double glo[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < cfg->dim; ++c) glo[c] = cfg->lo[c];
        if (!(sphbuf::binning_error_cells(cfg->dim, glo, cfg->cell_size, dims) < sphbuf::kMaxBinningError))
            return SPH_ERR_ARG;
    }

    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_ERR_HIP;
    c->dim = cfg->dim;
    for (int q = 0; q < 3; ++q) {
        c->lo[q] = q < cfg->dim ? cfg->lo[q] : 0.0;
        c->dims[q] = dims[q];
    }
    c->cs = cfg->cell_size;
    c->dp = cfg->dp;
    c->n_cells = (int64_t)cells;
    bk_layout(c);
    c->rbits = rank_bits(c->n_cells);
    c->blog2 = blog2;
    c->bmargin = cfg->brick_margin;
    for (int q = 0; q < 3; ++q) c->bdims[q] = bdims[q];
    c->n_bricks = blog2 > 0 ? (int64_t)bricks : 0;
    if (blog2 > 0) c->h_brick_slot.assign((size_t)c->n_bricks, -1);
    c->capacity = cfg->capacity;
    c->max_events = (unsigned)cfg->max_events;
    c->stream = (hipStream_t)cfg->stream;
    c->merged = cfg->update_path == SPH_UPDATE_MERGED;
    c->build_pref = cfg->build_method;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return SPH_ERR_HIP;
    }
    // grid sizes: a multiple of 8 blocks (XCD renumbering), enough to fill 256 CUs
    const int64_t want = (cfg->capacity + kBuildBlock - 1) / kBuildBlock;
    c->build_blocks = (int)std::max<int64_t>(8, std::min<int64_t>(8192, (want + 7) / 8 * 8));
    c->full_blocks = std::min(c->build_blocks, kMaxPartBlocks);
    const int64_t m = c->n_cells + 1;
    c->n_tiles = (m + kScanTile - 1) / kScanTile;
    const size_t ev = c->max_events;
    bool ok = hipMalloc(&c->d_bufs, sizeof(BufDev) * SPH_MAX_BUFFERS) == hipSuccess &&
              hipMalloc(&c->d_count, sizeof(int32_t) * m) == hipSuccess &&
              hipMalloc(&c->d_cell_start, sizeof(int32_t) * (m + 1)) == hipSuccess &&
              hipMalloc(&c->d_cell_idx, sizeof(int32_t) * c->capacity) == hipSuccess &&
              hipMalloc(&c->d_keyrank, sizeof(unsigned long long) * c->capacity) == hipSuccess &&
              hipMalloc(&c->d_keys, sizeof(uint32_t) * c->capacity) == hipSuccess &&
              hipMalloc(&c->d_cand, sizeof(unsigned long long) * (c->capacity + kCandSlack)) == hipSuccess &&
              hipMalloc(&c->d_tile_state, sizeof(unsigned long long) * c->n_tiles) == hipSuccess &&
              hipMalloc(&c->d_gen_idx, sizeof(uint32_t) * ev * kSeg) == hipSuccess &&
              hipMalloc(&c->d_del_idx, sizeof(uint32_t) * ev * kSeg) == hipSuccess &&
              hipMalloc(&c->d_gen_sorted, sizeof(uint32_t) * ev) == hipSuccess &&
              hipMalloc(&c->d_del_sorted, sizeof(uint32_t) * ev) == hipSuccess &&
              hipMalloc(&c->d_gen_new, sizeof(float) * ev * kSeg * 4) == hipSuccess &&
              hipMalloc(&c->d_rel, sizeof(unsigned long long) * ev * kSeg * kRelPerEvent) == hipSuccess &&
              hipMalloc(&c->d_dup, sizeof(float) * ev * kSeg * (3 + SPH_MAX_CARRIED)) == hipSuccess &&
              hipMalloc(&c->d_ctl, sizeof(Ctl)) == hipSuccess &&
              (blog2 == 0 || hipMalloc(&c->d_brick_slot, sizeof(int32_t) * c->n_bricks) == hipSuccess) &&
              hipMalloc(&c->d_part, sizeof(unsigned) * 2 * SPH_MAX_BUFFERS * kMaxPartBlocks) == hipSuccess &&
              hipMalloc(&c->d_result, sizeof(sph_result)) == hipSuccess &&
              hipMalloc(&c->d_bk_count, sizeof(uint32_t) * kMaxBuckets) == hipSuccess &&
              hipMalloc(&c->d_bk_start, sizeof(uint32_t) * (kMaxBuckets + 1)) == hipSuccess &&
              hipMalloc(&c->d_ent, sizeof(uint2) * c->capacity) == hipSuccess &&
              hipMalloc(&c->d_tmp, sizeof(uint2) * c->capacity) == hipSuccess &&
              hipMalloc(&c->d_bcfound, sizeof(unsigned) * kCountReplicas * SPH_MAX_BUFFERS) == hipSuccess &&
              hipHostMalloc(&c->h_bc_status, sizeof(unsigned), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&c->h_result, sizeof(sph_result), hipHostMallocDefault) == hipSuccess;
    if (ok) {
        Ctl init{};
        init.next_id = cfg->next_id;
        sph_result r0{};
        ok = hipMemsetAsync(c->d_count, 0, sizeof(int32_t) * m, c->stream) == hipSuccess &&
             hipMemsetAsync(c->d_cell_start, 0, sizeof(int32_t) * (m + 1), c->stream) == hipSuccess &&
             hipMemsetAsync(c->d_tile_state, 0, sizeof(unsigned long long) * c->n_tiles, c->stream) == hipSuccess &&
             hipMemsetAsync(c->d_part, 0, sizeof(unsigned) * 2 * SPH_MAX_BUFFERS * kMaxPartBlocks, c->stream) ==
                 hipSuccess &&
             hipMemcpyAsync(c->d_ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
             hipMemsetAsync(c->d_bcfound, 0, sizeof(unsigned) * kCountReplicas * SPH_MAX_BUFFERS, c->stream) ==
                 hipSuccess &&
             hipMemsetAsync(c->d_bk_count, 0, sizeof(uint32_t) * kMaxBuckets, c->stream) == hipSuccess &&
             (blog2 == 0 || hipMemsetAsync(c->d_brick_slot, 0xff, sizeof(int32_t) * c->n_bricks, c->stream) ==
                                hipSuccess) &&
             hipMemcpyAsync(c->d_result, &r0, sizeof(r0), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
             hipStreamSynchronize(c->stream) == hipSuccess;
    }
    if (ok && c->build_pref == SPH_BUILD_AUTO) (void)timers_ready(c);  // no events: the bucketed build, untimed
    if (!ok) {
        free_ctx(c);
        return SPH_ERR_HIP;
    }
    *out = c;
    return SPH_OK;
}

extern "C" sph_status sph_destroy(sph_ctx *ctx) {
    if (!ctx) return SPH_ERR_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
    return SPH_OK;
}

extern "C" sph_status sph_buffer_define(sph_ctx *ctx, sph_kind kind, const double origin[3], const double rot[9],
                                        const double half[3], double margin, int32_t *buffer_id) {
    if (!ctx || !origin || !rot || !half) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, true));
    if (kind != SPH_INLET && kind != SPH_OUTLET && kind != SPH_BIDIR) return SPH_ERR_ARG;
    const int dim = ctx->dim;
    double o[3] = {origin[0], origin[1], dim == 3 ? origin[2] : 0.0};
    double h[3] = {half[0], half[1], dim == 3 ? half[2] : 0.0};
    for (int c = 0; c < dim; ++c)
        if (!std::isfinite(o[c]) || !std::isfinite(h[c]) || !(h[c] > 0.0)) return SPH_ERR_ARG;
    if (!std::isfinite(margin)) return SPH_ERR_ARG;
    if (!(margin > 0.0)) margin = ctx->cs;
    const sph_status rs = sph_check_rotation(dim, rot);
    if (rs != SPH_OK) return rs;
    if (ctx->nb >= SPH_MAX_BUFFERS) return SPH_ERR_TOO_MANY_BUFFERS;
    double q[9];
    std::copy(rot, rot + 9, q);
    if (dim == 2) {
        q[2] = q[5] = q[6] = q[7] = 0.0;
        q[8] = 1.0;
    }
    for (int k = 0; k < ctx->nb; ++k)
        if (sphbuf::check_regions_overlap(dim, o, q, h, margin, ctx->b_origin[k], ctx->b_rot[k], ctx->b_half[k],
                                          ctx->b_margin[k]))
            return SPH_ERR_OVERLAP;
    std::vector<int32_t> first, len;
    {
        const sph_status cs = cover_runs(ctx, o, q, h, margin, first, len);
        if (cs != SPH_OK) return cs;
    }

    const int k = ctx->nb;
    const BufDev b = frame_record(ctx, kind, o, q, h, margin);
    // the new buffer's run range (sized for any orientation), its runs, the
    // compact list and the mask
    int32_t rmax = 0;
    int64_t rows = 0;
    run_range(ctx, h, margin, rmax, rows);
    HIP_CHECKED(grow_ranges(ctx, k, rmax, rows));
    ctx->hb[k] = b;
    HIP_TRY(hipMemcpyAsync(ctx->d_bufs + k, &ctx->hb[k], sizeof(BufDev), hipMemcpyHostToDevice, ctx->stream));
    ctx->nb = k + 1;
    const sph_status us = install_runs(ctx, {k}, {first}, {len});
    if (us != SPH_OK) {
        ctx->nb = k;
        return us;
    }
    for (int c = 0; c < 3; ++c) {
        ctx->b_origin[k][c] = o[c];
        ctx->b_half[k][c] = h[c];
    }
    std::copy(q, q + 9, ctx->b_rot[k]);
    ctx->b_margin[k] = margin;
    if (buffer_id) *buffer_id = k + 1;
    return SPH_OK;
}

extern "C" sph_status sph_celllist_build(sph_ctx *ctx, const sph_particles *p) {
    if (!ctx) return SPH_ERR_ARG;
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    HIP_CHECKED(merged_drop(ctx, true));
    ctx->built_capacity = pp.capacity;
    ctx->meth = pick_method(ctx);
    ctx->last_method = ctx->meth == kMethBucketed ? SPH_BUILD_BUCKETED : SPH_BUILD_COUNTING;
    // merged step (domains with buffers): the count pass also lists the candidates;
    // the cells pass is left for the update (or the next call that needs the list)
    const bool cand = ctx->merged && ctx->d_cover && ctx->nb > 0;
    tmark(ctx, 0);
    {
        ProfScope ps(ctx, SPH_PHASE_COUNT);
        if (ctx->meth == kMethBucketed) {
            const BkArgs ba = bk_args(ctx, &pp, cand);
            if (cand)
                hipLaunchKernelGGL(k_bk_count<true>, dim3(bk_blocks(pp.capacity)), dim3(kBkBlock), 0, ctx->stream, ba);
            else
                hipLaunchKernelGGL(k_bk_count<false>, dim3(bk_blocks(pp.capacity)), dim3(kBkBlock), 0, ctx->stream, ba);
        } else {
            const CountArgs ca = count_args(ctx, pp, cand);
            if (cand)
                hipLaunchKernelGGL(k_count<true>, dim3(count_blocks(pp.capacity)), dim3(kBuildBlock), 0, ctx->stream, ca);
            else
                hipLaunchKernelGGL(k_count<false>, dim3(count_blocks(pp.capacity)), dim3(kBuildBlock), 0, ctx->stream, ca);
        }
    }
    HIP_TRY(hipGetLastError());
    tmark(ctx, 1);
    ctx->built = true;
    if (!cand) return build_cells(ctx, nullptr);
    ctx->scan_pending = true;
    ctx->ev_pending = true;
    ctx->nf_full_next = true;
    return SPH_OK;
}

// ----------------------------------------- cell-list build, no allocation --
//
// The three-kernel build of sph_celllist_build for callers that cannot allocate
// device memory: every scratch array of the build (cell counts, packed (key,
// rank) words, their spill words, the scan's tile states, the control block)
// lives in one file-scope device array of fixed size, one copy per GPU for the
// life of the process.  Its address on a device is taken once, with that device
// current, and used for every launch there.

namespace {

constexpr int64_t kNaParticles = SPH_NOALLOC_MAX_PARTICLES;
constexpr int64_t kNaCells = SPH_NOALLOC_MAX_CELLS;
constexpr int64_t kNaTiles = (kNaCells + 1 + kScanTile - 1) / kScanTile;
constexpr size_t kNaAlign = 256;
constexpr size_t na_up(size_t b) { return (b + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr size_t kNaCountOff = 0;
constexpr size_t kNaPackedOff = kNaCountOff + na_up(sizeof(int32_t) * (kNaCells + 1));
constexpr size_t kNaSpillOff = kNaPackedOff + na_up(sizeof(uint32_t) * kNaParticles);
constexpr size_t kNaTileOff = kNaSpillOff + na_up(sizeof(unsigned long long) * kNaParticles);
constexpr size_t kNaCtlOff = kNaTileOff + na_up(sizeof(unsigned long long) * kNaTiles);
constexpr size_t kNaBytes = kNaCtlOff + na_up(sizeof(Ctl));
constexpr int kNaMaxDevices = 64;

// Clears a word range (the counts and the control block start at zero).
__global__ void k_fill_words(uint32_t *w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0u;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of scratch on each device (taken once per device, with that
// device current); host code uses these, never the symbol itself.
static unsigned char *g_na_ptr[kNaMaxDevices];
static std::mutex g_na_mutex;

extern "C" sph_status sph_celllist_build_noalloc(int32_t dim, const double lo[3], double cell_size,
                                                 const int32_t dims[3], const float *x, const float *y, const float *z,
                                                 const int64_t *n_dev, int64_t capacity, int32_t *cell_start,
                                                 int32_t *cell_idx, void *stream) {
    if ((dim != 2 && dim != 3) || !lo || !dims || !x || !y || (dim == 3 && !z) || !n_dev || !cell_start || !cell_idx)
        return SPH_ERR_ARG;
    if (!(cell_size > 0.0) || !std::isfinite(cell_size)) return SPH_ERR_ARG;
    if (capacity < 1 || capacity > kNaParticles) return SPH_ERR_ARG;
    int64_t cells = 1;
    int32_t d3[3] = {1, 1, 1};
    double glo[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < dim; ++c) {
        if (dims[c] < 1 || !std::isfinite(lo[c])) return SPH_ERR_ARG;
        d3[c] = dims[c];
        glo[c] = lo[c];
        cells *= dims[c];
        if (cells > kNaCells) return SPH_ERR_ARG;
    }
    if (!(sphbuf::binning_error_cells(dim, glo, cell_size, d3) < sphbuf::kMaxBinningError)) return SPH_ERR_ARG;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return SPH_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_na_mutex);
        if (!g_na_ptr[dev]) {
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            // the counts and the control block start at zero (later builds leave the
            // counts they used at zero again: the scan clears them)
            hipLaunchKernelGGL(k_fill_words, dim3(256), dim3(256), 0, st,
                               reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(ptr) + kNaCountOff),
                               (int64_t)(kNaPackedOff / 4));
            hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(256), 0, st,
                               reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(ptr) + kNaCtlOff),
                               (int64_t)(na_up(sizeof(Ctl)) / 4));
            HIP_TRY(hipGetLastError());
            g_na_ptr[dev] = static_cast<unsigned char *>(ptr);
        }
        base = g_na_ptr[dev];
    }
    Ctl *ctl = reinterpret_cast<Ctl *>(base + kNaCtlOff);
    Grid g{};
    for (int c = 0; c < 3; ++c) {
        g.lo[c] = (float)glo[c];
        g.dims[c] = d3[c];
        g.bdims[c] = 1;
    }
    g.inv_cs = (float)(1.0 / cell_size);
    g.dim = dim;
    g.blog2 = 0;
    g.brick_slot = nullptr;
    g.overflow_key = (uint32_t)(cells - 1);
    const int64_t m = cells + 1;
    CountArgs ca{};
    ca.x = x;
    ca.y = y;
    ca.z = dim == 3 ? z : nullptr;
    ca.n_dev = n_dev;
    ca.capacity = capacity;
    ca.g = g;
    ca.count = reinterpret_cast<int32_t *>(base + kNaCountOff);
    ca.packed = reinterpret_cast<uint32_t *>(base + kNaPackedOff);
    ca.spill = reinterpret_cast<unsigned long long *>(base + kNaSpillOff);
    ca.rbits = rank_bits(cells);
    ca.tile_state = reinterpret_cast<unsigned long long *>(base + kNaTileOff);
    ca.n_tiles = (m + kScanTile - 1) / kScanTile;
    ca.ctl = ctl;
    ca.nonfinite = &ctl->nonfinite_build;
    hipLaunchKernelGGL(k_count<false>, dim3(count_blocks(capacity)), dim3(kBuildBlock), 0, st, ca);
    ScanArgs sa{};
    sa.count = ca.count;
    sa.cell_start = cell_start;
    sa.m = m;
    sa.tile_state = ca.tile_state;
    sa.ctl = ctl;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)ca.n_tiles), dim3(kScanBlock), 0, st, sa);
    ScatterArgs xa{};
    xa.n_dev = &ctl->n_built;
    xa.capacity = capacity;
    xa.ctl = ctl;
    xa.packed = ca.packed;
    xa.spill = ca.spill;
    xa.rbits = ca.rbits;
    xa.cell_start = cell_start;
    xa.cell_idx = cell_idx;
    const int64_t want = (capacity + kBuildBlock - 1) / kBuildBlock;
    const int blocks = (int)std::max<int64_t>(8, std::min<int64_t>(8192, (want + 7) / 8 * 8));
    hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(kBuildBlock), 0, st, xa);
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

extern "C" sph_status sph_buffer_update_async(sph_ctx *ctx, sph_particles *p) {
    if (!ctx) return SPH_ERR_ARG;
    if (!ctx->built) return SPH_ERR_STATE;
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    if (ctx->fields.rho >= pp.nc) return SPH_ERR_ARG;
    if (ctx->merged && ctx->ev_pending) {
        // the count pass listed the candidates: their exact tests run beside the
        // build's scatter, then the finalize (or the tests alone if a call needed
        // the cell list first)
        const FullArgs fa = cand_args(ctx, pp);
        if (ctx->scan_pending) {
            ctx->scan_pending = false;
            HIP_CHECKED(build_cells(ctx, &fa));
        } else {
            {
                ProfScope ps(ctx, SPH_PHASE_CANDIDATES);
                hipLaunchKernelGGL(k_classify_cand, dim3(kCandBlocksMerged), dim3(kClassifyBlock), 0, ctx->stream, fa);
            }
            HIP_TRY(hipGetLastError());
        }
        ctx->ev_pending = false;
        ctx->built = false;
        return launch_finalize(ctx, pp, false, kCandBlocksMerged);
    }
    HIP_CHECKED(merged_cells(ctx));  // a merged build whose events were dropped: walk the cover cells
    int n_part = 0;
    if (ctx->n_runs > 0) {
        const LocalArgs la = local_args(ctx, pp);
        n_part = std::max(1, std::min(kMaxPartBlocks, (ctx->n_runs + kRunsPerBlock - 1) / kRunsPerBlock));
        ProfScope ps(ctx, SPH_PHASE_CLASSIFY);
        hipLaunchKernelGGL(k_classify_local, dim3(n_part), dim3(kClassifyBlock), 0, ctx->stream, la);
        HIP_TRY(hipGetLastError());
    }
    ctx->built = false;
    return launch_finalize(ctx, pp, true, n_part);
}

static sph_status fullscan_enqueue(sph_ctx *ctx, sph_particles *p) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, true));
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    if (ctx->fields.rho >= pp.nc) return SPH_ERR_ARG;
    const FullArgs fa = cand_args(ctx, pp);
    {
        ProfScope ps(ctx, SPH_PHASE_FULLSCAN);
        hipLaunchKernelGGL(k_filter_full, dim3(ctx->full_blocks), dim3(kClassifyBlock), 0, ctx->stream, fa);
    }
    HIP_TRY(hipGetLastError());
    {
        ProfScope ps(ctx, SPH_PHASE_CANDIDATES);
        hipLaunchKernelGGL(k_classify_cand, dim3(kCandBlocks), dim3(kClassifyBlock), 0, ctx->stream, fa);
    }
    HIP_TRY(hipGetLastError());
    ctx->built = false;
    return launch_finalize(ctx, pp, false, ctx->full_blocks);
}

extern "C" sph_status sph_buffer_update_fullscan_async(sph_ctx *ctx, sph_particles *p) {
    return fullscan_enqueue(ctx, p);
}

static sph_status finish_sync(sph_ctx *ctx, int64_t *n_generated, int64_t *n_deleted) {
    const sph_status w = wait_result(ctx);
    if (w != SPH_OK) return w;
    if (n_generated) *n_generated = ctx->h_result->n_generated;
    if (n_deleted) *n_deleted = ctx->h_result->n_deleted;
    return (sph_status)ctx->h_result->status;
}

extern "C" sph_status sph_buffer_update(sph_ctx *ctx, sph_particles *p, int64_t *n_generated, int64_t *n_deleted) {
    const sph_status st = sph_buffer_update_async(ctx, p);
    if (st != SPH_OK) return st;
    return finish_sync(ctx, n_generated, n_deleted);
}

extern "C" sph_status sph_buffer_update_fullscan(sph_ctx *ctx, sph_particles *p, int64_t *n_generated,
                                                 int64_t *n_deleted) {
    const sph_status st = fullscan_enqueue(ctx, p);
    if (st != SPH_OK) return st;
    return finish_sync(ctx, n_generated, n_deleted);
}

extern "C" sph_status sph_last_result(sph_ctx *ctx, sph_result *out) {
    if (!ctx || !out) return SPH_ERR_ARG;
    const sph_status w = wait_result(ctx);
    if (w != SPH_OK) return w;
    *out = *ctx->h_result;
    return SPH_OK;
}

extern "C" sph_status sph_last_events(sph_ctx *ctx, int64_t *gen_src, int64_t *del_idx, int64_t cap, int64_t *n_gen,
                                      int64_t *n_del) {
    if (!ctx || !n_gen || !n_del || cap < 0) return SPH_ERR_ARG;
    const sph_status w = wait_result(ctx);
    if (w != SPH_OK) return w;
    const sph_result r = *ctx->h_result;
    *n_gen = r.status == SPH_OK ? r.n_generated : 0;
    *n_del = r.status == SPH_OK ? r.n_deleted : 0;
    const int64_t g = std::min<int64_t>(cap, *n_gen), d = std::min<int64_t>(cap, *n_del);
    std::vector<uint32_t> tmp((size_t)std::max<int64_t>(1, std::max(g, d)));
    if (g > 0) {
        if (!gen_src) return SPH_ERR_ARG;
        HIP_TRY(hipMemcpy(tmp.data(), ctx->d_gen_sorted, sizeof(uint32_t) * g, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < g; ++j) gen_src[j] = (int64_t)tmp[j];
    }
    if (d > 0) {
        if (!del_idx) return SPH_ERR_ARG;
        HIP_TRY(hipMemcpy(tmp.data(), ctx->d_del_sorted, sizeof(uint32_t) * d, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < d; ++j) del_idx[j] = (int64_t)tmp[j];
    }
    return SPH_OK;
}

extern "C" sph_status sph_build_stats(sph_ctx *ctx, int32_t *method, double us[2], int64_t samples[2]) {
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->bt.init) timers_harvest(ctx);
    if (method) *method = ctx->last_method;
    for (int m = 0; m < 2; ++m) {
        if (us) us[m] = ctx->bt.samples[m] ? ctx->bt.est[m] : 0.0;
        if (samples) samples[m] = ctx->bt.samples[m];
    }
    return SPH_OK;
}

extern "C" sph_status sph_build_retune(sph_ctx *ctx) {
    if (!ctx) return SPH_ERR_ARG;
    BuildTimer &t = ctx->bt;
    if (t.init) timers_harvest(ctx);
    for (int m = 0; m < 2; ++m) {
        t.samples[m] = 0;
        t.est[m] = 0.0;
    }
    for (int s = 0; s < kTimerSets; ++s)  // timings in flight would count: drop them
        if (t.busy[s] && s != ctx->tset) t.busy[s] = false;
    t.builds = std::min<int64_t>(t.builds, 2);
    return SPH_OK;
}

extern "C" sph_status sph_celllist_view(sph_ctx *ctx, const int32_t **cell_start, const int32_t **cell_idx,
                                        int64_t *n_cells, int32_t dims[3]) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_cells(ctx));
    if (cell_start) *cell_start = ctx->d_cell_start;
    if (cell_idx) *cell_idx = ctx->d_cell_idx;
    if (n_cells) *n_cells = ctx->n_cells;
    if (dims)
        for (int c = 0; c < 3; ++c) dims[c] = ctx->dims[c];
    return SPH_OK;
}

extern "C" sph_status sph_neighbor_count(sph_ctx *ctx, const sph_particles *p, double radius, int32_t *counts) {
    if (!ctx || !counts) return SPH_ERR_ARG;
    HIP_CHECKED(merged_cells(ctx));
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    const double r2 = radius * radius;
    if (!(radius > 0.0) || !(radius <= ctx->cs) || !(r2 >= 1e-30)) return SPH_ERR_ARG;
    int max_dim = 1;
    for (int c = 0; c < ctx->dim; ++c) max_dim = std::max(max_dim, ctx->dims[c]);
    // FP32 cell coordinate t = fl(fl(x - lo) * inv_cs) is within 2u(t + 1) of the
    // exact one and the cell size times inv_cs within u of 1 (u = 2^-24): a pair
    // less than one cell apart is two cells apart only if one of them lies within
    // 2 * 2u(t + 1) + u of its cell's face
    const double band = 8.0 * 0x1p-24 * (double)(max_dim + 2);
    if (band >= 0.25) return SPH_ERR_ARG;
    if (!ctx->built) return SPH_ERR_STATE;
    NbrArgs a{};
    a.p = pp;
    a.g = grid_of(ctx);
    a.cell_start = ctx->d_cell_start;
    a.cell_idx = ctx->d_cell_idx;
    // the build's key scratch (4 + 8 bytes per particle) holds the ordered positions
    a.xs = reinterpret_cast<float *>(ctx->d_keys);
    a.ys = reinterpret_cast<float *>(ctx->d_keyrank);
    a.zs = a.ys + ctx->capacity;
    a.r2 = r2;
    // the FP32 squared distance is within 2^-21 (relative) of the exact one
    a.r2_in = (float)(r2 * (1.0 - 0x1p-16));
    a.r2_out = (float)(r2 * (1.0 + 0x1p-16));
    a.band = (float)band;
    a.counts = counts;
    // (a multiple of 8, so the XCD renumbering applies)
    const int blocks = (int)std::max<int64_t>(8, std::min<int64_t>(65536, (pp.capacity + kNbrBlock - 1) / kNbrBlock + 7) / 8 * 8);
    {
        ProfScope ps(ctx, SPH_PHASE_NEIGHBOR);
        hipLaunchKernelGGL(k_nbr_order, dim3(blocks), dim3(kNbrBlock), 0, ctx->stream, a);
        if (a.g.dim == 3)
            hipLaunchKernelGGL(k_neighbor_count<3>, dim3(blocks), dim3(kNbrBlock), 0, ctx->stream, a);
        else
            hipLaunchKernelGGL(k_neighbor_count<2>, dim3(blocks), dim3(kNbrBlock), 0, ctx->stream, a);
    }
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

// ------------------------------------- boundary conditions, rotating buffers --

extern "C" sph_status sph_set_fields(sph_ctx *ctx, const sph_fields *fields) {
    if (!ctx || !fields) return SPH_ERR_ARG;
    for (int c = 0; c < 3; ++c)
        if (fields->vel[c] < -1 || fields->vel[c] >= SPH_MAX_CARRIED) return SPH_ERR_ARG;
    if (fields->rho < -1 || fields->rho >= SPH_MAX_CARRIED) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));  // a merged build's duplicates were captured with the old fields
    if (fields->rho != ctx->fields.rho) ctx->layout_gen++;  // the density field is baked into batch tables
    ctx->fields = *fields;
    return SPH_OK;
}

extern "C" sph_status sph_buffer_set_bc(sph_ctx *ctx, int32_t buffer_id, const sph_bc *bc) {
    if (!ctx || !bc || buffer_id < 1 || buffer_id > ctx->nb) return SPH_ERR_ARG;
    if (bc->kind < SPH_BC_NONE || bc->kind > SPH_BC_PRESSURE) return SPH_ERR_ARG;
    if (bc->profile < SPH_PROFILE_PLUG || bc->profile > SPH_PROFILE_PARABOLIC_R) return SPH_ERR_ARG;
    if (!std::isfinite(bc->u) || !std::isfinite(bc->radius) || !std::isfinite(bc->p_b) || !std::isfinite(bc->rho0) ||
        !std::isfinite(bc->c0))
        return SPH_ERR_ARG;
    if (bc->kind == SPH_BC_VELOCITY && bc->profile != SPH_PROFILE_PLUG && !(bc->radius > 0.0)) return SPH_ERR_ARG;
    if (bc->kind == SPH_BC_PRESSURE && !(bc->c0 > 0.0)) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));  // a merged build emitted with the old boundary values
    BufDev &b = ctx->hb[buffer_id - 1];
    b.bc_kind = bc->kind;
    b.profile = bc->profile;
    b.bc_u = bc->u;
    b.bc_radius = bc->radius;
    // Eq. (postulate-density) with the EoS p = c0^2 (rho - rho0)
    b.rho_rec = bc->kind == SPH_BC_PRESSURE ? (float)(bc->rho0 + bc->p_b / (bc->c0 * bc->c0)) : 0.0f;
    HIP_TRY(hipMemcpyAsync(ctx->d_bufs + (buffer_id - 1), &b, sizeof(BufDev), hipMemcpyHostToDevice, ctx->stream));
    return SPH_OK;
}

// Velocity fields of a call: every component present and inside the carried arrays.
static bool velocity_fields_ok(const sph_ctx *ctx, const Parts &pp) {
    for (int c = 0; c < ctx->dim; ++c)
        if (ctx->fields.vel[c] < 0 || ctx->fields.vel[c] >= pp.nc) return false;
    return true;
}

static sph_status launch_buffer_pass(sph_ctx *ctx, const Parts &pp, int which, const double center[3],
                                     const double m[9]) {
    BcArgs a{};
    a.p = pp;
    a.bufs = ctx->d_bufs;
    a.nb = ctx->nb;
    a.run_first = ctx->d_run_first;
    a.run_len = ctx->d_run_len;
    a.run_buf = ctx->d_run_buf;
    a.ctl = ctx->d_ctl;
    a.cell_start = ctx->d_cell_start;
    a.cell_idx = ctx->d_cell_idx;
    for (int c = 0; c < 3; ++c) a.vel[c] = c < ctx->dim ? ctx->fields.vel[c] : -1;
    a.which = which;
    if (center)
        for (int c = 0; c < 3; ++c) a.center[c] = center[c];
    if (m)
        for (int i = 0; i < 9; ++i) a.m[i] = m[i];
    a.found = ctx->d_bcfound;
    if (ctx->n_runs > 0) {
        const int wpb = kClassifyBlock / kWave;
        const int blocks = std::max(1, std::min(kMaxPartBlocks, (ctx->n_runs + wpb - 1) / wpb));
        ProfScope ps(ctx, which < 0 ? SPH_PHASE_BC : SPH_PHASE_ROTATE);
        hipLaunchKernelGGL(k_buffer_bc, dim3(blocks), dim3(kClassifyBlock), 0, ctx->stream, a);
    }
    hipLaunchKernelGGL(k_bc_finish, dim3(1), dim3(kBcFinishBlock), 0, ctx->stream, ctx->d_bcfound, ctx->d_bufs, ctx->nb,
                       which, ctx->d_ctl);
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

static sph_status read_bc_status(sph_ctx *ctx) {
    HIP_TRY(hipMemcpyAsync(ctx->h_bc_status, &ctx->d_ctl->bc_status, sizeof(unsigned), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return (sph_status)*ctx->h_bc_status;
}

extern "C" sph_status sph_buffer_apply_bc_async(sph_ctx *ctx, sph_particles *p) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    if (!velocity_fields_ok(ctx, pp)) return SPH_ERR_ARG;
    if (!ctx->built) return SPH_ERR_STATE;
    return launch_buffer_pass(ctx, pp, -1, nullptr, nullptr);
}

extern "C" sph_status sph_buffer_apply_bc(sph_ctx *ctx, sph_particles *p) {
    HIP_CHECKED(sph_buffer_apply_bc_async(ctx, p));
    return read_bc_status(ctx);
}

extern "C" sph_status sph_last_bc_status(sph_ctx *ctx) {
    if (!ctx) return SPH_ERR_ARG;
    return read_bc_status(ctx);
}

// y = m x with rows summed left to right (two terms in 2-D), FP64 on the host.
static void mat_vec_host(int dim, const double m[9], const double x[3], double y[3]) {
    for (int r = 0; r < 3; ++r) {
        double acc = m[3 * r] * x[0] + m[3 * r + 1] * x[1];
        if (dim == 3) acc = acc + m[3 * r + 2] * x[2];
        y[r] = acc;
    }
}

extern "C" sph_status sph_buffer_rotate_async(sph_ctx *ctx, sph_particles *p, int32_t buffer_id,
                                              const double center[3], const double m[9]) {
    if (!ctx || !center || !m || buffer_id < 1 || buffer_id > ctx->nb) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));
    const int dim = ctx->dim;
    for (int c = 0; c < dim; ++c)
        if (!std::isfinite(center[c])) return SPH_ERR_ARG;
    const sph_status rs = sph_check_rotation(dim, m);
    if (rs != SPH_OK) return rs;
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    for (int c = 0; c < dim; ++c)
        if (ctx->fields.vel[c] >= pp.nc) return SPH_ERR_ARG;
    if (!ctx->built) return SPH_ERR_STATE;
    const int k = buffer_id - 1;
    // the frame follows the body: O' <- C + m (O' - C), rows of Q <- m (rows of Q)
    double o[3], q[9];
    {
        const double d[3] = {ctx->b_origin[k][0] - center[0], ctx->b_origin[k][1] - center[1],
                             dim == 3 ? ctx->b_origin[k][2] - center[2] : 0.0};
        double e[3];
        mat_vec_host(dim, m, d, e);
        for (int c = 0; c < 3; ++c) o[c] = c < dim ? center[c] + e[c] : ctx->b_origin[k][c];
        for (int r = 0; r < 3; ++r) {
            const double row[3] = {ctx->b_rot[k][3 * r], ctx->b_rot[k][3 * r + 1], ctx->b_rot[k][3 * r + 2]};
            double nr[3];
            mat_vec_host(dim, m, row, nr);
            for (int c = 0; c < 3; ++c) q[3 * r + c] = c < dim ? nr[c] : ctx->b_rot[k][3 * r + c];
        }
    }
    for (int j = 0; j < ctx->nb; ++j)
        if (j != k && sphbuf::check_regions_overlap(dim, o, q, ctx->b_half[k], ctx->b_margin[k], ctx->b_origin[j],
                                                    ctx->b_rot[j], ctx->b_half[j], ctx->b_margin[j]))
            return SPH_ERR_OVERLAP;
    // where the turned check region's cover is searched (host FP64, no device work)
    sphbuf::CoverBox cb;
    {
        const sph_status cs =
            sphbuf::cover_box(dim, ctx->lo, ctx->cs, ctx->dims, o, q, ctx->b_half[k], ctx->b_margin[k], cb);
        if (cs != SPH_OK) return cs;
    }
    // turn the particles with the old frame and cover, then compute the new cover on
    // the device: its rows (k_cover_rows), then its runs, mask bits, the new frame
    // record and the compact run list (k_cover_write); nothing waits for the stream
    const sph_status ls = launch_buffer_pass(ctx, pp, k, center, m);
    if (ls != SPH_OK) return ls;
    BufDev b = frame_record(ctx, ctx->hb[k].kind, o, q, ctx->b_half[k], ctx->b_margin[k]);
    copy_bc(b, ctx->hb[k]);
    ctx->hb[k] = b;
    CoverArgs ca = cover_args(ctx);
    ca.k = k;
    for (int i = 0; i < 3; ++i) {
        ca.obb.c[i] = cb.c[i];
        ca.obb.h[i] = cb.h[i];
        for (int j = 0; j < 3; ++j) ca.obb.ax[i][j] = cb.ax[i][j];
        ca.blo[i] = cb.blo[i];
        ca.bhi[i] = cb.bhi[i];
        ca.lo_i[i] = cb.lo_i[i];
        ca.hi_i[i] = cb.hi_i[i];
    }
    ca.eps = cb.eps;
    ca.rec = b;
    ca.bufs = ctx->d_bufs;
    {
        const int64_t rows = (int64_t)(cb.hi_i[1] - cb.lo_i[1] + 1) * (dim == 3 ? cb.hi_i[2] - cb.lo_i[2] + 1 : 1);
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (std::max(rows, (int64_t)ctx->hcnt[k]) + 255) / 256));
        ProfScope ps(ctx, SPH_PHASE_COVER);
        hipLaunchKernelGGL(k_cover_rows, dim3(blocks), dim3(256), 0, ctx->stream, ca);
        hipLaunchKernelGGL(k_cover_write, dim3(1), dim3(kCoverBlock), 0, ctx->stream, ca);
    }
    HIP_TRY(hipGetLastError());
    for (int c = 0; c < 3; ++c) ctx->b_origin[k][c] = o[c];
    std::copy(q, q + 9, ctx->b_rot[k]);
    ctx->built = false;  // the buffer's particles moved
    return SPH_OK;
}

extern "C" sph_status sph_buffer_rotate(sph_ctx *ctx, sph_particles *p, int32_t buffer_id, const double center[3],
                                        const double m[9]) {
    HIP_CHECKED(sph_buffer_rotate_async(ctx, p, buffer_id, center, m));
    return read_bc_status(ctx);
}

extern "C" sph_status sph_buffer_cover(sph_ctx *ctx, int32_t buffer_id, int32_t *first, int32_t *len, int64_t cap,
                                       int64_t *n_runs) {
    if (!ctx || !n_runs || buffer_id < 1 || buffer_id > ctx->nb || cap < 0) return SPH_ERR_ARG;
    const int k = buffer_id - 1;
    int32_t cnt = 0;
    HIP_TRY(hipMemcpyAsync(&cnt, &ctx->d_ctl->run_cnt[k], sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *n_runs = cnt;
    if (cnt > cap) return SPH_ERR_ARG;
    if (cnt > 0) {
        if (!first || !len) return SPH_ERR_ARG;
        HIP_TRY(hipMemcpy(first, ctx->d_src_first + ctx->rbase[k], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(len, ctx->d_src_len + ctx->rbase[k], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    }
    return SPH_OK;
}

extern "C" sph_status sph_buffer_identify(sph_ctx *ctx, sph_particles *p, int32_t buffer_id) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));
    if (buffer_id != -1 && (buffer_id < 1 || buffer_id > ctx->nb)) return SPH_ERR_ARG;
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    HIP_TRY(hipMemsetAsync(&ctx->d_ctl->ident_bad, 0, sizeof(unsigned), ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->d_ctl->ident_count, 0, sizeof(unsigned long long) * 16, ctx->stream));
    IdentArgs ia{};
    ia.p = pp;
    ia.bufs = ctx->d_bufs;
    ia.nb = ctx->nb;
    ia.which = buffer_id < 0 ? -1 : buffer_id - 1;
    ia.ctl = ctx->d_ctl;
    hipLaunchKernelGGL(k_ident_check, dim3(ctx->build_blocks), dim3(kBuildBlock), 0, ctx->stream, ia);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ident_apply, dim3(ctx->build_blocks), dim3(kBuildBlock), 0, ctx->stream, ia);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ident_commit, dim3(1), dim3(64), 0, ctx->stream, ia);
    HIP_TRY(hipGetLastError());
    unsigned bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, &ctx->d_ctl->ident_bad, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return bad ? SPH_ERR_NONFINITE : SPH_OK;
}

extern "C" sph_status sph_state_get(sph_ctx *ctx, int64_t *next_id, int64_t n_labelled[SPH_MAX_BUFFERS]) {
    if (!ctx) return SPH_ERR_ARG;
    Ctl h{};
    HIP_TRY(hipMemcpyAsync(&h, ctx->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (next_id) *next_id = h.next_id;
    if (n_labelled)
        for (int k = 0; k < SPH_MAX_BUFFERS; ++k) n_labelled[k] = h.n_labelled[k];
    return SPH_OK;
}

extern "C" sph_status sph_state_set(sph_ctx *ctx, int64_t next_id, const int64_t n_labelled[SPH_MAX_BUFFERS]) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));
    HIP_TRY(hipMemcpyAsync(&ctx->d_ctl->next_id, &next_id, sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    if (n_labelled)
        HIP_TRY(hipMemcpyAsync(ctx->d_ctl->n_labelled, n_labelled, sizeof(int64_t) * SPH_MAX_BUFFERS,
                               hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SPH_OK;
}

// Blob layout: tag, next_id, n_labelled[SPH_MAX_BUFFERS] (int64 each).
static constexpr uint64_t kStateTag = 0x31766174736870ull;  // "phstav1"
static_assert(SPH_STATE_BLOB_BYTES == 8 * (2 + SPH_MAX_BUFFERS), "state blob layout");

extern "C" sph_status sph_state_export(sph_ctx *ctx, void *blob, size_t *len) {
    if (!ctx || !len) return SPH_ERR_ARG;
    const size_t have = *len;
    *len = SPH_STATE_BLOB_BYTES;
    if (!blob || have < SPH_STATE_BLOB_BYTES) return SPH_ERR_ARG;
    int64_t w[2 + SPH_MAX_BUFFERS];
    w[0] = (int64_t)kStateTag;
    HIP_CHECKED(sph_state_get(ctx, &w[1], &w[2]));
    std::memcpy(blob, w, sizeof(w));
    return SPH_OK;
}

extern "C" sph_status sph_state_import(sph_ctx *ctx, const void *blob, size_t len) {
    if (!ctx || !blob || len != SPH_STATE_BLOB_BYTES) return SPH_ERR_ARG;
    int64_t w[2 + SPH_MAX_BUFFERS];
    std::memcpy(w, blob, sizeof(w));
    if ((uint64_t)w[0] != kStateTag) return SPH_ERR_ARG;
    return sph_state_set(ctx, w[1], &w[2]);
}

extern "C" sph_status sph_profile_enable(sph_ctx *ctx, int32_t on) {
    if (!ctx) return SPH_ERR_ARG;
    if (on && ctx->prof_ev.empty()) {
        ctx->prof_ev.resize(2 * kProfSlots);
        ctx->prof_phase.resize(kProfSlots);
        for (auto &e : ctx->prof_ev)
            if (hipEventCreate(&e) != hipSuccess) return SPH_ERR_HIP;
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->prof_used = 0;
    for (int i = 0; i < SPH_NPHASE; ++i) {
        ctx->prof_ms[i] = 0.0;
        ctx->prof_n[i] = 0;
    }
    ctx->prof_on = on != 0;
    return SPH_OK;
}

extern "C" sph_status sph_profile_read(sph_ctx *ctx, double ms[SPH_NPHASE], int64_t launches[SPH_NPHASE],
                                       int32_t reset) {
    if (!ctx) return SPH_ERR_ARG;
    prof_drain(ctx);
    for (int i = 0; i < SPH_NPHASE; ++i) {
        if (ms) ms[i] = ctx->prof_ms[i];
        if (launches) launches[i] = ctx->prof_n[i];
        if (reset) {
            ctx->prof_ms[i] = 0.0;
            ctx->prof_n[i] = 0;
        }
    }
    return SPH_OK;
}

extern "C" sph_status sph_grid_fit(sph_ctx *ctx, const sph_particles *p) {
    if (!ctx) return SPH_ERR_ARG;
    HIP_CHECKED(merged_drop(ctx, false));
    if (ctx->blog2 == 0) return SPH_OK;
    Parts pp;
    const sph_status st = parts_of(ctx, p, pp);
    if (st != SPH_OK) return st;
    const int64_t nb = ctx->n_bricks;
    uint8_t *d_mask = nullptr;
    HIP_TRY(hipMalloc(&d_mask, (size_t)nb));
    std::vector<uint8_t> occ((size_t)nb);
    bool ok = hipMemsetAsync(d_mask, 0, (size_t)nb, ctx->stream) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_mark_bricks, dim3(ctx->build_blocks), dim3(kBuildBlock), 0, ctx->stream, pp.pos[0],
                           pp.pos[1], pp.pos[2], pp.n_dev, pp.capacity, grid_of(ctx), d_mask);
        ok = hipGetLastError() == hipSuccess &&
             hipMemcpyAsync(occ.data(), d_mask, (size_t)nb, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
             hipStreamSynchronize(ctx->stream) == hipSuccess;
    }
    (void)hipFree(d_mask);
    if (!ok) return SPH_ERR_HIP;
    // dilate by the margin (Chebyshev distance in bricks), one axis at a time
    const int bd[3] = {ctx->bdims[0], ctx->bdims[1], ctx->bdims[2]};
    const int64_t stride[3] = {1, bd[0], (int64_t)bd[0] * bd[1]};
    std::vector<uint8_t> act = occ, tmp((size_t)nb);
    for (int ax = 0; ax < ctx->dim; ++ax) {
        tmp.assign((size_t)nb, 0);
        for (int64_t i = 0; i < nb; ++i) {
            if (!act[(size_t)i]) continue;
            const int64_t c = (i / stride[ax]) % bd[ax];
            for (int64_t d = -ctx->bmargin; d <= ctx->bmargin; ++d)
                if (c + d >= 0 && c + d < bd[ax]) tmp[(size_t)(i + d * stride[ax])] = 1;
        }
        act.swap(tmp);
    }
    int64_t n_active = 0;
    for (int64_t i = 0; i < nb; ++i) ctx->h_brick_slot[(size_t)i] = act[(size_t)i] ? (int32_t)n_active++ : -1;
    const int64_t per_brick = (int64_t)1 << (ctx->dim * ctx->blog2);
    const int64_t cells = n_active * per_brick + 1;
    if (cells >= 2147483000LL) return SPH_ERR_ARG;
    const int64_t m = cells + 1;
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    int32_t *cnt = nullptr, *start = nullptr;
    unsigned long long *ts = nullptr;
    if (hipMalloc(&cnt, sizeof(int32_t) * m) != hipSuccess || hipMalloc(&start, sizeof(int32_t) * (m + 1)) != hipSuccess ||
        hipMalloc(&ts, sizeof(unsigned long long) * tiles) != hipSuccess) {
        (void)hipFree(cnt);
        (void)hipFree(start);
        (void)hipFree(ts);
        return SPH_ERR_HIP;
    }
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * m, ctx->stream));
    HIP_TRY(hipMemsetAsync(start, 0, sizeof(int32_t) * (m + 1), ctx->stream));
    HIP_TRY(hipMemsetAsync(ts, 0, sizeof(unsigned long long) * tiles, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->d_brick_slot, ctx->h_brick_slot.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->d_count);
    (void)hipFree(ctx->d_cell_start);
    (void)hipFree(ctx->d_tile_state);
    ctx->layout_gen++;
    ctx->d_count = cnt;
    ctx->d_cell_start = start;
    ctx->d_tile_state = ts;
    ctx->n_cells = cells;
    bk_layout(ctx);
    ctx->rbits = rank_bits(cells);
    ctx->n_tiles = tiles;
    ctx->built = false;
    // candidate cells of every buffer in the new key space (frames as they are now)
    std::vector<int> which;
    std::vector<std::vector<int32_t>> rf, rl;
    for (int k = 0; k < ctx->nb; ++k) {
        std::vector<int32_t> f, l;
        const sph_status cs = cover_runs(ctx, ctx->b_origin[k], ctx->b_rot[k], ctx->b_half[k], ctx->b_margin[k], f, l);
        if (cs != SPH_OK) return cs;
        which.push_back(k);
        rf.push_back(std::move(f));
        rl.push_back(std::move(l));
    }
    return install_runs(ctx, which, rf, rl);
}

// ================================================================== batches ==

struct sph_batch {
    std::vector<sph_ctx *> doms;
    std::vector<uint64_t> gens;  // each member's layout generation when the tables were made
    std::vector<Parts> parts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int mode = SPH_BATCH_GRAPH;
    int count_ppb = 2048;  // particles per block of the count / scatter phases
    int cls_rpb = kRunsPerBlock;  // cover runs per classify workgroup (the gather schedule)
    int fin_blocks = 1;    // finalize workgroups per domain
    std::vector<LocalArgs> la_host;  // classify arguments per domain (re-uploaded with the schedule)
    CountArgs *d_ca = nullptr;
    ScanArgs *d_sa = nullptr;
    ScatterArgs *d_xa = nullptr;
    LocalArgs *d_la = nullptr;
    FinArgs *d_fa = nullptr;
    BlockMap *d_map_count = nullptr, *d_map_scan = nullptr, *d_map_cls = nullptr;
    int32_t *d_vg_count = nullptr, *d_vg_cls = nullptr;
    int nb_count = 0, nb_scan = 0, nb_cls = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    sph_result *h_res = nullptr;  // pinned, one per domain
    // optional per-launch timing of the five launches (launch mode only)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;  // 2 per launch slot
    std::vector<int> prof_phase;
    size_t prof_used = 0;
    double prof_ms[kBatchPhases] = {};
    int64_t prof_n[kBatchPhases] = {};
};

namespace {

void batch_drop_graph(sph_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

template <class T>
sph_status upload_table(T *&dst, const std::vector<T> &v, hipStream_t s) {
    (void)hipFree(dst);
    dst = nullptr;
    if (v.empty()) return SPH_OK;
    HIP_TRY(hipMalloc(&dst, sizeof(T) * v.size()));
    HIP_TRY(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return SPH_OK;
}

// Block maps of the count/scatter, scan and classify launches.
sph_status batch_layout(sph_batch *b) {
    batch_drop_graph(b);
    std::vector<BlockMap> mc, ms, ml;
    std::vector<int32_t> vgc, vgl;
    for (size_t d = 0; d < b->doms.size(); ++d) {
        const sph_ctx *c = b->doms[d];
        const int64_t cap = b->parts[d].capacity;
        const int vc = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (cap + b->count_ppb - 1) / b->count_ppb));
        vgc.push_back(vc);
        for (int v = 0; v < vc; ++v) mc.push_back({(int32_t)d, v});
        for (int64_t t = 0; t < c->n_tiles; ++t) ms.push_back({(int32_t)d, (int32_t)t});
        const int vl =
            c->n_runs > 0 ? std::max(1, std::min(kMaxPartBlocks, (c->n_runs + b->cls_rpb - 1) / b->cls_rpb)) : 0;
        vgl.push_back(vl);
        for (int v = 0; v < vl; ++v) ml.push_back({(int32_t)d, v});
    }
    for (auto *t : {&mc, &ms, &ml})  // padding for the XCD renumbering (a multiple of 8 blocks)
        while (!t->empty() && t->size() % 8) t->push_back({-1, 0});
    sph_status st;
    for (LocalArgs &la : b->la_host) la.rpb = b->cls_rpb;
    if ((st = upload_table(b->d_la, b->la_host, b->stream)) != SPH_OK) return st;
    if ((st = upload_table(b->d_map_count, mc, b->stream)) != SPH_OK) return st;
    if ((st = upload_table(b->d_map_scan, ms, b->stream)) != SPH_OK) return st;
    if ((st = upload_table(b->d_map_cls, ml, b->stream)) != SPH_OK) return st;
    if ((st = upload_table(b->d_vg_count, vgc, b->stream)) != SPH_OK) return st;
    if ((st = upload_table(b->d_vg_cls, vgl, b->stream)) != SPH_OK) return st;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->nb_count = (int)mc.size();
    b->nb_scan = (int)ms.size();
    b->nb_cls = (int)ml.size();
    return SPH_OK;
}

// Brackets one batch launch with events when the batch's profiling is on.
struct BatchProf {
    sph_batch *b;
    size_t slot = 0;
    bool on = false;
    BatchProf(sph_batch *bb, int phase) : b(bb) {
        if (!b->prof_on || b->prof_used >= kProfSlots) return;
        slot = b->prof_used++;
        b->prof_phase[slot] = phase;
        on = hipEventRecord(b->prof_ev[2 * slot], b->stream) == hipSuccess;
    }
    ~BatchProf() {
        if (on) (void)hipEventRecord(b->prof_ev[2 * slot + 1], b->stream);
    }
};

// One step of every domain: five launches whatever the number of domains.
sph_status batch_enqueue(sph_batch *b) {
    const int nd = (int)b->doms.size();
    {
        BatchProf p(b, 0);
        hipLaunchKernelGGL(kb_count, dim3(b->nb_count), dim3(kBuildBlock), 0, b->stream, b->d_ca, b->d_map_count,
                           b->d_vg_count);
    }
    {
        BatchProf p(b, 1);
        hipLaunchKernelGGL(kb_scan, dim3(b->nb_scan), dim3(kScanBlock), 0, b->stream, b->d_sa, b->d_map_scan);
    }
    {
        BatchProf p(b, 2);
        hipLaunchKernelGGL(kb_scatter, dim3(b->nb_count), dim3(kBuildBlock), 0, b->stream, b->d_xa, b->d_map_count,
                           b->d_vg_count);
    }
    if (b->nb_cls > 0) {
        BatchProf p(b, 3);
        hipLaunchKernelGGL(kb_classify, dim3(b->nb_cls), dim3(kClassifyBlock), 0, b->stream, b->d_la, b->d_map_cls,
                           b->d_vg_cls);
    }
    {
        BatchProf p(b, 4);
        hipLaunchKernelGGL(kb_finalize, dim3(nd * b->fin_blocks), dim3(kFinBlock), 0, b->stream, b->d_fa,
                           b->fin_blocks);
    }
    HIP_TRY(hipGetLastError());
    return SPH_OK;
}

void batch_free(sph_batch *b) {
    if (!b) return;
    batch_drop_graph(b);
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    (void)hipFree(b->d_ca);
    (void)hipFree(b->d_sa);
    (void)hipFree(b->d_xa);
    (void)hipFree(b->d_la);
    (void)hipFree(b->d_fa);
    (void)hipFree(b->d_map_count);
    (void)hipFree(b->d_map_scan);
    (void)hipFree(b->d_map_cls);
    (void)hipFree(b->d_vg_count);
    (void)hipFree(b->d_vg_cls);
    if (b->h_res) (void)hipHostFree(b->h_res);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" sph_status sph_batch_create(sph_ctx *const *domains, const sph_particles *particles, int32_t n_domains,
                                       void *stream, sph_batch **out) {
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    if (!domains || !particles || n_domains < 1 || n_domains > 65535) return SPH_ERR_ARG;
    for (int d = 0; d < n_domains; ++d) {  // no build work of a domain left in flight
        if (!domains[d]) return SPH_ERR_ARG;
        HIP_CHECKED(merged_drop(domains[d], true));
        HIP_TRY(hipStreamSynchronize(domains[d]->stream));
    }
    sph_batch *b = new (std::nothrow) sph_batch();
    if (!b) return SPH_ERR_HIP;
    b->stream = (hipStream_t)stream;
    if (!b->stream) {  // graphs cannot be captured on the null stream
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return SPH_ERR_HIP;
        }
        b->own_stream = true;
    }
    std::vector<CountArgs> ca;
    std::vector<ScanArgs> sa;
    std::vector<ScatterArgs> xa;
    std::vector<LocalArgs> la;
    std::vector<FinArgs> fa;
    for (int d = 0; d < n_domains; ++d) {
        sph_ctx *c = domains[d];
        Parts pp;
        sph_status st = c ? parts_of(c, &particles[d], pp) : SPH_ERR_ARG;
        if (st != SPH_OK) {
            batch_free(b);
            return st;
        }
        (void)hipStreamSynchronize(c->stream);
        b->doms.push_back(c);
        b->gens.push_back(c->layout_gen);
        b->parts.push_back(pp);
        ca.push_back(count_args(c, pp));
        sa.push_back(scan_args(c));
        xa.push_back(scatter_args(c, pp.capacity));
        la.push_back(local_args(c, pp));
        fa.push_back(fin_args(c, pp, true));
    }
    // one round of finalize workgroups over the CUs: fewer per domain in large batches
    b->fin_blocks = std::max(1, std::min(kFinBlocksMax, 256 / n_domains));
    sph_status st = SPH_OK;
    b->la_host = la;
    if ((st = upload_table(b->d_ca, ca, b->stream)) != SPH_OK || (st = upload_table(b->d_sa, sa, b->stream)) != SPH_OK ||
        (st = upload_table(b->d_xa, xa, b->stream)) != SPH_OK ||
        (st = upload_table(b->d_fa, fa, b->stream)) != SPH_OK || (st = batch_layout(b)) != SPH_OK ||
        hipHostMalloc(&b->h_res, sizeof(sph_result) * n_domains, hipHostMallocDefault) != hipSuccess) {
        batch_free(b);
        return st != SPH_OK ? st : SPH_ERR_HIP;
    }
    *out = b;
    return SPH_OK;
}

extern "C" sph_status sph_batch_destroy(sph_batch *b) {
    if (!b) return SPH_ERR_ARG;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return SPH_OK;
}

extern "C" sph_status sph_batch_set_mode(sph_batch *b, int32_t mode) {
    if (!b || mode < SPH_BATCH_KERNELS || mode > SPH_BATCH_GRAPH) return SPH_ERR_ARG;
    b->mode = mode;
    return SPH_OK;
}

extern "C" sph_status sph_batch_set_count_block(sph_batch *b, int32_t particles_per_block) {
    if (!b || particles_per_block < 256 || particles_per_block > (1 << 20)) return SPH_ERR_ARG;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->count_ppb = particles_per_block;
    return batch_layout(b);
}

extern "C" sph_status sph_batch_set_gather(sph_batch *b, int32_t runs_per_block) {
    if (!b || runs_per_block < 1 || runs_per_block > kMaxRunsPerBlock) return SPH_ERR_ARG;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->cls_rpb = runs_per_block;
    return batch_layout(b);
}

extern "C" sph_status sph_batch_get_config(sph_batch *b, int32_t *mode, int32_t *particles_per_block,
                                           int32_t *runs_per_block) {
    if (!b) return SPH_ERR_ARG;
    if (mode) *mode = b->mode;
    if (particles_per_block) *particles_per_block = b->count_ppb;
    if (runs_per_block) *runs_per_block = b->cls_rpb;
    return SPH_OK;
}

extern "C" sph_status sph_batch_step(sph_batch *b) {
    if (!b) return SPH_ERR_ARG;
    for (size_t d = 0; d < b->doms.size(); ++d)  // a member redefined since: stale tables, launch nothing
        if (b->doms[d]->layout_gen != b->gens[d]) return SPH_ERR_STATE;
    if (b->mode == SPH_BATCH_KERNELS) return batch_enqueue(b);
    return sph_batch_graph_launch(b);
}

extern "C" sph_status sph_batch_graph_capture(sph_batch *b) {
    if (!b) return SPH_ERR_ARG;
    for (size_t d = 0; d < b->doms.size(); ++d)
        if (b->doms[d]->layout_gen != b->gens[d]) return SPH_ERR_STATE;
    batch_drop_graph(b);
    b->mode = SPH_BATCH_GRAPH;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const sph_status st = batch_enqueue(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != SPH_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != SPH_OK ? st : SPH_ERR_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        batch_drop_graph(b);
        return SPH_ERR_HIP;
    }
    return SPH_OK;
}

extern "C" sph_status sph_batch_graph_launch(sph_batch *b) {
    if (!b) return SPH_ERR_ARG;
    for (size_t d = 0; d < b->doms.size(); ++d)
        if (b->doms[d]->layout_gen != b->gens[d]) return SPH_ERR_STATE;
    if (!b->exec) HIP_CHECKED(sph_batch_graph_capture(b));
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    return SPH_OK;
}

extern "C" sph_status sph_batch_profile_enable(sph_batch *b, int32_t on) {
    if (!b) return SPH_ERR_ARG;
    if (on && b->prof_ev.empty()) {
        b->prof_ev.resize(2 * kProfSlots);
        b->prof_phase.resize(kProfSlots);
        for (auto &e : b->prof_ev)
            if (hipEventCreate(&e) != hipSuccess) return SPH_ERR_HIP;
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->prof_used = 0;
    for (int i = 0; i < kBatchPhases; ++i) {
        b->prof_ms[i] = 0.0;
        b->prof_n[i] = 0;
    }
    b->prof_on = on != 0;
    return SPH_OK;
}

extern "C" sph_status sph_batch_profile_read(sph_batch *b, double ms[5], int64_t launches[5], int32_t reset) {
    if (!b) return SPH_ERR_ARG;
    for (size_t s = 0; s < b->prof_used; ++s) {
        float t = 0.0f;
        if (hipEventSynchronize(b->prof_ev[2 * s + 1]) == hipSuccess &&
            hipEventElapsedTime(&t, b->prof_ev[2 * s], b->prof_ev[2 * s + 1]) == hipSuccess) {
            b->prof_ms[b->prof_phase[s]] += t;
            b->prof_n[b->prof_phase[s]] += 1;
        }
    }
    b->prof_used = 0;
    for (int i = 0; i < kBatchPhases; ++i) {
        if (ms) ms[i] = b->prof_ms[i];
        if (launches) launches[i] = b->prof_n[i];
        if (reset) {
            b->prof_ms[i] = 0.0;
            b->prof_n[i] = 0;
        }
    }
    return SPH_OK;
}

extern "C" sph_status sph_batch_results(sph_batch *b, sph_result *out) {
    if (!b || !out) return SPH_ERR_ARG;
    for (size_t d = 0; d < b->doms.size(); ++d)
        HIP_TRY(hipMemcpyAsync(&b->h_res[d], b->doms[d]->d_result, sizeof(sph_result), hipMemcpyDeviceToHost,
                               b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t d = 0; d < b->doms.size(); ++d) out[d] = b->h_res[d];
    return SPH_OK;
}

// Autotuner: times `trials` real steps of every candidate and keeps the fastest:
// first launch mode x particles per count block, then, at the best of those, the
// cover runs per classify workgroup (the gather schedule).  Steps during tuning
// are genuine updates; once a state has been updated, further updates of
// unchanged positions change nothing.  With a cache path, the choice is read from
// / appended to a text file keyed by device, domain count and total capacity.
extern "C" sph_status sph_batch_tune(sph_batch *b, int32_t trials, const char *cache_path, int32_t *mode_out,
                                     int32_t *ppb_out, double *ms_out) {
    if (!b || trials < 1) return SPH_ERR_ARG;
    int64_t total = 0;
    for (const Parts &p : b->parts) total += p.capacity;
    char key[160];
    hipDeviceProp_t prop{};
    HIP_TRY(hipGetDeviceProperties(&prop, b->doms[0]->device));
    std::snprintf(key, sizeof(key), "%s nd=%zu cap=%lld", prop.gcnArchName, b->doms.size(), (long long)total);
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[256];
            int m = -1, ppb = 0, rpb = 0;
            double ms = 0;
            while (std::fgets(line, sizeof(line), f)) {
                char k2[160];
                int mm, pp2, rr;
                double t;
                if (std::sscanf(line, "%159[^|]|%d|%d|%d|%lf", k2, &mm, &pp2, &rr, &t) == 5 && std::strcmp(k2, key) == 0) {
                    m = mm;
                    ppb = pp2;
                    rpb = rr;
                    ms = t;
                }
            }
            std::fclose(f);
            if (m >= 0 && rpb >= 1 && rpb <= kMaxRunsPerBlock) {
                b->mode = m;
                b->count_ppb = ppb;
                b->cls_rpb = rpb;
                HIP_CHECKED(batch_layout(b));
                if (mode_out) *mode_out = m;
                if (ppb_out) *ppb_out = ppb;
                if (ms_out) *ms_out = ms;
                return SPH_OK;
            }
        }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto time_config = [&](int mode, int ppb, int rpb, double &ms_step) -> sph_status {
        b->mode = mode;
        if (ppb != b->count_ppb || rpb != b->cls_rpb) {
            b->count_ppb = ppb;
            b->cls_rpb = rpb;
            HIP_CHECKED(batch_layout(b));
        }
        for (int w = 0; w < 2; ++w) HIP_CHECKED(sph_batch_step(b));
        HIP_TRY(hipEventRecord(e0, b->stream));
        for (int t = 0; t < trials; ++t) HIP_CHECKED(sph_batch_step(b));
        HIP_TRY(hipEventRecord(e1, b->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms_step = ms / trials;
        return SPH_OK;
    };
    const int ppbs[] = {1024, 2048, 4096, 8192};
    const int rpbs[] = {1, 2, 3, 4, 6, 8};
    double best = 1e30;
    int best_mode = b->mode, best_ppb = b->count_ppb, best_rpb = b->cls_rpb;
    for (int mode = SPH_BATCH_KERNELS; mode <= SPH_BATCH_GRAPH; ++mode)
        for (int ppb : ppbs) {
            double ms = 0;
            HIP_CHECKED(time_config(mode, ppb, best_rpb, ms));
            if (ms < best) {
                best = ms;
                best_mode = mode;
                best_ppb = ppb;
            }
        }
    for (int rpb : rpbs) {
        if (rpb == best_rpb) continue;
        double ms = 0;
        HIP_CHECKED(time_config(best_mode, best_ppb, rpb, ms));
        if (ms < best) {
            best = ms;
            best_rpb = rpb;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->mode = best_mode;
    b->count_ppb = best_ppb;
    b->cls_rpb = best_rpb;
    HIP_CHECKED(batch_layout(b));
    if (cache_path)
        if (FILE *f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s|%d|%d|%d|%.6f\n", key, best_mode, best_ppb, best_rpb, best);
            std::fclose(f);
        }
    if (mode_out) *mode_out = best_mode;
    if (ppb_out) *ppb_out = best_ppb;
    if (ms_out) *ms_out = best;
    return SPH_OK;
}
