// trace.hip -- closest-hit / any-hit traversal kernels and their entry points
// (the per-ray closest hit, any hit and miss outcomes of the paper's
// section 1).  The traversal itself is in trace_core.h.
#include <atomic>
#include <mutex>

#include "trace_core.h"

namespace {

// Results of finished rays are gathered per 64-ray packet in LDS and written
// out packet by packet (one coalesced store per output array), instead of one
// scattered store per ray and array whenever a ray finishes.  Each wave keeps
// a ring of kStageSlots packets; a packet's slot is claimed when its first
// ray is taken, filled as its rays finish (a bit per ray in the slot's mask),
// and written out when all its rays are in.  A packet that still has a ray in
// flight when its slot is needed again (a straggler) is written out as far as
// it got; its late rays then store their results directly.
constexpr int kStageSlots = 4;
constexpr uint32_t kClaimMin = 16;  // packets per wave from which a launch claims its last quarter
template <bool ANY, int MODE>
struct StageShape {
    // words per ray: closest hit (inst, prim); any hit (occluded, inst, prim);
    // render closest hit (t, record, slot); render any hit (occluded)
    static constexpr int K = MODE == rgt::kCounts ? 0
                             : MODE == rgt::kRender ? (ANY ? 1 : 3)
                                                    : (ANY ? 3 : 2);
};
// LDS bytes per wave of the staging ring
template <int K>
constexpr size_t stage_wave_bytes() {
    return (size_t)kStageSlots * (K * 64 * 4 + 16);  // words, then mask, owner and packet per slot
}
// Orders one wave's LDS accesses across lanes: a compiler fence at
// wavefront scope and a wave barrier (the LDS serves a wave's accesses in
// order).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Persistent traversal: each wave walks its own sequence of 64-ray packets,
// and lanes whose ray has finished take the next rays of that sequence
// together, once at least `refill` lanes are idle.  Rays of a packet stay
// neighbours, and no lane idles while work is left.  The sequence: first the
// wave's share of about three quarters of the packets, interleaved (packets
// wave, wave + waves, ...: the waves of a workgroup run neighbouring packets
// at the same time and share their nodes in the caches), then packets
// claimed one at a time from the launch's counter (a.work), so that waves
// that drew cheap packets take more and all run out of work together (Aila &
// Laine 2009).  Each claim is issued one packet ahead, so its latency
// overlaps traversal; the first is issued at the start.  a.work[0] counts
// the claims, a.work[1] the waves that have left; the last wave to leave
// clears both for the next launch that uses them (every wave waits for its
// memory operations first, so no claim of this launch can land after that).
// Only long launches claim: in a short one the counter's traffic at the
// start and at the end costs more than the imbalance it removes, and every
// packet goes out interleaved.
template <int W, bool ANY, int MODE, bool OPT>
__global__ void __launch_bounds__(rgt::kThreads) k_trace(RgTraceArgs a, int refill, int lds_depth, int leaf_batch,
                                                         int inst_batch) {
    constexpr int K = StageShape<ANY, MODE>::K;
    extern __shared__ uint32_t lds_stack[];  // lds_depth * kThreads stack entries, then the staging rings
    const int lane = threadIdx.x & 63;
    // a device count never exceeds the launch size (the queue capacity)
    // (a launch holds fewer than 2^31 rays: positions and indices fit 32 bits)
    const uint32_t n = (uint32_t)(a.count ? ((int64_t)*a.count < a.n ? (int64_t)*a.count : a.n) : a.n);
    const uint32_t n_packets = (n + 63) >> 6;
    // wave-uniform values kept in scalar registers
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave in the block
    const uint32_t wave = blockIdx.x * (rgt::kThreads / 64) + wib;
    const uint32_t n_waves = gridDim.x * (rgt::kThreads / 64);
    // long launches (kClaimMin packets per wave or more): interleaved packets
    // per wave, the packets they cover, the rest claimed; shorter ones take
    // every packet interleaved and touch no counter
    const bool claims = n_packets >= kClaimMin * n_waves;
    const uint32_t n_fixed = claims ? (3u * n_packets) / (4u * n_waves) : ~0u;
    const uint32_t n_static = claims ? n_fixed * n_waves : n_packets;
    rgt::Tracer<W, ANY, MODE, OPT> tr;
    tr.tlas_nodes = reinterpret_cast<const RgNode<W> *>(a.nodes);
    tr.recs = a.recs;
    uint32_t priv_stack[rgt::kPrivStack];
    tr.st.lds = (uint32_t RG_LDS *)&lds_stack[threadIdx.x];
    tr.st.priv = priv_stack;
    tr.st.n_lds = lds_depth;
    if (OPT) {
        tr.call_cull = a.ray_flags & (RG_RAY_CULL_BACK | RG_RAY_CULL_FRONT);
        tr.rmask = a.mask;
    }
    // this wave's staging ring: words [slot][K][64], mask [slot], owner
    // [slot] (packet number q in the wave's sequence, ~0u: free), packet
    // [slot] (the launch's packet that q stands for)
    char RG_LDS *ring = (char RG_LDS *)&lds_stack[lds_depth * rgt::kThreads] + wib * stage_wave_bytes<K>();
    uint32_t RG_LDS *sw = (uint32_t RG_LDS *)ring;
    uint64_t RG_LDS *smask = (uint64_t RG_LDS *)(ring + kStageSlots * K * 64 * 4);
    uint32_t RG_LDS *sown = (uint32_t RG_LDS *)(ring + kStageSlots * (K * 64 * 4 + 8));
    uint32_t RG_LDS *spkt = (uint32_t RG_LDS *)(ring + kStageSlots * (K * 64 * 4 + 12));
    if (lane < kStageSlots) {
        sown[lane] = ~0u;
        smask[lane] = 0ull;
        spkt[lane] = ~0u;
    }
    wave_sync();
    uint32_t ahead = 0u;  // lane 0: the claimed packet for the wave's next claimed packet number
    if (lane == 0 && n_static < n_packets) ahead = atomicAdd(a.work, 1u);
    uint32_t q_end = 0u;   // packet numbers below this one have their packet (uniform)
    bool out_of_work = false;  // a claim came back past the last packet (uniform)
    uint32_t next = 0;   // position in this wave's ray sequence (the same in all lanes)
    uint32_t ray_j = 0;  // position of this lane's ray in the sequence
    uint32_t ray_i = 0;  // index of this lane's ray in the launch
    bool has = false;
    // A finished ray's result stays in its lane until the next refill round
    // (or the wave's end), where all finished lanes place theirs together.
    bool pend = false;
    uint32_t stalled = 0u;  // rounds since a ray of this wave last finished or was taken
    auto word = [&](int w) -> uint32_t {
        if (MODE == rgt::kRender && !ANY) {
            // the render's closest hits carry their float32 t to shading
            if (w == 0) return __float_as_uint(tr.found ? tr.best : INFINITY);
            return w == 1 ? tr.h.inst : tr.h.prim;
        }
        if (ANY) return w == 0 ? (tr.found ? 1u : 0u) : (w == 1 ? tr.h.inst : tr.h.prim);
        return w == 0 ? tr.h.inst : tr.h.prim;
    };
    // word w of a ray goes to ...
    auto store = [&](int w, uint32_t i, uint32_t v) {
        if (MODE == rgt::kRender && !ANY) {
            if (w == 0) { if (a.t) a.t[i] = __uint_as_float(v); }
            else if (w == 1) { if (a.inst) a.inst[i] = v; }
            else if (a.prim) a.prim[i] = v;
        } else if (ANY) {
            if (w == 0) { if (a.occluded) a.occluded[i] = (uint8_t)v; }
            else if (w == 1) { if (a.inst) a.inst[i] = v; }
            else if (a.prim) a.prim[i] = v;
        } else {
            if (w == 0) { if (a.inst) a.inst[i] = v; }
            else if (a.prim) a.prim[i] = v;
        }
    };
    auto write_result = [&]() {  // the visit counts: stored directly
        const uint64_t i = ray_i;
        a.counts[3 * i] = tr.h.n_nodes;
        a.counts[3 * i + 1] = tr.h.n_tris;
        a.counts[3 * i + 2] = tr.h.n_inst;
    };
    // Writes slot s's staged rays, those of launch packet pkt (all lanes
    // together; uniform arguments).
    auto flush_slot = [&](int s, uint32_t pkt, uint64_t m) {
        if ((m >> lane) & 1ull) {
            const uint32_t i = pkt * 64 + lane;
#pragma unroll
            for (int w = 0; w < K; ++w) store(w, i, sw[(s * K + w) * 64 + lane]);
        }
    };
    // Rays of launch packet pkt: 64, fewer for the batch's last packet.
    auto full_mask = [&](uint32_t pkt) -> uint64_t {
        const uint32_t first = pkt * 64;
        const uint32_t cnt = n - first < 64u ? n - first : 64u;
        return cnt >= 64u ? ~0ull : ((1ull << cnt) - 1ull);
    };
    // Places the results of lanes with `pend` (all lanes together), then
    // writes out complete packets; with `all`, writes out every slot.
    auto place = [&](bool all) {
        const uint32_t q = ray_j >> 6;
        const int s = (int)(q & (kStageSlots - 1));
        if (pend) {
            if (sown[s] == q) {
#pragma unroll
                for (int w = 0; w < K; ++w) sw[(s * K + w) * 64 + (ray_j & 63)] = word(w);
                __hip_atomic_fetch_or(&smask[s], 1ull << (ray_j & 63), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
            } else {
                const uint32_t i = ray_i;  // a straggler's packet left the ring
#pragma unroll
                for (int w = 0; w < K; ++w) store(w, i, word(w));
            }
            pend = false;
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < kStageSlots; ++k) {
            const uint32_t o = __builtin_amdgcn_readfirstlane(sown[k]);
            if (o == ~0u) continue;
            const uint64_t m = smask[k];
            const uint64_t mu = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
                                __builtin_amdgcn_readfirstlane((uint32_t)m);
            const uint32_t pkt = __builtin_amdgcn_readfirstlane(spkt[k]);
            if (all || mu == full_mask(pkt)) {
                flush_slot(k, pkt, mu);
                wave_sync();
                if (lane == 0) {
                    sown[k] = ~0u;
                    smask[k] = 0ull;
                }
                wave_sync();
            }
        }
    };
    // Gives the packet numbers whose first position is among [p0, p0 + cnt)
    // of the sequence their launch packets (an interleaved one, else the
    // claimed one ahead, then the next claim issued) and their slots (all
    // lanes together).
    auto claim = [&](uint32_t p0, uint32_t cnt) {
        for (uint32_t q = (p0 + 63) >> 6; q * 64 < p0 + cnt; ++q) {
            if (out_of_work) break;
            uint32_t pkt = q < n_fixed ? wave + q * n_waves : n_static;
            if (pkt >= n_static) {
                if (n_static >= n_packets) {
                    out_of_work = true;
                    break;
                }
                pkt = n_static + __builtin_amdgcn_readfirstlane(ahead);
                if (pkt >= n_packets) {
                    out_of_work = true;
                    break;
                }
                if (lane == 0) ahead = atomicAdd(a.work, 1u);
            }
            const int k = (int)(q & (kStageSlots - 1));
            const uint32_t o = __builtin_amdgcn_readfirstlane(sown[k]);
            if (K > 0 && o != ~0u) {  // a straggler: write out what it has
                const uint64_t m = smask[k];
                const uint64_t mu = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
                                    __builtin_amdgcn_readfirstlane((uint32_t)m);
                flush_slot(k, __builtin_amdgcn_readfirstlane(spkt[k]), mu);
                wave_sync();
            }
            if (lane == 0) {
                sown[k] = (uint32_t)q;
                smask[k] = 0ull;
                spkt[k] = pkt;
            }
            wave_sync();
            q_end = q + 1;
        }
    };
    while (true) {
        // every ballot and every update of `next` below is executed by all
        // lanes together, so `next` stays uniform across the wave
        const uint64_t need = __ballot(!has);
        const int n_need = __popcll(need);
        bool took = false;
        if (n_need >= refill) {
            if (K > 0) place(false);
            claim(next, (uint32_t)n_need);
            if (!has) {
                // this lane's rank among the idle lanes
                const uint32_t j = next + __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                const uint32_t pkt = (j >> 6) < q_end ? spkt[(j >> 6) & (kStageSlots - 1)] : ~0u;
                const uint32_t idx = pkt * 64 + (j & 63);
                if (pkt < n_packets && idx < n) {
                    if (K == 0 && pend) write_result();
                    rgt::Ray R;
                    R.o[0] = a.ray[0][idx]; R.o[1] = a.ray[1][idx]; R.o[2] = a.ray[2][idx];
                    R.d[0] = a.ray[3][idx]; R.d[1] = a.ray[4][idx]; R.d[2] = a.ray[5][idx];
                    R.tmin = a.ray[6][idx];
                    R.tmax = a.ray[7][idx];
                    ray_j = j;
                    ray_i = idx;
                    if (MODE == rgt::kRender && a.ray_job) {  // only frames carry per-ray top levels
                        const RgTlasRef J = a.jobs[a.ray_job[idx]];
                        tr.tlas_nodes = reinterpret_cast<const RgNode<W> *>(J.nodes);
                        tr.recs = J.recs;
                    }
                    has = tr.begin(R);
                    if (OPT) tr.rmask = a.ray_mask ? (uint32_t)a.ray_mask[idx] : a.mask;
                    pend = !has;  // empty interval: a miss without traversal
                    took = true;
                }
            }
            next += n_need;
        }
        if (__ballot(has) == 0) {
            // no lane holds a ray after a refill attempt of all 64 lanes: the
            // wave is done once its claims have run past the last packet
            if (out_of_work) break;
            continue;
        }
        // Which kinds of unit run this round: inner nodes whenever a lane
        // has one; leaves and instance entries (each a long stretch of code
        // that runs for the whole wave if any lane needs it) once enough
        // lanes wait for one, or when nothing else is left.  A lane that
        // waits keeps its state; every round runs at least one kind present.
        const uint32_t my = has ? tr.kind() : 0u;
        const int n_inner = __popcll(__ballot(my == rgt::kUnitInner));
        const int n_leaf = __popcll(__ballot(my == rgt::kUnitLeaf));
        const int n_inst = __popcll(__ballot(my == rgt::kUnitInst));
        uint32_t run = n_inner ? rgt::kUnitInner : 0u;
        if (n_leaf && (n_leaf >= leaf_batch || n_inner == 0)) run |= rgt::kUnitLeaf;
        if (n_inst && (n_inst >= inst_batch || run == 0)) run |= rgt::kUnitInst;
        const bool fin = (run & my) != 0u && tr.step();  // my == 0 for lanes without a ray
        if (fin) {
            has = false;
            pend = true;
        }
        // loop bound: a wave whose rays stop finishing (only a corrupt
        // hierarchy can make a traversal cycle) gives up on them
        if (__ballot(fin || took) != 0ull) {
            stalled = 0u;
        } else if (++stalled > rgt::kMaxSteps) {
            if (has) pend = true;
            has = false;
        }
    }
    if (K > 0) place(true);
    else if (pend) write_result();
    if (claims && lane == 0) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's claims have come back
        if (atomicAdd(a.work + 1, 1u) == n_waves - 1u) {
            atomicExch(a.work, 0u);
            atomicExch(a.work + 1, 0u);
        }
    }
}

// The reported hit in double precision.  The traversal decides in float32
// which triangle a ray hits (the decisions are the watertight ones); float32
// cannot give that triangle's t to 1e-5 of its value when the ray starts
// close to it (a secondary ray leaving a surface: the vertex offsets cancel
// to a few bits).  So the trace calls recompute t, u and v of the chosen
// triangle from the exact float32 inputs: the triangle's object-space
// vertices mapped to world space with the instance's matrix, and the world
// ray, intersected with Moller-Trumbore (Moller & Trumbore 1997) in double.
// t is parametric in the ray, so the world-space t is the object-space t.
// One thread per ray; reads the ray and the traversal's (inst, prim) in
// order, gathers the matrix, the triangle's leaf slot and the triangle.
struct RefineArgs {
    const float *ray[8];
    int64_t n;
    const uint32_t *inst, *prim;  // the traversal's result (input indices)
    float *t, *u, *v;             // outputs, nullable
    const RgInst *recs;
    const uint32_t *rec_of;       // record of each input instance
    const float *xf;              // object -> world matrices, input order
};

__global__ void __launch_bounds__(256) k_refine(RefineArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t in = a.inst[i];
    float t = INFINITY, u = 0.0f, v = 0.0f;
    if (in != RG_MISS) {
        const uint32_t p = a.prim[i];
        const RgBlasHdr *H = reinterpret_cast<const RgBlasHdr *>(a.recs[a.rec_of[in]].hdr);
        const uint32_t slot = reinterpret_cast<const uint32_t *>(H->slots)[p];
        const RgTri tri = reinterpret_cast<const RgTri *>(H->tris)[slot];
        const float *M = a.xf + 12 * (uint64_t)in;
        double P[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                P[k][r] = (double)M[4 * r] * tri.v[3 * k] + (double)M[4 * r + 1] * tri.v[3 * k + 1] +
                          (double)M[4 * r + 2] * tri.v[3 * k + 2] + (double)M[4 * r + 3];
        const double o[3] = {a.ray[0][i], a.ray[1][i], a.ray[2][i]};
        const double d[3] = {a.ray[3][i], a.ray[4][i], a.ray[5][i]};
        const float tmin = a.ray[6][i], tmax = a.ray[7][i];
        double e1[3], e2[3], s[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            e1[r] = P[1][r] - P[0][r];
            e2[r] = P[2][r] - P[0][r];
            s[r] = o[r] - P[0][r];
        }
        const double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
        const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
        t = tmin;  // a hit whose plane is exactly parallel to the ray in double: grazing, reported at tmin
        if (det != 0.0) {
            const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
            const double r = 1.0 / det;
            const double uu = (s[0] * pv[0] + s[1] * pv[1] + s[2] * pv[2]) * r;
            const double vv = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * r;
            const double tt = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * r;
            // the hit was found inside the triangle and the interval by the
            // float32 test: keep the refined values there too
            t = fminf(fmaxf((float)tt, tmin), tmax);
            u = fminf(fmaxf((float)uu, 0.0f), 1.0f);
            v = fminf(fmaxf((float)vv, 0.0f), 1.0f);
        }
    }
    if (a.t) a.t[i] = t;
    if (a.u) a.u[i] = u;
    if (a.v) a.v[i] = v;
}

// Launch parameters per family of calls (RG_TUNE_*): refill threshold,
// resident waves per CU, LDS stack entries per lane, lanes waiting at leaves
// / instance entries before a wave runs that code.  Incoherent ray batches
// gain from waiting lanes; the coherent rays of frames do not.  Every launch
// takes at most the waves its variant keeps resident: the closest-hit
// variant of frames fits 4 per SIMD, the any-hit one 5 at widths 2 and 4.
// The engine runs a pass's any-hit launch beside the next pass's
// closest-hit launch, and there the any-hit launch's fifth wave per SIMD
// pays; single frames and batches gain nothing from it.  The engine's
// passes mix the rays of many frames and depths: like incoherent batches
// they gain from lanes waiting at leaves and instance entries, and from
// refilling later (a measured sweep: refill 20..28 with leaf batch 12 best).
rg_trace_tune g_tune[RG_TUNE_SCOPES] = {
    {16, 20, 16, 12, 6},  // RG_TUNE_TRACE: rg_trace_closest / any / counts (5 waves per SIMD fit)
    {8, 16, 16, 1, 1},    // RG_TUNE_FRAME: rg_render, rg_batch_render
    {24, 20, 16, 12, 6},  // RG_TUNE_ENGINE: rg_engine_step
};

}  // namespace

int rg_cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus = c;
    }
    return cus;
}

namespace {

unsigned persistent_blocks(int64_t n, int waves_per_cu) {
    int64_t want = (int64_t)rg_cu_count() * waves_per_cu / (rgt::kThreads / 64);
    int64_t need = rg_blocks(n, rgt::kThreads);
    return (unsigned)(need < want ? need : want);
}

// A persistent launch takes no more blocks than the kernel variant can keep
// resident (its registers and LDS decide how many fit on a CU): blocks
// beyond that would wait for a resident one to finish and start its share
// of the sequence late.
template <class Kernel>
unsigned resident_cap(Kernel kernel, unsigned blocks, size_t shm) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, rgt::kThreads, shm) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        return blocks;
    }
    const unsigned cap = (unsigned)per_cu * (unsigned)rg_cu_count();
    return blocks < cap ? blocks : cap;
}

template <int W, bool ANY, int MODE, bool OPT>
void launch_one(const RgTraceArgs &a, hipStream_t st, unsigned blocks, size_t shm, const rg_trace_tune &t) {
    auto kernel = k_trace<W, ANY, MODE, OPT>;
    blocks = resident_cap(kernel, blocks, shm);
    kernel<<<blocks, rgt::kThreads, shm, st>>>(a, t.refill, t.lds_depth, t.leaf_batch, t.inst_batch);
}

template <int W, bool OPT>
void launch_mode(bool any, int mode, const RgTraceArgs &a, hipStream_t st, unsigned blocks, size_t shm,
                 const rg_trace_tune &t) {
    if (mode == rgt::kCounts) {
        if (any) launch_one<W, true, rgt::kCounts, OPT>(a, st, blocks, shm, t);
        else launch_one<W, false, rgt::kCounts, OPT>(a, st, blocks, shm, t);
    } else if (mode == rgt::kRender) {
        if (any) launch_one<W, true, rgt::kRender, OPT>(a, st, blocks, shm, t);
        else launch_one<W, false, rgt::kRender, OPT>(a, st, blocks, shm, t);
    } else {
        if (any) launch_one<W, true, rgt::kClosest, OPT>(a, st, blocks, shm, t);
        else launch_one<W, false, rgt::kClosest, OPT>(a, st, blocks, shm, t);
    }
}

// Packet counters of the persistent traversal: each launch takes the next
// of kWorkSlots pairs of device words (so launches in flight on different
// streams count apart; a launch captured into a graph keeps a pair of its
// own); the launch leaves its pair cleared (zero from the module's load on),
// so a graph that captured a launch can replay it.  The
// array lives in the library's code object, one copy per device; its device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current.
constexpr uint32_t kWorkSlots = 4096;     // handed out in turn to launches
constexpr uint32_t kCaptureSlots = 1024;  // each launch captured into a graph keeps one of its own
constexpr int kMaxDevices = 64;
std::mutex g_work_mu;
uint32_t *g_work_ptr[kMaxDevices] = {};
std::atomic<uint32_t> g_work_seq{0}, g_capture_seq{0};

}  // namespace

static __device__ __align__(256) uint32_t work_counters[2 * (kWorkSlots + kCaptureSlots)];

namespace {

rg_status work_counter(hipStream_t st, uint32_t **out) {
    int dev = 0;
    RG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return RG_ERR_UNSUPPORTED;
    uint32_t *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_work_mu);
        if (!g_work_ptr[dev]) {
            void *p = nullptr;
            RG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(work_counters)));
            if (!p) return RG_ERR_HIP;
            g_work_ptr[dev] = static_cast<uint32_t *>(p);
        }
        base = g_work_ptr[dev];
    }
    // a launch being captured gets a pair no other launch uses (the graph
    // replays it again and again); others take the next pair of the ring
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    RG_HIP(hipStreamIsCapturing(st, &cs));
    const uint32_t slot = cs == hipStreamCaptureStatusActive
                              ? kWorkSlots + g_capture_seq.fetch_add(1u, std::memory_order_relaxed) % kCaptureSlots
                              : g_work_seq.fetch_add(1u, std::memory_order_relaxed) % kWorkSlots;
    *out = base + 2 * slot;
    return RG_OK;
}

template <int W>
rg_status launch_w(bool any, int mode, const RgTraceArgs &a, hipStream_t st, const rg_trace_tune &t) {
    unsigned blocks = persistent_blocks(a.n, t.waves_per_cu);
    // the traversal stacks, then one staging ring per wave
    const int K = mode == rgt::kCounts ? 0 : (mode == rgt::kRender ? (any ? 1 : 3) : (any ? 3 : 2));
    size_t shm = (size_t)t.lds_depth * rgt::kThreads * sizeof(uint32_t) +
                 (rgt::kThreads / 64) * (size_t)kStageSlots * (K * 64 * 4 + 16);
    if (a.opt) launch_mode<W, true>(any, mode, a, st, blocks, shm, t);
    else launch_mode<W, false>(any, mode, a, st, blocks, shm, t);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

bool rays_ok(const rg_rays &r) {
    return r.ox && r.oy && r.oz && r.dx && r.dy && r.dz && r.tmin && r.tmax;
}

void fill_rays(RgTraceArgs &a, const rg_rays &r) {
    a.ray[0] = r.ox; a.ray[1] = r.oy; a.ray[2] = r.oz;
    a.ray[3] = r.dx; a.ray[4] = r.dy; a.ray[5] = r.dz;
    a.ray[6] = r.tmin; a.ray[7] = r.tmax;
}

bool set_opts(RgTraceArgs &a, const rg_trace_opts *o) {
    if (!o) return true;
    if ((o->flags & ~(RG_RAY_CULL_BACK | RG_RAY_CULL_FRONT)) || o->mask > 0xFFu) return false;
    a.ray_flags = o->flags;
    a.mask = o->mask;
    a.ray_mask = o->ray_mask;
    a.opt = o->flags != 0u || o->mask != RG_INST_MASK_ALL || o->ray_mask != nullptr;
    return true;
}

// rays per trace call: the kernels keep a ray's index and its position in
// the wave's sequence in 32 bits
constexpr int64_t kMaxRays = 0x7FFFFFFFll;

bool tlas_ok(const rg_tlas *t) {
    return t && t->buf && t->n_inst >= 1 && (t->width == 2 || t->width == 4 || t->width == 8);
}

// t, u and v are computed from the hit's identity: asking for any of them
// needs inst and prim too.
bool hits_ok(const rg_hits &h) { return !(h.t || h.u || h.v) || (h.inst && h.prim); }

rg_status refine(const rg_tlas *tlas, const RgTraceArgs &a, const rg_hits &h, hipStream_t st) {
    if (!(h.t || h.u || h.v)) return RG_OK;
    RefineArgs r;
    for (int c = 0; c < 8; ++c) r.ray[c] = a.ray[c];
    r.n = a.n;
    r.inst = h.inst;
    r.prim = h.prim;
    r.t = h.t;
    r.u = h.u;
    r.v = h.v;
    r.recs = a.recs;
    r.rec_of = (const uint32_t *)((const char *)tlas->buf + tlas->rec_off);
    r.xf = (const float *)((const char *)tlas->buf + tlas->xf_off);
    k_refine<<<rg_blocks(a.n, 256), 256, 0, st>>>(r);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

}  // namespace

bool rg_trace_depth_ok(const rg_tlas *t) {
    int64_t need = (int64_t)(t->width - 1) * (t->depth + t->max_blas_depth) + 1;
    return need <= rgt::kStackCap;
}

rg_status rg_trace_launch(int width, bool any, int mode, const RgTraceArgs &a_in, hipStream_t st, int scope) {
    if (a_in.n <= 0) return RG_OK;
    if (scope < 0 || scope >= RG_TUNE_SCOPES) return RG_ERR_INVALID_ARG;
    if (width != 2 && width != 4 && width != 8) return RG_ERR_INVALID_ARG;
    const rg_trace_tune t = g_tune[scope];
    RgTraceArgs a = a_in;
    rg_status r = work_counter(st, &a.work);
    if (r != RG_OK) return r;
    if (width == 2) return rg_debug_done(launch_w<2>(any, mode, a, st, t), st);
    if (width == 4) return rg_debug_done(launch_w<4>(any, mode, a, st, t), st);
    return rg_debug_done(launch_w<8>(any, mode, a, st, t), st);
}

extern "C" {

rg_status rg_trace_tuning(int32_t scope, const rg_trace_tune *set, rg_trace_tune *get) {
    if (scope < 0 || scope >= RG_TUNE_SCOPES) return RG_ERR_INVALID_ARG;
    if (set) {
        if (set->refill < 1 || set->refill > 64 || set->waves_per_cu < 4 || set->waves_per_cu > 64 ||
            set->lds_depth < 8 || set->lds_depth > rgt::kMaxLdsStack || set->leaf_batch < 1 ||
            set->leaf_batch > 64 || set->inst_batch < 1 || set->inst_batch > 64)
            return RG_ERR_INVALID_ARG;
        g_tune[scope] = *set;
    }
    if (get) *get = g_tune[scope];
    return RG_OK;
}

rg_status rg_trace_closest(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, void *stream) {
    return rg_trace_closest_ex(tlas, rays, n, out, nullptr, stream);
}

rg_status rg_trace_any(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded, const rg_hits *found,
                       void *stream) {
    return rg_trace_any_ex(tlas, rays, n, occluded, found, nullptr, stream);
}

rg_status rg_trace_closest_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, rg_hits out, const rg_trace_opts *opts,
                              void *stream) {
    if (!tlas_ok(tlas) || n < 0 || n > kMaxRays || (n > 0 && !rays_ok(rays)) || !hits_ok(out))
        return RG_ERR_INVALID_ARG;
    RgTraceArgs a = {};
    if (!set_opts(a, opts)) return RG_ERR_INVALID_ARG;
    a.opt = a.opt || tlas->has_inst_flags != 0;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.inst = out.inst;
    a.prim = out.prim;
    const hipStream_t st = (hipStream_t)stream;
    rg_status r = rg_trace_launch(tlas->width, false, rgt::kClosest, a, st, RG_TUNE_TRACE);
    if (r != RG_OK) return r;
    return rg_debug_done(refine(tlas, a, out, st), st);
}

rg_status rg_trace_any_ex(const rg_tlas *tlas, rg_rays rays, int64_t n, uint8_t *occluded, const rg_hits *found,
                          const rg_trace_opts *opts, void *stream) {
    if (!tlas_ok(tlas) || n < 0 || n > kMaxRays || (n > 0 && (!rays_ok(rays) || !occluded)))
        return RG_ERR_INVALID_ARG;
    if (found && !hits_ok(*found)) return RG_ERR_INVALID_ARG;
    RgTraceArgs a = {};
    if (!set_opts(a, opts)) return RG_ERR_INVALID_ARG;
    a.opt = a.opt || tlas->has_inst_flags != 0;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.occluded = occluded;
    if (found) {
        a.inst = found->inst;
        a.prim = found->prim;
    }
    const hipStream_t st = (hipStream_t)stream;
    rg_status r = rg_trace_launch(tlas->width, true, rgt::kClosest, a, st, RG_TUNE_TRACE);
    if (r != RG_OK || !found) return r;
    return rg_debug_done(refine(tlas, a, *found, st), st);
}

rg_status rg_trace_counts(const rg_tlas *tlas, rg_rays rays, int64_t n, int32_t any_hit, uint32_t *counts,
                          void *stream) {
    if (!tlas_ok(tlas) || n < 0 || n > kMaxRays || (n > 0 && (!rays_ok(rays) || !counts)))
        return RG_ERR_INVALID_ARG;
    if (!rg_trace_depth_ok(tlas)) return RG_ERR_UNSUPPORTED;
    if (n == 0) return RG_OK;
    RgTraceArgs a = {};
    a.nodes = (const char *)tlas->buf + tlas->nodes_off;
    a.recs = (const RgInst *)((const char *)tlas->buf + tlas->inst_off);
    fill_rays(a, rays);
    a.n = n;
    a.counts = counts;
    a.opt = tlas->has_inst_flags != 0;
    return rg_trace_launch(tlas->width, any_hit != 0, rgt::kCounts, a, (hipStream_t)stream, RG_TUNE_TRACE);
}

}  // extern "C"
