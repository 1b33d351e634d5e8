// Persistent serving launch: continuous batching of render requests over a resident scene
// (Sec. 4.2, real-time rendering at any viewing distance), executed by one kernel that stays
// on the device for the life of the server.
//
// A job is one batch of requests: the Program of stages that clod_project, clod_bin_sort and
// clod_render_fwd would launch one kernel at a time (projection with the LoD mask, binning,
// blending).  The host writes a job into a ring of slots in pinned host memory and bumps a
// publish counter.  Workgroup 0 (the dispatcher) copies each published job into device memory
// and activates it.  Every other workgroup (a worker) claims blocks ("items") of the open
// stage of the oldest active job that still has unclaimed items, runs them with the same
// block bodies as the per-stage kernels (this file is compiled together with them), and
// counts them done; the worker that completes a stage opens the next, and the one that
// completes a job's last stage writes the job's completion record to host memory.  Stages of
// different jobs interleave freely, so the tail of one job's stage does not idle the device.
//
// Waits are bounded.  Every loop polls the stop flag (raised by the dispatcher when the host
// asks to stop, or by any workgroup on an error) and a deadline on the device's constant-rate
// clock; no workgroup ever waits for another particular workgroup, and a claimed item always
// runs to its end.
//
// Visibility across the per-XCD L2 caches follows the agent-scope memory model, and its
// fences are the expensive part on this device (each one writes back or invalidates an L2;
// they serialise device-wide at tens of ns each).  So a worker fences once per stage it takes
// part in, not per item: it acquires when it enters a stage (before reading the stage's
// arguments and inputs), keeps claiming items of that stage, and releases its items and counts
// them done when the stage has none left to claim.  One wave fences for the workgroup, after a
// barrier (the scoped model makes the other waves' writes visible through it).  Idle workers
// poll one epoch word, bumped whenever a job or a stage opens, instead of the claim words.
#include "project.hip"
#include "sort.hip"
#include "blend.hip"

#include <stddef.h>
#include <string.h>

namespace clod {

hipError_t launch_stage(const Stage& st, hipStream_t s) {
  switch (st.kind) {
    case kStViewSetup: case kStFill: case kStFrustumMax: case kStFold: case kStClassify: case kStProject:
    case kStSelectHist: case kStSelectPick:
      return launch_project_stage(st, s);
    case kStScanReduce: case kStScanPartials: case kStCompact: case kStRadixUp: case kStRadixScan:
    case kStRadixDown: case kStEmitReduce: case kStEmitPartials: case kStEmitOffsets: case kStEmit:
    case kStRanges: case kStTileCount: case kStTileScatter:
      return launch_sort_stage(st, s);
    case kStBlend: case kStReducePairs: case kStLongMask:
      return launch_blend_stage(st, s);
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------- shared state
struct alignas(16) SrvJob {
  uint32_t n_stages, n_views;
  uint64_t seq;
  const unsigned long long* hdr;   // the job's workspace header: D and the overflow flag
  uint64_t reserved;
  clod_view views[kSrvMaxViews];   // read by the job's view-setup stage
  Stage st[kMaxStages];
};

struct SrvDone {
  uint64_t seq1;       // sequence number + 1 of the last job completed in the slot
  uint64_t t_end;      // device clock at its completion
  uint64_t overflow;   // the job's duplicate buffer overflowed (outputs not written)
  uint64_t n_dup;      // tile pairs of the job
  uint64_t t_open[kMaxStages];   // device clock when each stage opened (stage 0: activation)
};

// Pinned host memory (coherent, mapped).
struct SrvHost {
  uint64_t published;   // host: number of jobs published
  uint32_t stop;        // host: 1 asks the server to stop
  uint32_t running;     // device: 1 once the dispatcher runs
  uint64_t t_start;     // device clock when the dispatcher started
  uint64_t heartbeat;   // device clock, refreshed by the dispatcher on every poll
  uint64_t reserved[4];
  SrvDone done[kSrvSlots];
  SrvJob ring[kSrvSlots];
};

// Device memory.  Words written by many workgroups sit on cache lines of their own.
struct alignas(128) SrvSlot {
  unsigned long long claim;   // open stage and claim cursor (claim_word)
  uint32_t done;              // items of the open stage completed
  uint32_t active;            // (sequence number mod 2^32 - 1) + 1 of the job, 0 = free
};
constexpr unsigned long long kStopBit = 1ull << 63;
struct SrvDev {
  alignas(128) unsigned long long epoch;   // bumped when a job or a stage opens; kStopBit: stop
  alignas(128) uint32_t status;            // largest SrvStatus raised
  alignas(128) SrvSlot slot[kSrvSlots];
  SrvJob job[kSrvSlots];
};

// Claim word: stage (8 bits) | log2 of the items per claim (4) | stage items (24) | cursor (28).
constexpr uint32_t kNoStage = 255;
__host__ __device__ constexpr unsigned long long claim_word(uint32_t stage, uint32_t lchunk, uint32_t limit) {
  return ((unsigned long long)stage << 56) | ((unsigned long long)lchunk << 52) | ((unsigned long long)limit << 28);
}
__device__ __forceinline__ uint32_t cw_cursor(unsigned long long w) { return (uint32_t)(w & 0xFFFFFFFull); }
__device__ __forceinline__ uint32_t cw_limit(unsigned long long w) { return (uint32_t)((w >> 28) & 0xFFFFFFull); }
__device__ __forceinline__ uint32_t cw_lchunk(unsigned long long w) { return (uint32_t)((w >> 52) & 15ull); }
__device__ __forceinline__ uint32_t cw_stage(unsigned long long w) { return (uint32_t)(w >> 56); }

// Items per claim: one tile at a time for the blend (tiles come longest first and vary a lot),
// else about one claim per worker, a power of two.  (Fewer, larger claims cost more than they
// save: consecutive blocks of the radix passes and the emission hold most of the real work, so
// concentrating them on few workers lengthens the stage.)
__device__ __forceinline__ uint32_t claim_lchunk(int32_t kind, uint32_t items, uint32_t workers) {
  if (kind == kStBlend) return 0;
  const uint32_t per = items / workers;
  if (per <= 1) return 0;
  const uint32_t l = 31u - (uint32_t)__clz(per);
  return l > 15u ? 15u : l;
}

template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ld_sys_acquire(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class T>
__device__ __forceinline__ void st_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class T>
__device__ __forceinline__ void st_sys_release(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t dev_clock() { return (uint64_t)wall_clock64(); }

__device__ __forceinline__ void raise_stop(SrvDev* D, uint32_t status) {
  atomicMax(&D->status, status);
  __hip_atomic_fetch_or(&D->epoch, kStopBit, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bump_epoch(SrvDev* D) {
  __hip_atomic_fetch_add(&D->epoch, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------- dispatcher
// Wave 0 of workgroup 0.  Copies every newly published job from the host ring into its device
// slot, opens its first stage and activates it; stops on the host's request or the deadline.
__device__ void srv_dispatch(SrvDev* D, SrvHost* H, uint64_t deadline) {
  if (threadIdx.x >= 64) return;
  const uint32_t lane = lane_id();
  const uint32_t workers = gridDim.x - 1;
  if (lane == 0) {
    const uint64_t t = dev_clock();
    st_sys(&H->t_start, t);
    st_sys(&H->heartbeat, t);
    st_sys_release(&H->running, 1u);
  }
  uint64_t next = 0;
  for (;;) {
    const uint64_t now = dev_clock();
    if (lane == 0) st_sys(&H->heartbeat, now);
    if (now > deadline) {
      if (lane == 0) raise_stop(D, kSrvDeadline);
      return;
    }
    if (ld_agent(&D->epoch) & kStopBit) return;   // a worker raised an error
    const uint64_t pub = ld_sys_acquire(&H->published);
    const uint32_t hstop = ld_sys_acquire(&H->stop);
    while (next < pub) {
      const uint32_t slot = (uint32_t)(next % kSrvSlots);
      const SrvJob& src = H->ring[slot];
      const uint32_t ns = src.n_stages, nv = src.n_views;
      if (ld_agent(&D->slot[slot].active) != 0u || src.seq != next || ns < 1 || ns > (uint32_t)kMaxStages ||
          nv > (uint32_t)kSrvMaxViews) {
        if (lane == 0) raise_stop(D, kSrvProtocol);
        return;
      }
      // Eight 16-byte loads per lane in flight per round: the ring is read across the bus.
      const uint32_t nq = (uint32_t)((offsetof(SrvJob, st) + (size_t)ns * sizeof(Stage) + 15) / 16);
      const uint4* s4 = reinterpret_cast<const uint4*>(&src);
      uint4* d4 = reinterpret_cast<uint4*>(&D->job[slot]);
      for (uint32_t q0 = 0; q0 < nq; q0 += 8 * 64) {
        uint4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t q = q0 + (uint32_t)k * 64 + lane;
          if (q < nq) v[k] = s4[q];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t q = q0 + (uint32_t)k * 64 + lane;
          if (q < nq) d4[q] = v[k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0) {
        const uint32_t items = src.st[0].items;
        SrvSlot& S = D->slot[slot];
        atomicExch(&S.done, 0u);
        __hip_atomic_store(&S.active, (uint32_t)(next % 0xFFFFFFFFull) + 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_exchange(&S.claim, claim_word(0, claim_lchunk(src.st[0].kind, items, workers), items),
                              __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        bump_epoch(D);
        st_sys(&H->done[slot].t_open[0], dev_clock());
      }
      ++next;
    }
    if (hstop) {
      if (lane == 0) raise_stop(D, kSrvStopped);
      return;
    }
    __builtin_amdgcn_s_sleep(32);
  }
}

// ---------------------------------------------------------------------------- workers
union SrvLds {
  TileLds tile;
  CompactLds compact;
  UpsweepLds up;
  DownsweepLds down;
  OffsetsLds offsets;
  EmitLds emit;
  uint32_t words[kMaxProjBlocks + 3 * kSrvMaxViews];   // classify: 3 V words; projection: G + V
};

// Arguments read from LDS into wave-uniform registers.
template <class T>
__device__ __forceinline__ T uniform_copy(const T& x) {
  static_assert(sizeof(T) % 4 == 0, "argument structs are whole words");
  T r;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(&x);
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
  return r;
}

// Runs item b of a stage with the per-stage kernels' block bodies.  Returns false for a stage
// variant the server does not carry (projection must read packed SH coefficients).
__device__ bool srv_run(int32_t kind, const Stage& st, Blk b, SrvLds& U) {
  switch (kind) {
    case kStViewSetup: view_setup_body(uniform_copy(st.a.view_setup), b); return true;
    case kStFill: fill_body(uniform_copy(st.a.fill), b); return true;
    case kStFrustumMax: frustum_max_body(uniform_copy(st.a.frustum), b); return true;
    case kStFold: fold_body(uniform_copy(st.a.fold), b); return true;
    case kStClassify: {
      const ClassifyArgs a = uniform_copy(st.a.classify);
      if (a.write) classify_body<true>(a, b, U.words);
      else classify_body<false>(a, b, U.words);
      return true;
    }
    case kStProject: {
      const ProjectArgs a = uniform_copy(st.a.project);
      if (!a.packed || !a.write) return false;
      switch (a.sc.sh_degree) {
        case 0: project_body<0, true, true>(a, b, U.words); break;
        case 1: project_body<1, true, true>(a, b, U.words); break;
        case 2: project_body<2, true, true>(a, b, U.words); break;
        default: project_body<3, true, true>(a, b, U.words); break;
      }
      return true;
    }
    case kStSelectHist: select_hist_body(uniform_copy(st.a.select), b); return true;
    case kStSelectPick: select_pick_body(uniform_copy(st.a.select), b); return true;
    case kStScanReduce: scan_reduce_body(uniform_copy(st.a.scan_reduce), b); return true;
    case kStScanPartials: scan_partials_body(uniform_copy(st.a.scan_partials), b); return true;
    case kStCompact: compact_body(uniform_copy(st.a.compact), b, U.compact); return true;
    case kStRadixUp: radix_upsweep_body(uniform_copy(st.a.radix), b, U.up); return true;
    case kStRadixScan: radix_digit_scan_body(uniform_copy(st.a.radix), b); return true;
    case kStRadixDown: radix_downsweep_body(uniform_copy(st.a.radix), b, U.down); return true;
    case kStEmitReduce: emit_reduce_body(uniform_copy(st.a.emit_reduce), b); return true;
    case kStEmitPartials: emit_partials_body(uniform_copy(st.a.emit_partials), b); return true;
    case kStEmitOffsets: emit_offsets_body(uniform_copy(st.a.emit_offsets), b, U.offsets); return true;
    case kStEmit: emit_body(uniform_copy(st.a.emit), b, U.emit); return true;
    case kStRanges: ranges_body(uniform_copy(st.a.ranges), b); return true;
    case kStTileCount: tile_count_body(uniform_copy(st.a.tile_order), b); return true;
    case kStTileScatter: tile_scatter_body(uniform_copy(st.a.tile_order), b); return true;
    case kStBlend: {
      // Items in claim order: the long tiles' blocks first, then the tiles.
      const BlendArgs a = uniform_copy(st.a.blend);
      if (a.count) blend_item<true>(a, b.id, U.tile);
      else blend_item<false>(a, b.id, U.tile);
      return true;
    }
    case kStReducePairs: reduce_pairs_body(uniform_copy(st.a.reduce_pairs), b); return true;
    case kStLongMask: long_mask_body(uniform_copy(st.a.long_mask), b); return true;
    default: return false;
  }
}

// Items of stage k of a job as it opens (after an acquire of the stages before it).  A
// blend claims only the items its tile order needs, not the bound its per-stage launch covers.
__device__ uint32_t open_items(const SrvJob& job, uint32_t k, int32_t kind) {
  if (kind == kStBlend) {
    const BlendArgs& a = job.st[k].a.blend;
    const uint32_t* tord =
        reinterpret_cast<const uint32_t*>(ld_agent(reinterpret_cast<const uint64_t*>(&a.tord)));
    const uint32_t nl = ld_agent(tord + kTileLongWord), lmax = ld_agent(&a.long_max);
    return long_grid(nl < lmax ? nl : lmax) + xcd_grid(ld_agent(&a.tiles_total));
  }
  return ld_agent(&job.st[k].items);
}

// Thread 0 of a worker: n items of `stage` in `slot` are done (and released).  The worker
// that completes the stage opens the next one, or completes the job.
__device__ void srv_complete(SrvDev* D, SrvHost* H, uint32_t slot, uint32_t stage, uint32_t n, uint32_t limit,
                             uint32_t workers) {
  SrvSlot& S = D->slot[slot];
  const uint32_t prev = atomicAdd(&S.done, n);
  if (prev + n != limit) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const SrvJob& job = D->job[slot];
  const uint32_t ns = ld_agent(&job.n_stages);
  const uint32_t next = stage + 1;
  if (next < ns) {
    const int32_t kind = ld_agent(&job.st[next].kind);
    const uint32_t items = open_items(job, next, kind);
    atomicExch(&S.done, 0u);
    __hip_atomic_exchange(&S.claim, claim_word(next, claim_lchunk(kind, items, workers), items), __ATOMIC_RELEASE,
                          __HIP_MEMORY_SCOPE_AGENT);
    bump_epoch(D);
    st_sys(&H->done[slot].t_open[next], dev_clock());
    return;
  }
  // The job is complete.  The slot is freed before the record is written: the host reuses a
  // slot only after it has seen the record.
  const unsigned long long* hdr =
      reinterpret_cast<const unsigned long long*>(ld_agent(reinterpret_cast<const uint64_t*>(&job.hdr)));
  const uint64_t ovf = ld_agent(hdr + kHdrOverflow), nd = ld_agent(hdr + kHdrDup), seq = ld_agent(&job.seq);
  __hip_atomic_exchange(&S.claim, claim_word(kNoStage, 0, 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&S.active, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  SrvDone& r = H->done[slot];
  st_sys(&r.overflow, ovf);
  st_sys(&r.n_dup, nd);
  st_sys(&r.t_end, dev_clock());
  st_sys_release(&r.seq1, seq + 1);
}

__device__ void srv_work(SrvDev* D, SrvHost* H, uint64_t deadline, SrvLds& U) {
  __shared__ uint32_t c_go, c_fresh, c_slot, c_stage, c_i0, c_i1;
  __shared__ Stage c_st;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t workers = gridDim.x - 1;
  // Wave 0's view of the stage this worker is in (kNone: none) and its items not yet counted.
  uint32_t cur_slot = kNone, cur_stage = 0, cur_limit = 0, pending = 0;
  for (;;) {
    if (threadIdx.x < 64) {
      const uint32_t lane = lane_id();
      uint32_t go = 0, fresh = 0, idle = 0, slot = 0, stage = 0, i0 = 0, i1 = 0;
      unsigned long long seen = ~0ull;   // epoch of the last scan that found nothing
      for (;;) {
        if (cur_slot != kNone) {
          // More items of the current stage?
          unsigned long long old = 0;
          uint32_t add = 0;
          if (lane == 0) {
            const unsigned long long w = ld_agent(&D->slot[cur_slot].claim);
            if (cw_stage(w) == cur_stage && cw_cursor(w) < cw_limit(w)) {
              add = 1u << cw_lchunk(w);
              old = atomicAdd(&D->slot[cur_slot].claim, (unsigned long long)add);
            }
          }
          add = __shfl(add, 0, 64);
          old = __shfl(old, 0, 64);
          if (add != 0u && cw_stage(old) == cur_stage && cw_cursor(old) < cw_limit(old)) {
            slot = cur_slot;
            stage = cur_stage;
            i0 = cw_cursor(old);
            i1 = i0 + add < cw_limit(old) ? i0 + add : cw_limit(old);
            go = 1;
            break;
          }
          // None left to claim: release this worker's items of the stage and count them.
          if (pending) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) srv_complete(D, H, cur_slot, cur_stage, pending, cur_limit, workers);
            pending = 0;
          }
          cur_slot = kNone;
        }
        const unsigned long long e = ld_agent(&D->epoch);
        if (e & kStopBit) break;
        if (dev_clock() > deadline) {
          if (lane == 0) raise_stop(D, kSrvDeadline);
          break;
        }
        if (e == seen) {
          // Back off while idle: about 0.2 us, growing to about 3 us.
          idle = idle < 16 ? idle + 1 : 16;
          for (uint32_t k = 0; k < idle; ++k) __builtin_amdgcn_s_sleep(8);
          continue;
        }
        // Lane j inspects slot j; the oldest job with unclaimed items wins.  A free slot's
        // claim word has no items, so only slots with items read their job's number (a number
        // not yet visible ranks the slot last, it does not hide its items).
        unsigned long long w = 0;
        uint32_t act = 0;
        if (lane < (uint32_t)kSrvSlots) {
          w = ld_agent(&D->slot[lane].claim);
          if (cw_cursor(w) < cw_limit(w)) {
            act = ld_agent(&D->slot[lane].active);
            if (act == 0u) act = 0xFFFFFFFFu;
          }
        }
        unsigned long long key = act != 0u ? ((unsigned long long)act << 8) | lane : ~0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const unsigned long long other = __shfl_xor(key, o, 64);
          key = other < key ? other : key;
        }
        if (key == ~0ull) {
          seen = e;
          continue;
        }
        idle = 0;
        const uint32_t j = (uint32_t)(key & 0xFFu);
        unsigned long long old = 0;
        uint32_t add = 0;
        if (lane == j) {
          add = 1u << cw_lchunk(w);
          old = atomicAdd(&D->slot[j].claim, (unsigned long long)add);
        }
        old = __shfl(old, (int)j, 64);
        add = __shfl(add, (int)j, 64);
        if (cw_cursor(old) >= cw_limit(old)) continue;   // another worker took the last items first
        slot = j;
        stage = cw_stage(old);
        i0 = cw_cursor(old);
        i1 = i0 + add < cw_limit(old) ? i0 + add : cw_limit(old);
        cur_slot = slot;
        cur_stage = stage;
        cur_limit = cw_limit(old);
        go = 1;
        fresh = 1;
        break;
      }
      // Entering a stage: acquire before anything of it is read.
      if (fresh) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) {
        c_go = go;
        c_fresh = fresh;
        c_slot = slot;
        c_stage = stage;
        c_i0 = i0;
        c_i1 = i1;
      }
      if (go) pending += i1 - i0;
    }
    __syncthreads();
    if (!c_go) return;
    const uint32_t slot = __builtin_amdgcn_readfirstlane(c_slot), stage = __builtin_amdgcn_readfirstlane(c_stage);
    const uint32_t i0 = __builtin_amdgcn_readfirstlane(c_i0), i1 = __builtin_amdgcn_readfirstlane(c_i1);
    if (__builtin_amdgcn_readfirstlane(c_fresh)) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&D->job[slot].st[stage]);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&c_st);
      for (uint32_t q = threadIdx.x; q < (uint32_t)(sizeof(Stage) / 4); q += kBlock) dst[q] = ld_agent(src + q);
      __syncthreads();
    }
    const int32_t kind = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)c_st.kind);
    const uint32_t items = __builtin_amdgcn_readfirstlane(c_st.items);
    bool ok = true;
    for (uint32_t it = i0; it < i1 && ok; ++it) {
      ok = srv_run(kind, c_st, Blk{it, items}, U);
      __syncthreads();
    }
    if (!ok) {
      if (threadIdx.x == 0) raise_stop(D, kSrvUnsupported);
      return;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_server(SrvDev* D, SrvHost* H, uint64_t max_ticks) {
  __shared__ SrvLds U;
  const uint64_t deadline = dev_clock() + max_ticks;
  if (blockIdx.x == 0) {
    srv_dispatch(D, H, deadline);
    return;
  }
  srv_work(D, H, deadline, U);
}

// ---------------------------------------------------------------------------- host side
struct Server {
  hipStream_t stream = nullptr;
  SrvDev* dev = nullptr;
  SrvHost* host = nullptr;
  uint32_t workers = 0;
  uint64_t published = 0;
  double tick_hz = 0.0;
  bool launched = false;
};

static void server_free(Server* S) {
  if (S->host) (void)hipHostFree(S->host);
  if (S->dev) (void)hipFree(S->dev);
  delete S;
}

hipError_t server_start(int32_t workers, double max_seconds, hipStream_t s, Server** out, int32_t* used_workers) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (s) {
    e = hipStreamGetDevice(s, &dev);
    if (e != hipSuccess) return e;
  }
  int cus = 0, khz = 0, per_cu = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_server), kBlock, 0)) !=
      hipSuccess)
    return e;
  if (khz <= 0 || cus <= 0 || per_cu <= 0) return hipErrorInvalidValue;
  // Default: the resident capacity minus one workgroup per CU, so that small kernels of other
  // streams (copies, the caller's own work) still find room while the server runs.
  const int resident = cus * per_cu;
  int w = workers > 0 ? workers : resident - cus;
  if (w < 1) w = 1;
  if (w > resident - 1) w = resident - 1;
  if (w < 1) return hipErrorInvalidConfiguration;
  Server* S = new Server();
  S->stream = s;
  S->workers = (uint32_t)w;
  S->tick_hz = (double)khz * 1e3;
  e = hipMalloc(reinterpret_cast<void**>(&S->dev), sizeof(SrvDev));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&S->host), sizeof(SrvHost), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) {
    server_free(S);
    return e;
  }
  ::memset(S->host, 0, sizeof(SrvHost));
  e = hipMemsetAsync(S->dev, 0, sizeof(SrvDev), s);
  // Free slots: no stage open.
  SrvSlot init[kSrvSlots];
  ::memset(init, 0, sizeof(init));
  for (int j = 0; j < kSrvSlots; ++j) init[j].claim = claim_word(kNoStage, 0, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(S->dev->slot, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    server_free(S);
    return e;
  }
  double secs = max_seconds > 0.0 ? max_seconds : 60.0;
  if (secs > 3600.0) secs = 3600.0;
  const uint64_t ticks = (uint64_t)(secs * S->tick_hz);
  SrvHost* hdev = nullptr;
  e = hipHostGetDevicePointer(reinterpret_cast<void**>(&hdev), S->host, 0);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_server, dim3((unsigned)w + 1), dim3(kBlock), 0, s, S->dev, hdev, ticks);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    server_free(S);
    return e;
  }
  S->launched = true;
  *out = S;
  if (used_workers) *used_workers = w;
  return hipSuccess;
}

const clod_view* server_views_dev(Server* S, int64_t seq) {
  return S->dev->job[seq % kSrvSlots].views;
}

int64_t server_next_seq(Server* S) { return (int64_t)S->published; }

bool server_slot_free(Server* S) {
  const uint64_t q = S->published;
  if (q < (uint64_t)kSrvSlots) return true;
  const volatile SrvDone& r = S->host->done[q % kSrvSlots];
  return __atomic_load_n(&r.seq1, __ATOMIC_ACQUIRE) == q - kSrvSlots + 1;
}

hipError_t server_publish(Server* S, const Program& P, int32_t n_views, const clod_view* views_host,
                          const void* hdr_dev, int64_t* seq) {
  if (P.full || P.n < 1 || n_views < 1 || n_views > kSrvMaxViews) return hipErrorInvalidValue;
  const uint64_t q = S->published;
  SrvJob& J = S->host->ring[q % kSrvSlots];
  J.n_stages = (uint32_t)P.n;
  J.n_views = (uint32_t)n_views;
  J.seq = q;
  J.hdr = reinterpret_cast<const unsigned long long*>(hdr_dev);
  J.reserved = 0;
  ::memcpy(J.views, views_host, sizeof(clod_view) * (size_t)n_views);
  ::memcpy(J.st, P.st, sizeof(Stage) * (size_t)P.n);
  S->published = q + 1;
  __atomic_store_n(&S->host->published, q + 1, __ATOMIC_RELEASE);
  *seq = (int64_t)q;
  return hipSuccess;
}

// 1 and info = {overflow, D, completion time in ns since the server started} once job `seq`
// is complete, 0 while it is not, -1 if seq was never published or its slot was reused.
int server_poll(Server* S, int64_t seq, int64_t* info) {
  if (seq < 0 || (uint64_t)seq >= S->published) return -1;
  const SrvDone& r = S->host->done[seq % kSrvSlots];
  const uint64_t s1 = __atomic_load_n(&r.seq1, __ATOMIC_ACQUIRE);
  if (s1 < (uint64_t)seq + 1) return 0;
  if (s1 != (uint64_t)seq + 1) return -1;
  if (info) {
    info[0] = (int64_t)__atomic_load_n(&r.overflow, __ATOMIC_RELAXED);
    info[1] = (int64_t)__atomic_load_n(&r.n_dup, __ATOMIC_RELAXED);
    const uint64_t t0 = __atomic_load_n(&S->host->t_start, __ATOMIC_RELAXED);
    const uint64_t t1 = __atomic_load_n(&r.t_end, __ATOMIC_RELAXED);
    info[2] = (int64_t)((double)(t1 - t0) * 1e9 / S->tick_hz);
  }
  // A slot is only reused after its job was seen complete (server_slot_free), so the fields
  // read above belong to this job unless the slot's next job finished in between.
  return __atomic_load_n(&r.seq1, __ATOMIC_ACQUIRE) == (uint64_t)seq + 1 ? 1 : -1;
}

// Stage opening times of completed job seq in ns since the server started and the stage kinds
// (n_stages of them, at most max), followed by its completion time (kind 0); returns the count
// written, -1 as server_poll.  Valid until the slot takes its next job.
int server_stage_times(Server* S, int64_t seq, int64_t* ns, int32_t* kinds, int32_t max) {
  int64_t info[3];
  if (server_poll(S, seq, info) != 1) return -1;
  const SrvDone& r = S->host->done[seq % kSrvSlots];
  const SrvJob& J = S->host->ring[seq % kSrvSlots];
  const uint64_t t0 = __atomic_load_n(&S->host->t_start, __ATOMIC_RELAXED);
  const int n = (int)J.n_stages;
  int k = 0;
  for (; k < n && k < max; ++k) {
    ns[k] = (int64_t)((double)(__atomic_load_n(&r.t_open[k], __ATOMIC_RELAXED) - t0) * 1e9 / S->tick_hz);
    if (kinds) kinds[k] = J.st[k].kind;
  }
  if (k < max) {
    ns[k] = info[2];
    if (kinds) kinds[k] = 0;
    ++k;
  }
  return k;
}

// Device clock in ns since the server started (the dispatcher's last heartbeat), -1 before it runs.
int64_t server_clock_ns(Server* S) {
  if (!__atomic_load_n(&S->host->running, __ATOMIC_ACQUIRE)) return -1;
  const uint64_t t0 = __atomic_load_n(&S->host->t_start, __ATOMIC_RELAXED);
  const uint64_t t = __atomic_load_n(&S->host->heartbeat, __ATOMIC_RELAXED);
  return (int64_t)((double)(t - t0) * 1e9 / S->tick_hz);
}

hipError_t server_stop(Server* S, int32_t* status) {
  __atomic_store_n(&S->host->stop, 1u, __ATOMIC_RELEASE);
  hipError_t e = hipStreamSynchronize(S->stream);
  uint32_t st = 0;
  if (e == hipSuccess) e = hipMemcpy(&st, &S->dev->status, sizeof(st), hipMemcpyDeviceToHost);
  if (status) *status = (int32_t)st;
  server_free(S);
  return e;
}

}  // namespace clod
